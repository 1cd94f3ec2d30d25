// Host-side symbolic analysis of the condensed KKT pattern.
//
// The condensed matrix of LiftedKKT (K_tau = W + Sigma_x + J^T Sigma_s J,
// Sec. 3.2) and of HyKKT (K_gamma = K + gamma G^T G, Sec. 3.1) have the same
// pattern: pattern(W) U diag U pattern(J^T J) with J = [G; H].  Everything
// here depends on that pattern only and is computed once; the numeric
// phases reuse it for every new system, as the paper does with its solver's
// symbolic factorization (Sec. 6.1, analysis column of tab:linsol:time).
#pragma once
#include <cstdint>
#include <exception>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace ckkt {

struct PatternIn {
    int64_t n = 0, m_eq = 0, m_ineq = 0;
    std::vector<int32_t> w_ptr, w_idx, g_ptr, g_idx, h_ptr, h_idx;
};

// Symmetric adjacency (no diagonal), CSR.
struct Graph {
    int32_t n = 0;
    std::vector<int32_t> ptr, adj;
};

// Approximate minimum degree ordering. perm[k] = vertex eliminated k-th.
std::vector<int32_t> amd_order(const Graph& g);

struct Plan {
    // ---- sizes
    int32_t n = 0, m_eq = 0, m_ineq = 0, m = 0;
    int64_t nnz_w = 0, nnz_g = 0, nnz_h = 0;

    // ---- ordering: perm[new] = old, iperm[old] = new
    std::vector<int32_t> perm, iperm;

    // ---- K lower triangle in the new numbering, CSC: column j holds rows >= j
    std::vector<int32_t> kcolptr, krow;
    // assembly recipe per K slot
    std::vector<int32_t> k_wsrc;      // index into W values or -1
    std::vector<int32_t> k_diag;      // original index of the diagonal (sigma_x) or -1
    std::vector<int32_t> prod_ptr;    // nnz_k + 1
    std::vector<int32_t> prod_r, prod_a, prod_b;  // J row, two J value indices (G values then H values)
    std::vector<int32_t> dense_rows;  // rows of J kept out of K (AnalyzeOptions::dense_row_min)

    // ---- supernodes (new numbering, columns contiguous)
    int32_t ns = 0;
    std::vector<int32_t> sn_start;    // ns + 1
    std::vector<int32_t> sn_rowptr;   // ns + 1, offsets into sn_rows
    std::vector<int32_t> sn_rows;     // front row lists: own columns then the rows below
    std::vector<int32_t> sn_parent;   // -1 for roots
    std::vector<int32_t> child_ptr, child_list;
    std::vector<int32_t> relmap;      // aligned with sn_rows: row position inside the parent front
    std::vector<int32_t> kmap;        // per K slot: row position inside its supernode's front
    std::vector<int32_t> kcol;        // per K slot: its column (factor numbering)
    // Children contributions bucketed by destination position of the parent
    // front (aligned with sn_rows, children in child order): for front
    // position q of supernode s, entries [cb_ptr[sn_rowptr[s]+q], ...+1) list
    // child rows/columns landing on q.  cb_src indexes relmap/uvec (the
    // child's row), cb_len = rows of that child column from there down,
    // cb_uoff = arena offset of the child's update entry on its diagonal.
    std::vector<int32_t> cb_ptr, cb_src, cb_len;
    std::vector<int64_t> cb_uoff;
    std::vector<int64_t> l_off;       // start of the supernode's region in the factor arena
    std::vector<int64_t> u_off;       // start of its update (Schur) matrix in the arena
    std::vector<int32_t> u_ld;        // leading dimension of the update matrix
    std::vector<uint8_t> big;         // 1 if factored by the tiled path
    int64_t arena = 0;                // factor arena length (elements)
    int64_t nnz_l = 0, nnz_l_stored = 0;
    double flops = 0.0;
    int32_t max_front = 0, n_big = 0;

    // ---- level schedule (level 0 = leaves)
    int32_t nlev = 0;
    std::vector<int32_t> sn_level;        // level of each supernode (0 = leaf, parent > child)
    std::vector<int32_t> lvl_ptr;         // nlev + 1, into lvl_small / lvl_big
    std::vector<int32_t> lvl_small;       // small-front supernodes grouped by level
    std::vector<int32_t> lvl_small_ptr;   // nlev + 1
    std::vector<int32_t> lvl_big;         // big-front supernodes grouped by level
    std::vector<int32_t> lvl_big_ptr;     // nlev + 1
    std::vector<int32_t> lvl_all;         // all supernodes grouped by level (sweeps)
    std::vector<int32_t> lvl_all_ptr;
    std::vector<int32_t> lvl_maxw_big;    // per level, max supernode width among big fronts
    std::vector<int32_t> big_tiles_ptr;   // per level: prefix count of column tiles over big fronts
    std::vector<int32_t> big_tile_sn, big_tile_col;  // (supernode, first column of tile)

    // ---- unassembled operators for the residual (original numbering)
    std::vector<int32_t> wf_ptr, wf_col, wf_vidx;   // full symmetric W, value index into W lower
    std::vector<int32_t> j_ptr, j_col;              // J = [G; H] rows, value index = position
    std::vector<int32_t> jt_ptr, jt_row, jt_vidx, jt_gend;  // J^T by column; G rows first

    // ---- batched instances (block-diagonal union); one instance otherwise
    int32_t ninst = 1;
    std::vector<int32_t> inst_n;      // ninst + 1 prefix over variables
    std::vector<int32_t> inst_meq;    // ninst + 1 prefix over equality rows
    std::vector<int32_t> inst_of_var; // n
    std::vector<int32_t> inst_of_eqrow; // m_eq

    double analyze_seconds = 0.0;
    // not serialized: the part of analyze_seconds spent up to the ordering
    // (pattern keys and AMD), and in the symbolic factorization steps that
    // SymbolicDevice can take over (0 for a loaded plan)
    double order_seconds = 0.0, symbolic_seconds = 0.0;
};

// The symbolic factorization steps that can run on the device once the
// ordering is fixed (the paper's solver orders on the host and factors
// symbolically on the GPU, Sec. 1).  With AnalyzeOptions::device set,
// analyze() hands these steps to it; each must produce exactly what the host
// steps produce, element by element, so that both give the same plan.
class SymbolicDevice {
public:
    virtual ~SymbolicDevice() = default;
    // Elimination tree and its postorder (children in increasing order) of
    // the pattern `keys` (pairs (i << 32) | j, i > j, original numbering)
    // ordered by perm0 (ip0 its inverse): fills P.perm, P.iperm, P.kcolptr,
    // P.krow, the etree `parent` (new numbering, -1 at roots) and the column
    // counts of L with the diagonal.
    virtual std::string order(int32_t n, const std::vector<uint64_t>& keys, const std::vector<int32_t>& perm0,
                              const std::vector<int32_t>& ip0, Plan& P, std::vector<int32_t>& parent,
                              std::vector<int64_t>& cnt) = 0;
    // Fills P.sn_rows, P.relmap and P.kmap from P.sn_start, P.sn_rowptr and
    // P.sn_parent (and the arrays order() produced).
    virtual std::string fronts(Plan& P) = 0;
    // Fills P.prod_ptr, P.prod_r, P.prod_a, P.prod_b: the K slots of the
    // products J_ra J_rb (a <= b) of the rows not flagged in `dense`.
    virtual std::string products(Plan& P, const std::vector<char>& dense) = 0;
};

struct AnalyzeOptions {
    int ordering = 0;      // 0 AMD, 1 natural
    int relax = 1;
    int big_front = 96;    // fronts larger than this go to the tiled path
    int tile = 64;         // column tile of the tiled path
    int dense_row_min = 0; // rows of J with at least this many entries stay out of K (0: none)
    const std::vector<int32_t>* perm = nullptr;  // fill-reducing ordering given by the caller (AMD mode)
    int threads = 1;       // host threads (assembly recipe; per-block pair keys)
    // block-diagonal pattern (a batch): prefix offsets of the blocks' variables,
    // equality rows and inequality rows; their pair keys are built per block
    const std::vector<int32_t>* block_n = nullptr;
    const std::vector<int32_t>* block_meq = nullptr;
    const std::vector<int32_t>* block_mineq = nullptr;
    // symbolic factorization on the device (null: on the host)
    SymbolicDevice* device = nullptr;
};

// AMD ordering of one pattern's K = W + J^T J graph (rows of J with at least
// dense_row_min entries left out when dense_row_min > 0); identity for n <= 1.
std::vector<int32_t> order_pattern(const PatternIn& p, int dense_row_min);

// Runs share(t) for t = 0 .. nthreads-1: share 0 on the calling thread, the
// others on host threads.  A share whose thread cannot be started runs on
// the calling thread after share 0.  Every started thread is joined before
// this returns (also when a share throws), and the first exception thrown
// by any share is rethrown here, on the calling thread, so that nothing
// escapes a worker (which would terminate the process).
template <class F>
void run_threads(int nthreads, F&& share) {
    std::exception_ptr first;
    std::mutex mu;
    auto guarded = [&](int t) {
        try {
            share(t);
        } catch (...) {
            std::lock_guard<std::mutex> lk(mu);
            if (!first) first = std::current_exception();
        }
    };
    struct Joiner {
        std::vector<std::thread> pool;
        ~Joiner() {
            for (auto& th : pool)
                if (th.joinable()) th.join();
        }
    } j;
    std::vector<int> not_started;
    for (int t = 1; t < nthreads; ++t) {
        try {
            j.pool.emplace_back(guarded, t);
        } catch (...) {
            not_started.push_back(t);
        }
    }
    guarded(0);
    for (int t : not_started) guarded(t);
    for (auto& th : j.pool) th.join();
    if (first) std::rethrow_exception(first);
}

// Returns an empty string on success, else a description of the pattern error.
std::string validate(const PatternIn& p);
std::string analyze(const PatternIn& p, const AnalyzeOptions& o, Plan& plan);

}  // namespace ckkt
