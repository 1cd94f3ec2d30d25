// Symbolic factorization on the device.
//
// The paper's solver computes the fill-reducing ordering on the host and the
// symbolic factorization on the GPU (Sec. 1, hybrid execution mode off;
// Sec. 6.1, the analysis column of tab:linsol:time).  Given the host
// ordering, the steps below run in kernels and produce, element by element,
// the arrays the host analysis produces:
//
//  * elimination tree.  Every entry (i, j), i > j, of the ordered lower
//    pattern is a token of value i that starts at node j.  At each node a it
//    reaches, the token registers itself with p[a] = min(p[a], i) and moves
//    on to the old value while that is smaller than i.  Each registered value
//    is an entry of column a of L (two entries of one column give an entry of
//    the column of the smaller), so p only decreases towards the smallest
//    entry, the etree parent (Liu 1990); rounds repeat until no token moves,
//    and then p is that parent: the token of the entry that puts parent(x)
//    into column x cannot jump past x, and rests at x.
//  * postorder with children (and roots) in increasing order: the Euler tour
//    of the forest, ranked by pointer jumping (Wyllie), gives every node its
//    postorder number and subtree size.
//  * column counts (Gilbert, Ng and Peyton 1994): for each row i with sorted
//    entries k_1 < ... < k_m below the diagonal, +1 at every k_t, -1 at
//    lca(k_{t-1}, k_t) and -1 at i; the count of column j is one plus the sum
//    over its subtree, a contiguous range in postorder.  In a postordered
//    tree lca(a, b), a < b, is the first ancestor of a numbered at least b,
//    found by binary lifting.
//  * rows below each supernode: the path from k_t up to lca(k_{t-1}, k_t)
//    (up to i for t = 1) is disjoint from the other paths of row i; walked on
//    the supernodal tree each emits (supernode, i) pairs, which sorted and
//    made unique are the front row lists.
//  * the position of every child row in its parent front and of every K entry
//    in its front (binary search), and the K slot of every product
//    J_ra J_rb of the assembly (binary search in the K columns), grouped by
//    slot with a stable radix sort so that each slot keeps the row order.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "analysis.hpp"
#include "device.hpp"

namespace ckkt {
namespace {

constexpr int kThreads = 256;

inline unsigned grid_for(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + kThreads - 1) / kThreads); }

inline int bit_length(uint64_t v) {
    int b = 0;
    while (v) { ++b; v >>= 1; }
    return b;
}

template <class T>
struct DBuf {
    T* p = nullptr;
    size_t n = 0;
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    ~DBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    hipError_t alloc(size_t count) {
        release();
        n = count;
        return hipMalloc(reinterpret_cast<void**>(&p), std::max<size_t>(count, 1) * sizeof(T));
    }
};

// ------------------------------------------------------------------ kernels

__global__ void k_fill(int32_t* x, int64_t n, int32_t v) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) x[t] = v;
}

// Tokens of the ordered lower pattern: value (the larger index) and the node
// the token sits at (starts at the smaller index).
__global__ void k_tokens(const uint64_t* keys, int64_t m, const int32_t* ip, int32_t* tv, int32_t* ta) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    const uint64_t k = keys[t];
    const int32_t a = ip[(int32_t)(k >> 32)], b = ip[(int32_t)(uint32_t)k];
    tv[t] = max(a, b);
    ta[t] = min(a, b);
}

// Every token registers at its start node before the first climb, so that
// in a round where no token moves no value is registered anywhere.
__global__ void k_register(const int32_t* tv, const int32_t* ta, int64_t m, int32_t* p) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < m) atomicMin(&p[ta[t]], tv[t]);
}

// One round of the etree climb.  p holds n where nothing is registered.
__global__ void k_etree_climb(const int32_t* tv, int32_t* ta, int64_t m, int32_t* p, int32_t* moved) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool mv = false;
    if (t < m) {
        const int32_t i = tv[t];
        int32_t a = ta[t];
        for (;;) {
            const int32_t q = atomicMin(&p[a], i);  // registers i at a, returns the old minimum
            if (q >= i) break;
            a = q;  // an entry of column a smaller than i: i is in column q too
            mv = true;
        }
        if (mv) ta[t] = a;
    }
    if (__any(mv) && (threadIdx.x & 63) == 0) atomicOr(moved, 1);
}

// (parent, child) keys; roots get parent n so that they sort as children of
// a virtual root, in increasing order.
__global__ void k_child_keys(const int32_t* p, int32_t n, uint64_t* key) {
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t par = p[v] < n ? p[v] : n;
    key[v] = ((uint64_t)(uint32_t)par << 32) | (uint32_t)v;
}

__global__ void k_child_links(const uint64_t* key, int32_t n, int32_t* first_child, int32_t* next_sib) {
    const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const uint32_t par = (uint32_t)(key[k] >> 32);
    const int32_t v = (int32_t)(uint32_t)key[k];
    if (k == 0 || (uint32_t)(key[k - 1] >> 32) != par) first_child[par] = v;
    next_sib[v] = (k + 1 < n && (uint32_t)(key[k + 1] >> 32) == par) ? (int32_t)(uint32_t)key[k + 1] : -1;
}

// Euler tour: event 2v enters v, 2v + 1 leaves it; leaving events weigh 1.
__global__ void k_euler(const int32_t* p, int32_t n, const int32_t* first_child, const int32_t* next_sib,
                        int32_t* nxt, int32_t* rank) {
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t fc = first_child[v];
    nxt[2 * v] = fc >= 0 ? 2 * fc : 2 * v + 1;
    rank[2 * v] = 0;
    const int32_t ns = next_sib[v];
    nxt[2 * v + 1] = ns >= 0 ? 2 * ns : (p[v] < n ? 2 * p[v] + 1 : -1);
    rank[2 * v + 1] = 1;
}

__global__ void k_rank_step(const int32_t* nxt, const int32_t* rank, int32_t* nxt2, int32_t* rank2, int32_t ne) {
    const int32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    const int32_t q = nxt[e];
    if (q >= 0) {
        rank2[e] = rank[e] + rank[q];
        nxt2[e] = nxt[q];
    } else {
        rank2[e] = rank[e];
        nxt2[e] = -1;
    }
}

// rank[e] = leaving events from e to the end of the tour
__global__ void k_post_number(const int32_t* rank, int32_t n, int32_t* pos) {
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) pos[v] = n - rank[2 * v + 1];
}

__global__ void k_relabel(const int32_t* rank, const int32_t* pos, const int32_t* p, const int32_t* perm0, int32_t n,
                          int32_t* perm, int32_t* iperm, int32_t* parent, int32_t* first) {
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t k = pos[v];
    perm[k] = perm0[v];
    iperm[perm0[v]] = k;
    parent[k] = p[v] < n ? pos[p[v]] : -1;
    first[k] = k - (rank[2 * v] - rank[2 * v + 1]);  // subtree size - 1 below k
}

// Entries in the postordered numbering: column-major and row-major keys.
__global__ void k_new_keys(const uint64_t* keys, int64_t m, const int32_t* ip0, const int32_t* pos, uint64_t* colkey,
                           uint64_t* rowkey) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    const uint64_t k = keys[t];
    const int32_t a = pos[ip0[(int32_t)(k >> 32)]], b = pos[ip0[(int32_t)(uint32_t)k]];
    const uint32_t hi = (uint32_t)max(a, b), lo = (uint32_t)min(a, b);
    colkey[t] = ((uint64_t)lo << 32) | hi;
    rowkey[t] = ((uint64_t)hi << 32) | lo;
}

__global__ void k_count_major(const uint64_t* key, int64_t m, int32_t* count) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < m) atomicAdd(&count[(int32_t)(key[t] >> 32)], 1);
}

__global__ void k_plus_one(int32_t* x, int32_t n) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) x[j] += 1;
}

// K lower CSC: the diagonal first, then the sorted rows.  Entry t of the
// sorted column keys of column J lands at kcolptr[J] + 1 + (t - (kcolptr[J] - J)).
__global__ void k_krow(const uint64_t* colkey, int64_t m, const int32_t* kcolptr, int32_t n, int32_t* krow) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) krow[kcolptr[t]] = (int32_t)t;
    if (t < m) {
        const int64_t J = (int64_t)(colkey[t] >> 32);
        krow[t + J + 1] = (int32_t)(uint32_t)colkey[t];
    }
}

__global__ void k_lift(const int32_t* prev, int32_t* next, int32_t n) {
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t u = prev[v];
    next[v] = u < 0 ? -1 : prev[u];
}

// Nearest common ancestor of a < b in the postordered forest: the first
// ancestor of a numbered at least b (-1 if there is none).
__device__ int32_t lca_post(const int32_t* up, int32_t levels, int32_t n, int32_t a, int32_t b) {
    int32_t u = a;
    for (int32_t k = levels - 1; k >= 0; --k) {
        const int32_t v = up[(int64_t)k * n + u];
        if (v >= 0 && v < b) u = v;
    }
    return up[u];  // level 0: the parent
}

// Upper end (exclusive) of the path that entry t of its row adds to the row
// subtree: lca with the previous entry of the row, or the row itself.
__device__ int32_t path_stop(const uint64_t* rowkey, int64_t t, const int32_t* up, int32_t levels, int32_t n) {
    const int32_t i = (int32_t)(rowkey[t] >> 32), k = (int32_t)(uint32_t)rowkey[t];
    if (t > 0 && (int32_t)(rowkey[t - 1] >> 32) == i) return lca_post(up, levels, n, (int32_t)(uint32_t)rowkey[t - 1], k);
    return i;
}

__global__ void k_count_deltas(const uint64_t* rowkey, int64_t m, const int32_t* up, int32_t levels, int32_t n,
                               int32_t* w, int32_t* err) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    const int32_t k = (int32_t)(uint32_t)rowkey[t];
    const int32_t stop = path_stop(rowkey, t, up, levels, n);
    if (stop < 0 || stop >= n) {
        *err = 1;
        return;
    }
    atomicAdd(&w[k], 1);
    atomicAdd(&w[stop], -1);
}

__global__ void k_widen(const int32_t* w, int64_t* s, int32_t n) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) s[j] = w[j];
}

__global__ void k_colcounts(const int64_t* S, const int32_t* first, int32_t n, int64_t* cnt) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int32_t f = first[j];
    cnt[j] = 1 + S[j] - (f > 0 ? S[f - 1] : 0);
}

// ---- fronts

__global__ void k_col2sn(const int32_t* sn_start, int32_t ns, int32_t n, int32_t* col2sn) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int32_t b = 0, e = ns;  // last s with sn_start[s] <= j
    while (e - b > 1) {
        const int32_t mid = b + (e - b) / 2;
        if (sn_start[mid] <= j) b = mid;
        else e = mid;
    }
    col2sn[j] = b;
}

// Supernodes crossed by the path of entry t (emit = false: count them).
__global__ void k_front_pairs(const uint64_t* rowkey, int64_t m, const int32_t* up, int32_t levels, int32_t n,
                              const int32_t* col2sn, const int32_t* sn_start, const int32_t* sn_parent,
                              const int64_t* off, int64_t* count, uint64_t* pairs, int32_t* err) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    const int32_t i = (int32_t)(rowkey[t] >> 32), k = (int32_t)(uint32_t)rowkey[t];
    const int32_t stop = path_stop(rowkey, t, up, levels, n);
    if (stop < 0 || stop >= n) {
        *err = 2;
        return;
    }
    int32_t s = col2sn[k];
    const int32_t s_stop = col2sn[stop];
    int64_t c = 0;
    for (;;) {
        if (i >= sn_start[s + 1]) {
            if (pairs) pairs[off[t] + c] = ((uint64_t)(uint32_t)s << 32) | (uint32_t)i;
            ++c;
        }
        if (s == s_stop) break;
        s = sn_parent[s];
        if (s < 0 || s > s_stop) {
            *err = 2;
            break;
        }
    }
    if (!pairs) count[t] = c;
}

__global__ void k_front_rows(const uint64_t* uniq, int64_t nu, const int32_t* sn_start, const int32_t* sn_rowptr,
                             int32_t* sn_rows, int32_t* err) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= nu) return;
    const int32_t s = (int32_t)(uniq[u] >> 32);
    const int64_t lo = (int64_t)sn_rowptr[s] - sn_start[s], hi = (int64_t)sn_rowptr[s + 1] - sn_start[s + 1];
    if (u < lo || u >= hi) {  // a supernode with more or fewer rows than its column count says
        *err = 3;
        return;
    }
    sn_rows[u + sn_start[s + 1]] = (int32_t)(uint32_t)uniq[u];
}

__global__ void k_front_own(const int32_t* col2sn, const int32_t* sn_start, const int32_t* sn_rowptr, int32_t n,
                            int32_t* sn_rows) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int32_t s = col2sn[j];
    sn_rows[sn_rowptr[s] + j - sn_start[s]] = j;
}

// Position of row i inside the front of supernode s, or -1.
__device__ int32_t front_pos(const int32_t* sn_rows, const int32_t* sn_start, const int32_t* sn_rowptr, int32_t s,
                             int32_t i) {
    const int32_t c0 = sn_start[s], c1 = sn_start[s + 1];
    if (i >= c0 && i < c1) return i - c0;
    const int32_t lo = sn_rowptr[s] + (c1 - c0), hi = sn_rowptr[s + 1];
    int32_t b = lo, e = hi;
    while (b < e) {
        const int32_t mid = b + (e - b) / 2;
        if (sn_rows[mid] < i) b = mid + 1;
        else e = mid;
    }
    if (b == hi || sn_rows[b] != i) return -1;
    return (c1 - c0) + (b - lo);
}

__global__ void k_relmap(const uint64_t* uniq, int64_t nu, const int32_t* sn_rows, const int32_t* sn_start,
                         const int32_t* sn_rowptr, const int32_t* sn_parent, int32_t* relmap, int32_t* err) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= nu) return;
    const int32_t s = (int32_t)(uniq[u] >> 32), i = (int32_t)(uint32_t)uniq[u];
    const int32_t ps = sn_parent[s];
    if (ps < 0) return;
    const int32_t q = front_pos(sn_rows, sn_start, sn_rowptr, ps, i);
    if (q < 0) *err = 4;
    relmap[u + sn_start[s + 1]] = q;
}

__global__ void k_kmap(const uint64_t* colkey, int64_t m, const int32_t* kcolptr, int32_t n, const int32_t* col2sn,
                       const int32_t* sn_rows, const int32_t* sn_start, const int32_t* sn_rowptr, int32_t* kmap,
                       int32_t* err) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) kmap[kcolptr[t]] = (int32_t)t - sn_start[col2sn[t]];
    if (t < m) {
        const int32_t J = (int32_t)(colkey[t] >> 32), I = (int32_t)(uint32_t)colkey[t];
        const int32_t q = front_pos(sn_rows, sn_start, sn_rowptr, col2sn[J], I);
        if (q < 0) *err = 5;
        kmap[t + J + 1] = q;
    }
}

// ---- products of the assembly

// Row r and the pair (a <= b) of entry offsets of product x (products of a
// row numbered a-major).
__device__ void product_of(const int64_t* poff, int32_t m, const int32_t* j_ptr, int64_t x, int32_t& r, int32_t& a,
                           int32_t& b) {
    int32_t lo = 0, hi = m;  // last r with poff[r] <= x
    while (hi - lo > 1) {
        const int32_t mid = lo + (hi - lo) / 2;
        if (poff[mid] <= x) lo = mid;
        else hi = mid;
    }
    r = lo;
    const int64_t q = j_ptr[r + 1] - j_ptr[r];
    const int64_t loc = x - poff[r];
    // before block a: a*q - a(a-1)/2 products
    auto before = [q](int64_t aa) { return aa * q - aa * (aa - 1) / 2; };
    const double qq = 2.0 * (double)q + 1.0;
    int64_t aa = (int64_t)std::floor((qq - std::sqrt(std::max(0.0, qq * qq - 8.0 * (double)loc))) * 0.5);
    aa = std::max<int64_t>(0, std::min<int64_t>(aa, q - 1));
    while (aa > 0 && before(aa) > loc) --aa;
    while (aa + 1 < q && before(aa + 1) <= loc) ++aa;
    a = (int32_t)aa;
    b = (int32_t)(aa + (loc - before(aa)));
}

__global__ void k_product_slots(const int64_t* poff, int32_t m, const int32_t* j_ptr, const int32_t* j_col,
                                const int32_t* iperm, const int32_t* kcolptr, const int32_t* krow, int64_t np,
                                int32_t* pslot, int32_t* pidx, int32_t* err) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= np) return;
    int32_t r, a, b;
    product_of(poff, m, j_ptr, x, r, a, b);
    const int32_t I = iperm[j_col[j_ptr[r] + a]], J = iperm[j_col[j_ptr[r] + b]];
    const int32_t hi = max(I, J), lo = min(I, J);
    int32_t bb = kcolptr[lo], e = kcolptr[lo + 1];
    const int32_t end = e;
    while (bb < e) {
        const int32_t mid = bb + (e - bb) / 2;
        if (krow[mid] < hi) bb = mid + 1;
        else e = mid;
    }
    if (bb == end || krow[bb] != hi) {
        *err = 6;
        bb = 0;
    }
    pslot[x] = bb;
    pidx[x] = (int32_t)x;
}

__global__ void k_slot_ptr(const int32_t* sorted_slot, int64_t np, int32_t nnzk, int32_t* prod_ptr) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s > nnzk) return;
    int64_t b = 0, e = np;  // first position with slot >= s
    while (b < e) {
        const int64_t mid = b + (e - b) / 2;
        if (sorted_slot[mid] < s) b = mid + 1;
        else e = mid;
    }
    prod_ptr[s] = (int32_t)b;
}

__global__ void k_product_rows(const int32_t* sorted_idx, int64_t np, const int64_t* poff, int32_t m,
                               const int32_t* j_ptr, int32_t* prod_r, int32_t* prod_a, int32_t* prod_b) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= np) return;
    int32_t r, a, b;
    product_of(poff, m, j_ptr, sorted_idx[x], r, a, b);
    prod_r[x] = r;
    prod_a[x] = j_ptr[r] + a;
    prod_b[x] = j_ptr[r] + b;
}

// ------------------------------------------------------------- the driver

#define SYM_TRY(call)                                                                   \
    do {                                                                                \
        const hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess) return std::string("device: ") + hipGetErrorString(e_);   \
    } while (0)

class DeviceSymbolic final : public SymbolicDevice {
public:
    explicit DeviceSymbolic(hipStream_t st) : st_(st) {}

    std::string order(int32_t n, const std::vector<uint64_t>& keys, const std::vector<int32_t>& perm0,
                      const std::vector<int32_t>& ip0, Plan& P, std::vector<int32_t>& parent,
                      std::vector<int64_t>& cnt) override {
        n_ = n;
        m_ = (int64_t)keys.size();
        if (m_ + n_ >= ((int64_t)1 << 31)) return "device: K too large for 32-bit slots";
        SYM_TRY(err_.alloc(1));
        SYM_TRY(hipMemsetAsync(err_.p, 0, sizeof(int32_t), st_));
        DBuf<int32_t> perm0_d;
        SYM_TRY(keys_.alloc(m_));
        SYM_TRY(ip0_.alloc(n));
        SYM_TRY(perm0_d.alloc(n));
        SYM_TRY(hipMemcpyAsync(keys_.p, keys.data(), m_ * sizeof(uint64_t), hipMemcpyHostToDevice, st_));
        SYM_TRY(hipMemcpyAsync(ip0_.p, ip0.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, st_));
        SYM_TRY(hipMemcpyAsync(perm0_d.p, perm0.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, st_));

        // ---- etree of the ordered pattern
        DBuf<int32_t> p, moved;
        SYM_TRY(p.alloc(n));
        SYM_TRY(moved.alloc(1));
        {
            DBuf<int32_t> tv, ta;
            SYM_TRY(tv.alloc(m_));
            SYM_TRY(ta.alloc(m_));
            k_fill<<<grid_for(n), kThreads, 0, st_>>>(p.p, n, n);
            if (m_ > 0) {
                k_tokens<<<grid_for(m_), kThreads, 0, st_>>>(keys_.p, m_, ip0_.p, tv.p, ta.p);
                k_register<<<grid_for(m_), kThreads, 0, st_>>>(tv.p, ta.p, m_, p.p);
            }
            SYM_TRY(hipGetLastError());
            rounds_ = 0;
            for (int32_t flag = m_ > 0 ? 1 : 0; flag;) {
                SYM_TRY(hipMemsetAsync(moved.p, 0, sizeof(int32_t), st_));
                k_etree_climb<<<grid_for(m_), kThreads, 0, st_>>>(tv.p, ta.p, m_, p.p, moved.p);
                SYM_TRY(hipGetLastError());
                SYM_TRY(hipMemcpyAsync(&flag, moved.p, sizeof(int32_t), hipMemcpyDeviceToHost, st_));
                SYM_TRY(hipStreamSynchronize(st_));
                if (++rounds_ > n + 1) return "internal: etree climb did not settle";
            }
        }

        // ---- postorder: Euler tour of the forest, ranked by pointer jumping
        DBuf<int32_t> pos, rank;
        SYM_TRY(pos.alloc(n));
        SYM_TRY(rank.alloc(2 * (size_t)n));
        {
            DBuf<uint64_t> ck, ck_sorted;
            DBuf<int32_t> first_child, next_sib, nxt, nxt2, rank2;
            SYM_TRY(ck.alloc(n));
            SYM_TRY(ck_sorted.alloc(n));
            SYM_TRY(first_child.alloc((size_t)n + 1));
            SYM_TRY(next_sib.alloc(n));
            SYM_TRY(nxt.alloc(2 * (size_t)n));
            SYM_TRY(nxt2.alloc(2 * (size_t)n));
            SYM_TRY(rank2.alloc(2 * (size_t)n));
            k_child_keys<<<grid_for(n), kThreads, 0, st_>>>(p.p, n, ck.p);
            SYM_TRY(hipGetLastError());
            std::string e = sort_keys(ck.p, ck_sorted.p, n, 32 + bit_length((uint64_t)n));
            if (!e.empty()) return e;
            k_fill<<<grid_for((int64_t)n + 1), kThreads, 0, st_>>>(first_child.p, (int64_t)n + 1, -1);
            k_child_links<<<grid_for(n), kThreads, 0, st_>>>(ck_sorted.p, n, first_child.p, next_sib.p);
            k_euler<<<grid_for(n), kThreads, 0, st_>>>(p.p, n, first_child.p, next_sib.p, nxt.p, rank.p);
            SYM_TRY(hipGetLastError());
            const int32_t ne = 2 * n;
            int32_t *r0 = rank.p, *r1 = rank2.p, *x0 = nxt.p, *x1 = nxt2.p;
            for (int step = 0; ((int64_t)1 << step) < (int64_t)ne + 1; ++step) {
                k_rank_step<<<grid_for(ne), kThreads, 0, st_>>>(x0, r0, x1, r1, ne);
                std::swap(r0, r1);
                std::swap(x0, x1);
            }
            SYM_TRY(hipGetLastError());
            if (r0 != rank.p) SYM_TRY(hipMemcpyAsync(rank.p, r0, (size_t)ne * sizeof(int32_t), hipMemcpyDeviceToDevice, st_));
            k_post_number<<<grid_for(n), kThreads, 0, st_>>>(rank.p, n, pos.p);
            SYM_TRY(hipGetLastError());
        }
        DBuf<int32_t> perm_d;
        SYM_TRY(perm_d.alloc(n));
        SYM_TRY(iperm_.alloc(n));
        SYM_TRY(parent_.alloc(n));
        SYM_TRY(first_.alloc(n));
        k_relabel<<<grid_for(n), kThreads, 0, st_>>>(rank.p, pos.p, p.p, perm0_d.p, n, perm_d.p, iperm_.p,
                                                     parent_.p, first_.p);
        SYM_TRY(hipGetLastError());

        // ---- K in the postordered numbering: lower CSC and lower rows
        SYM_TRY(colkey_.alloc(m_));
        SYM_TRY(rowkey_.alloc(m_));
        SYM_TRY(kcolptr_.alloc((size_t)n + 1));
        {
            DBuf<uint64_t> tmpk;
            SYM_TRY(tmpk.alloc(m_));
            const int bits = 32 + bit_length((uint64_t)n);
            if (m_ > 0) {
                // column keys into tmpk, row keys into colkey_ for the moment
                k_new_keys<<<grid_for(m_), kThreads, 0, st_>>>(keys_.p, m_, ip0_.p, pos.p, tmpk.p, colkey_.p);
                SYM_TRY(hipGetLastError());
                std::string e = sort_keys(colkey_.p, rowkey_.p, m_, bits);  // rows sorted
                if (!e.empty()) return e;
                e = sort_keys(tmpk.p, colkey_.p, m_, bits);  // columns sorted
                if (!e.empty()) return e;
            }
            DBuf<int32_t> colsize;
            SYM_TRY(colsize.alloc((size_t)n + 1));
            SYM_TRY(hipMemsetAsync(colsize.p, 0, ((size_t)n + 1) * sizeof(int32_t), st_));
            if (m_ > 0) k_count_major<<<grid_for(m_), kThreads, 0, st_>>>(colkey_.p, m_, colsize.p);
            k_plus_one<<<grid_for(n), kThreads, 0, st_>>>(colsize.p, n);
            SYM_TRY(hipGetLastError());
            std::string e = exclusive_sum(colsize.p, kcolptr_.p, n + 1);
            if (!e.empty()) return e;
            SYM_TRY(krow_.alloc((size_t)(m_ + n)));
            k_krow<<<grid_for(std::max<int64_t>(m_, n)), kThreads, 0, st_>>>(colkey_.p, m_, kcolptr_.p, n, krow_.p);
            SYM_TRY(hipGetLastError());
        }

        // ---- column counts
        levels_ = std::max(1, bit_length((uint64_t)n));
        SYM_TRY(up_.alloc((size_t)levels_ * n));
        SYM_TRY(hipMemcpyAsync(up_.p, parent_.p, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, st_));
        for (int k = 1; k < levels_; ++k)
            k_lift<<<grid_for(n), kThreads, 0, st_>>>(up_.p + (size_t)(k - 1) * n, up_.p + (size_t)k * n, n);
        SYM_TRY(hipGetLastError());
        DBuf<int64_t> cnt_d;
        SYM_TRY(cnt_d.alloc(n));
        {
            DBuf<int32_t> w;
            DBuf<int64_t> S, S2;
            SYM_TRY(w.alloc(n));
            SYM_TRY(S.alloc(n));
            SYM_TRY(S2.alloc(n));
            SYM_TRY(hipMemsetAsync(w.p, 0, (size_t)n * sizeof(int32_t), st_));
            if (m_ > 0)
                k_count_deltas<<<grid_for(m_), kThreads, 0, st_>>>(rowkey_.p, m_, up_.p, levels_, n, w.p, err_.p);
            k_widen<<<grid_for(n), kThreads, 0, st_>>>(w.p, S.p, n);
            SYM_TRY(hipGetLastError());
            std::string e = inclusive_sum(S.p, S2.p, n);
            if (!e.empty()) return e;
            k_colcounts<<<grid_for(n), kThreads, 0, st_>>>(S2.p, first_.p, n, cnt_d.p);
            SYM_TRY(hipGetLastError());
        }

        // ---- results to the host
        P.perm.resize(n);
        P.iperm.resize(n);
        parent.resize(n);
        cnt.resize(n);
        P.kcolptr.resize((size_t)n + 1);
        P.krow.resize((size_t)(m_ + n));
        SYM_TRY(hipMemcpyAsync(P.perm.data(), perm_d.p, (size_t)n * 4, hipMemcpyDeviceToHost, st_));
        SYM_TRY(hipMemcpyAsync(P.iperm.data(), iperm_.p, (size_t)n * 4, hipMemcpyDeviceToHost, st_));
        SYM_TRY(hipMemcpyAsync(parent.data(), parent_.p, (size_t)n * 4, hipMemcpyDeviceToHost, st_));
        SYM_TRY(hipMemcpyAsync(cnt.data(), cnt_d.p, (size_t)n * 8, hipMemcpyDeviceToHost, st_));
        SYM_TRY(hipMemcpyAsync(P.kcolptr.data(), kcolptr_.p, ((size_t)n + 1) * 4, hipMemcpyDeviceToHost, st_));
        SYM_TRY(hipMemcpyAsync(P.krow.data(), krow_.p, (size_t)(m_ + n) * 4, hipMemcpyDeviceToHost, st_));
        std::string e = check_err();
        if (!e.empty()) return e;
        // the relabelling must be a permutation whose etree is postordered
        std::vector<char> seen(n, 0);
        for (int32_t k = 0; k < n; ++k) {
            const int32_t v = P.perm[k];
            if (v < 0 || v >= n || seen[v] || P.iperm[v] != k) return "internal: postorder incomplete";
            seen[v] = 1;
        }
        for (int32_t j = 0; j < n; ++j)
            if (parent[j] != -1 && parent[j] <= j) return "internal: etree not postordered";
        return "";
    }

    std::string fronts(Plan& P) override {
        const int32_t n = n_, ns = P.ns;
        const int64_t nrows = P.sn_rowptr[ns];
        DBuf<int32_t> sn_start, sn_parent, sn_rowptr, rows, relmap, kmap;
        SYM_TRY(sn_start.alloc((size_t)ns + 1));
        SYM_TRY(sn_parent.alloc(ns));
        SYM_TRY(sn_rowptr.alloc((size_t)ns + 1));
        SYM_TRY(col2sn_.alloc(n));
        SYM_TRY(hipMemcpyAsync(sn_start.p, P.sn_start.data(), ((size_t)ns + 1) * 4, hipMemcpyHostToDevice, st_));
        SYM_TRY(hipMemcpyAsync(sn_parent.p, P.sn_parent.data(), (size_t)ns * 4, hipMemcpyHostToDevice, st_));
        SYM_TRY(hipMemcpyAsync(sn_rowptr.p, P.sn_rowptr.data(), ((size_t)ns + 1) * 4, hipMemcpyHostToDevice, st_));
        k_col2sn<<<grid_for(n), kThreads, 0, st_>>>(sn_start.p, ns, n, col2sn_.p);
        SYM_TRY(hipGetLastError());
        const int64_t below = nrows - n;  // rows below the supernodes, all fronts
        SYM_TRY(rows.alloc(nrows));
        DBuf<uint64_t> uniq;
        int64_t nu = 0;
        if (m_ > 0) {
            DBuf<int64_t> count, off;
            SYM_TRY(count.alloc(m_));
            SYM_TRY(off.alloc(m_ + 1));
            k_front_pairs<<<grid_for(m_), kThreads, 0, st_>>>(rowkey_.p, m_, up_.p, levels_, n, col2sn_.p, sn_start.p,
                                                            sn_parent.p, nullptr, count.p, nullptr, err_.p);
            SYM_TRY(hipGetLastError());
            std::string e = exclusive_sum(count.p, off.p, m_);
            if (!e.empty()) return e;
            int64_t last_off = 0, last_cnt = 0;
            SYM_TRY(hipMemcpyAsync(&last_off, off.p + (m_ - 1), 8, hipMemcpyDeviceToHost, st_));
            SYM_TRY(hipMemcpyAsync(&last_cnt, count.p + (m_ - 1), 8, hipMemcpyDeviceToHost, st_));
            SYM_TRY(hipStreamSynchronize(st_));
            e = check_err();
            if (!e.empty()) return e;
            const int64_t npairs = last_off + last_cnt;
            if (npairs >= ((int64_t)1 << 31)) return "device: too many front rows";
            DBuf<uint64_t> pairs, sorted;
            DBuf<int64_t> nsel;
            SYM_TRY(pairs.alloc(npairs));
            SYM_TRY(sorted.alloc(npairs));
            SYM_TRY(nsel.alloc(1));
            k_front_pairs<<<grid_for(m_), kThreads, 0, st_>>>(rowkey_.p, m_, up_.p, levels_, n, col2sn_.p, sn_start.p,
                                                            sn_parent.p, off.p, nullptr, pairs.p, err_.p);
            SYM_TRY(hipGetLastError());
            if (npairs > 0) {
                e = sort_keys(pairs.p, sorted.p, npairs, 64);
                if (!e.empty()) return e;
                SYM_TRY(uniq.alloc(npairs));
                size_t bytes = 0;
                SYM_TRY(hipcub::DeviceSelect::Unique(nullptr, bytes, sorted.p, uniq.p, nsel.p, (int)npairs, st_));
                SYM_TRY(grow_tmp(bytes));
                SYM_TRY(hipcub::DeviceSelect::Unique(tmp_.p, bytes, sorted.p, uniq.p, nsel.p, (int)npairs, st_));
                SYM_TRY(hipMemcpyAsync(&nu, nsel.p, 8, hipMemcpyDeviceToHost, st_));
                SYM_TRY(hipStreamSynchronize(st_));
            }
        }
        if (nu != below) return "internal: supernode structure mismatch";
        if (nu > 0)
            k_front_rows<<<grid_for(nu), kThreads, 0, st_>>>(uniq.p, nu, sn_start.p, sn_rowptr.p, rows.p, err_.p);
        k_front_own<<<grid_for(n), kThreads, 0, st_>>>(col2sn_.p, sn_start.p, sn_rowptr.p, n, rows.p);
        SYM_TRY(relmap.alloc(nrows));
        k_fill<<<grid_for(nrows), kThreads, 0, st_>>>(relmap.p, nrows, -1);
        if (nu > 0)
            k_relmap<<<grid_for(nu), kThreads, 0, st_>>>(uniq.p, nu, rows.p, sn_start.p, sn_rowptr.p, sn_parent.p,
                                                         relmap.p, err_.p);
        SYM_TRY(kmap.alloc((size_t)(m_ + n)));
        k_kmap<<<grid_for(std::max<int64_t>(m_, n)), kThreads, 0, st_>>>(colkey_.p, m_, kcolptr_.p, n, col2sn_.p, rows.p,
                                                                         sn_start.p, sn_rowptr.p, kmap.p, err_.p);
        SYM_TRY(hipGetLastError());
        P.sn_rows.resize(nrows);
        P.relmap.resize(nrows);
        P.kmap.resize((size_t)(m_ + n));
        SYM_TRY(hipMemcpyAsync(P.sn_rows.data(), rows.p, (size_t)nrows * 4, hipMemcpyDeviceToHost, st_));
        SYM_TRY(hipMemcpyAsync(P.relmap.data(), relmap.p, (size_t)nrows * 4, hipMemcpyDeviceToHost, st_));
        SYM_TRY(hipMemcpyAsync(P.kmap.data(), kmap.p, (size_t)(m_ + n) * 4, hipMemcpyDeviceToHost, st_));
        std::string e = check_err();
        if (e == "internal: device step 4") return "internal: child row missing from parent front";
        if (e == "internal: device step 5") return "internal: K entry outside its front";
        if (e == "internal: device step 3") return "internal: supernode structure mismatch";
        return e;
    }

    std::string products(Plan& P, const std::vector<char>& dense) override {
        const int32_t m = P.m;
        const int64_t nnzk = m_ + n_;
        std::vector<int64_t> poff((size_t)m + 1, 0);
        for (int32_t r = 0; r < m; ++r) {
            const int64_t q = dense[r] ? 0 : P.j_ptr[r + 1] - P.j_ptr[r];
            poff[r + 1] = poff[r] + q * (q + 1) / 2;
        }
        const int64_t np = poff[m];
        if (np >= ((int64_t)1 << 31)) return "device: too many J products for 32-bit offsets";
        P.prod_ptr.assign((size_t)nnzk + 1, 0);
        P.prod_r.resize(np);
        P.prod_a.resize(np);
        P.prod_b.resize(np);
        if (np == 0) return "";
        DBuf<int64_t> poff_d;
        DBuf<int32_t> j_ptr, j_col, pslot, pidx, sslot, sidx, prod_ptr, pr, pa, pb;
        SYM_TRY(poff_d.alloc((size_t)m + 1));
        SYM_TRY(j_ptr.alloc((size_t)m + 1));
        SYM_TRY(j_col.alloc(P.j_col.size()));
        SYM_TRY(hipMemcpyAsync(poff_d.p, poff.data(), ((size_t)m + 1) * 8, hipMemcpyHostToDevice, st_));
        SYM_TRY(hipMemcpyAsync(j_ptr.p, P.j_ptr.data(), ((size_t)m + 1) * 4, hipMemcpyHostToDevice, st_));
        SYM_TRY(hipMemcpyAsync(j_col.p, P.j_col.data(), P.j_col.size() * 4, hipMemcpyHostToDevice, st_));
        SYM_TRY(pslot.alloc(np));
        SYM_TRY(pidx.alloc(np));
        SYM_TRY(sslot.alloc(np));
        SYM_TRY(sidx.alloc(np));
        k_product_slots<<<grid_for(np), kThreads, 0, st_>>>(poff_d.p, m, j_ptr.p, j_col.p, iperm_.p, kcolptr_.p,
                                                           krow_.p, np, pslot.p, pidx.p, err_.p);
        SYM_TRY(hipGetLastError());
        size_t bytes = 0;
        const int bits = std::max(1, bit_length((uint64_t)nnzk));
        SYM_TRY(hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, pslot.p, sslot.p, pidx.p, sidx.p, (int)np, 0, bits,
                                                   st_));
        SYM_TRY(grow_tmp(bytes));
        SYM_TRY(hipcub::DeviceRadixSort::SortPairs(tmp_.p, bytes, pslot.p, sslot.p, pidx.p, sidx.p, (int)np, 0, bits,
                                                   st_));
        SYM_TRY(prod_ptr.alloc((size_t)nnzk + 1));
        SYM_TRY(pr.alloc(np));
        SYM_TRY(pa.alloc(np));
        SYM_TRY(pb.alloc(np));
        k_slot_ptr<<<grid_for(nnzk + 1), kThreads, 0, st_>>>(sslot.p, np, (int32_t)nnzk, prod_ptr.p);
        k_product_rows<<<grid_for(np), kThreads, 0, st_>>>(sidx.p, np, poff_d.p, m, j_ptr.p, pr.p, pa.p, pb.p);
        SYM_TRY(hipGetLastError());
        SYM_TRY(hipMemcpyAsync(P.prod_ptr.data(), prod_ptr.p, ((size_t)nnzk + 1) * 4, hipMemcpyDeviceToHost, st_));
        SYM_TRY(hipMemcpyAsync(P.prod_r.data(), pr.p, (size_t)np * 4, hipMemcpyDeviceToHost, st_));
        SYM_TRY(hipMemcpyAsync(P.prod_a.data(), pa.p, (size_t)np * 4, hipMemcpyDeviceToHost, st_));
        SYM_TRY(hipMemcpyAsync(P.prod_b.data(), pb.p, (size_t)np * 4, hipMemcpyDeviceToHost, st_));
        std::string e = check_err();
        if (e == "internal: device step 6") return "internal: J product missing from K";
        return e;
    }

private:
    hipError_t grow_tmp(size_t bytes) {
        if (tmp_.n >= bytes && tmp_.p) return hipSuccess;
        return tmp_.alloc(bytes);
    }

    std::string sort_keys(uint64_t* in, uint64_t* out, int64_t count, int end_bit) {
        if (count <= 0) return "";
        if (count >= ((int64_t)1 << 31)) return "device: sort too large";
        size_t bytes = 0;
        SYM_TRY(hipcub::DeviceRadixSort::SortKeys(nullptr, bytes, in, out, (int)count, 0, end_bit, st_));
        SYM_TRY(grow_tmp(bytes));
        SYM_TRY(hipcub::DeviceRadixSort::SortKeys(tmp_.p, bytes, in, out, (int)count, 0, end_bit, st_));
        return "";
    }

    template <class T>
    std::string exclusive_sum(T* in, T* out, int64_t count) {
        if (count <= 0) return "";
        size_t bytes = 0;
        SYM_TRY(hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, in, out, (int)count, st_));
        SYM_TRY(grow_tmp(bytes));
        SYM_TRY(hipcub::DeviceScan::ExclusiveSum(tmp_.p, bytes, in, out, (int)count, st_));
        return "";
    }

    template <class T>
    std::string inclusive_sum(T* in, T* out, int64_t count) {
        if (count <= 0) return "";
        size_t bytes = 0;
        SYM_TRY(hipcub::DeviceScan::InclusiveSum(nullptr, bytes, in, out, (int)count, st_));
        SYM_TRY(grow_tmp(bytes));
        SYM_TRY(hipcub::DeviceScan::InclusiveSum(tmp_.p, bytes, in, out, (int)count, st_));
        return "";
    }

    // Synchronizes and reports the first failed device-side check.
    std::string check_err() {
        int32_t e = 0;
        SYM_TRY(hipMemcpyAsync(&e, err_.p, sizeof(int32_t), hipMemcpyDeviceToHost, st_));
        SYM_TRY(hipStreamSynchronize(st_));
        if (e) return "internal: device step " + std::to_string(e);
        return "";
    }

    hipStream_t st_;
    int32_t n_ = 0;
    int64_t m_ = 0;
    int levels_ = 1;
    int rounds_ = 0;
    DBuf<char> tmp_;
    DBuf<int32_t> err_;
    DBuf<uint64_t> keys_, colkey_, rowkey_;
    DBuf<int32_t> ip0_, iperm_, parent_, first_, up_, kcolptr_, krow_, col2sn_;
};

}  // namespace

std::unique_ptr<SymbolicDevice> make_symbolic_device(hipStream_t stream) {
    return std::unique_ptr<SymbolicDevice>(new DeviceSymbolic(stream));
}

}  // namespace ckkt
