// Device-side view of the analysis plan and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>

namespace ckkt {

class SymbolicDevice;
// The symbolic factorization steps of the analysis run by kernels on
// `stream` (symbolic.hip).
std::unique_ptr<SymbolicDevice> make_symbolic_device(hipStream_t stream);

// Plain pointers into the bound workspace; passed to kernels by value.
struct DevPlan {
    int32_t n, m_eq, m_ineq, m, ns, ninst, hy;
    int64_t nnzk, nnzg;
    const int32_t *perm, *iperm;
    const int32_t *kcolptr, *k_wsrc, *k_diag, *prod_ptr, *prod_r, *prod_a, *prod_b;
    const int32_t *sn_start, *sn_rowptr, *sn_rows, *child_ptr, *child_list, *relmap, *kmap, *kcol;
    const int32_t *sn_parent, *sn_level;
    const int32_t *cb_ptr, *cb_src, *cb_len;
    const int64_t* cb_uoff;
    const int64_t *l_off, *u_off;
    const int32_t *u_ld;
    const int32_t *lvl_small, *lvl_big, *lvl_all, *big_tile_sn, *big_tile_col;
    const int32_t *wf_ptr, *wf_col, *wf_vidx;
    const int32_t *j_ptr, *j_col, *jt_ptr, *jt_row, *jt_vidx, *jt_gend;
    const int32_t *inst_of_var, *inst_of_eqrow;
    // rows of J split off K (dense_min > 0): rows with at least dense_min
    // entries, listed in drows; drowdot holds (J x)_r and (|J||x|)_r of each,
    // written by a launch of their own before a row kernel reads them
    const int32_t* drows;
    int32_t ndense, dense_min;
    double* drowdot;
    double* drowpart;  // per-chunk partials of drowdot (kDenseChunks per row)
};

// Values of the current system (device pointers owned by the caller).
struct SysVals {
    const double *w_val, *g_val, *h_val, *sigma_x, *sigma_s;
    double gamma;
    double delta_c = 0.0;  // HyKKT: K1 carries -delta_c I in its (2,2) block (Remark 1)
};

// Per-level launch geometry, computed on the host from the plan.
// The only large front of a level (loff < 0: the level has several), given
// to its panel and trailing-update launches as arguments: their workgroups
// then skip two rounds of dependent metadata loads.
struct BigOne {
    int32_t c0, w, f;
    int64_t loff;
};

struct LevelInfo {
    int32_t small_begin, small_count, small_maxf;
    int32_t small_split, small_split32;  // fronts [begin, begin+split) have f <= kCompactFront64 / 32
    int32_t small_maxf_a, small_maxf_a32;  // largest front of that compact class
    int32_t big_begin, big_count, big_maxw, big_maxf;
    int32_t all_begin, all_count, all_maxf, all_maxw;
    int32_t small_threads_a;   // workgroup size of the compact small-front class
    int32_t sweep_threads;     // workgroup size of the sweep kernels on this level
    int32_t tile_begin, tile_count;
    int32_t wide_front;         // FP64 levels whose largest big front reaches this use wide panels
    int32_t sweep_tiled_f;      // fronts with f >= this are swept by the tiled kernels
    int32_t sweep_small_count;  // fronts of the level swept one workgroup each (f < sweep_tiled_f)
    int32_t tflag_off;          // first block flag of the level's tiled fronts
    BigOne big_one;             // its only large front (loff < 0 if not one)
};

constexpr int kBigTile = 64;    // column tile of the tiled front path
// fronts of at most this many rows are assembled one column per wave in LDS
// (four column buffers of this length per workgroup)
constexpr int kInitColRows = 2048;
constexpr int kLdsBytes = 160 * 1024;   // LDS per workgroup on gfx950
constexpr int kFactorStaticLds = 2304;  // upper bound of k_factor_small's static LDS
constexpr int kSweepStaticLds = 1024;   // upper bound of k_fwd / k_bwd static LDS
// largest FP64 front held whole in LDS next to the kernel's static arrays:
// 140^2 * 8 + 2304 <= 160 KiB
constexpr int kLdsFront64 = 140;
// Leading dimension of a sweep's staged diagonal block for panels of at most
// maxw columns: at least min(64, maxw), odd (a row read across the lanes
// then falls on distinct LDS banks).
constexpr int sweep_diag_ld(int maxw) { return (maxw < 64 ? (maxw < 1 ? 1 : maxw) : 64) | 1; }
// largest front the sweep kernels can stage (front vector + 65 x 65 block)
constexpr int kSweepMaxFront = (kLdsBytes - kSweepStaticLds) / 8 - 65 * 65;
constexpr int kCompactFront64 = 64;  // fronts with f^2 * 8 <= 32 KiB (several workgroups per CU)
constexpr int kCompactFront32 = 90;  // fronts with f^2 * 4 <= 32 KiB
constexpr int kPanelNB = 32;    // panel width of the tiled front path
constexpr int kPanelRows = 256; // rows of the panel solved per workgroup
constexpr int kPanelLd = 64;    // leading dimension of the panel's diagonal block in LDS (one wave's rows)
// FP64 panel launch: rows below the block per workgroup (32 per wave), and
// its LDS (one kPanelLd x kPanelNB column exchange per wave)
constexpr int kFusedPanelRows = 128;
constexpr int kFusedPanelLds = 4 * kPanelLd * kPanelNB * 8;
// FP64 levels with fronts of at least kWideFront rows update their trailing
// matrices once per kWideRank columns (rank-kWideRank MFMA updates)
constexpr int kWideRank = 128;
constexpr int kWideFront = 2048;
constexpr int kWideTile = 64;  // trailing-matrix tile of the wide update
static_assert(kWideRank % kPanelNB == 0, "a wide panel is a whole number of panels");
// fronts with at least this many rows are swept by the tiled kernels (many
// workgroups, one launch per 64-column block); every such front is in the
// level's big list, whose fronts all exceed the LDS front limit
constexpr int kSweepTiledFront = 1024;
static_assert(kSweepTiledFront > kLdsFront64, "tiled sweep fronts must be big fronts");
static_assert(kSweepTiledFront <= kSweepMaxFront, "fronts below the tiled size fit the sweep LDS");

// ---- launchers (kernels.hip)
void launch_row_weights(const DevPlan& P, const SysVals& v, double* d, hipStream_t st);
void launch_assemble(const DevPlan& P, const SysVals& v, const double* d, double* K, int32_t* nonfinite,
                     hipStream_t st);
void launch_init_status(int32_t* status, bool keep_inputs, hipStream_t st);

// A second stream with its fork/join events (default priority): the
// tiled path of a level runs there, concurrently with its LDS fronts.
struct SideStream {
    hipStream_t stream = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};
constexpr int kMergeCompactFronts = 512;  // one launch for both LDS classes up to this many compact fronts

// Returns false (and launches nothing) if a launch would exceed the LDS limit.
// dscr: kPanelNB^2 doubles per tiled front of the level (factored diagonal
// blocks in transit between the panel and update launches).
template <typename T>
bool launch_factor_level(const DevPlan& P, const LevelInfo& L, const double* K, T* arena,
                         int32_t* status, const double* scale, hipStream_t st, const SideStream* side,
                         double* dscr);
// Completion flags of the tiled fronts' blocks when a level's tiled fronts
// are swept in one launch (null: one launch per column block).
struct TiledSync {
    const unsigned* ctl = nullptr;   // ctl[kCtlEpoch]: application counter
    unsigned* flags = nullptr;       // per level at LevelInfo::tflag_off, big_count x blocks
    int32_t* err = nullptr;          // set to 1 when a wait times out
    unsigned long long ticks = 0;    // wait limit in wall-clock ticks
};
template <typename T>
void launch_fwd_level(const DevPlan& P, const LevelInfo& L, const T* arena, double* v_perm,
                      double* uvec, hipStream_t st, const TiledSync* ts);
template <typename T>
void launch_bwd_level(const DevPlan& P, const LevelInfo& L, const T* arena, double* x_perm,
                      hipStream_t st, const TiledSync* ts);

// Dependency-driven sweeps: the supernodes lvl_all[0, wave_t1) (whole
// levels below wave_lvl, every front of order <= 64) are processed by
// single-wave workers, the rest by workgroup workers; both take supernodes
// from ticket counters in level order and wait on per-supernode flags.
struct SweepSched {
    int32_t wave_t1 = 0, wave_lvl = 0, ns = 0;
    // hybrid schedule: levels below pair_lvl (fronts of order <= 128 and
    // width <= 64) swept level by level, the workgroup workers from
    // lvl_all[pair_t1] on
    int32_t pair_t1 = 0, pair_lvl = 0;
    int32_t wave_grid = 1, group_grid = 1, ldd = 1;
    size_t group_lds = 0;
    // every workgroup-swept front has at most kGroupThreads rows: the
    // forward workgroup sweep holds the fronts of levels rows_lvl and above
    // (lvl_all[rows_t0] on) one row per thread, in a launch of its own
    bool rows = false;
    int32_t rows_grid = 1, rows_lvl = 0, rows_t0 = 0;
    unsigned long long ticks = 0;  // wait limit in wall-clock ticks
};
constexpr int kSweepWaveFront = 64;   // largest front of the single-wave class
// workgroup size of the row-held forward workgroup sweep: a front of at
// most this many rows is held one row per thread (its panel row of the
// current 64-column block in registers)
constexpr int kGroupThreads = 768;
// levels whose fronts all have at most this many rows stay on the LDS
// forward workgroup sweep (256 threads)
constexpr int kRowsMinFront = 256;
constexpr int kRowsMaxGrid = 48;  // workgroups of the row-held forward launch
constexpr int kSweepWaitSeconds = 4;  // a dependency wait longer than this is reported as an error
constexpr int kSweepCtlWords = 8;     // ticket counters and epoch
// largest number of supernodes above the single-wave levels for which the
// hybrid schedule is the default
constexpr int kHybridMaxTasks = 8192;
void launch_sweep_prep(unsigned* ctl, hipStream_t st);  // reset the tickets, advance the epoch
template <typename T>
void launch_fwd_sched(const DevPlan& P, const SweepSched& S, const T* arena, double* v_perm, double* uvec,
                      unsigned* ctl, unsigned* done, int32_t* err, hipStream_t st, bool waves);
template <typename T>
void launch_bwd_sched(const DevPlan& P, const SweepSched& S, const T* arena, double* x_perm, unsigned* ctl,
                      unsigned* done, int32_t* err, hipStream_t st, bool waves);
// Grid sizes (resident workgroups) and the wait limit for the current device.
bool sweep_sched_grids(SweepSched& S, int device);

// out[k] = in[perm[k]] * (scale ? scale[k] : 1)      (to the factor numbering)
void launch_gather_perm(const DevPlan& P, const double* in, double* out, const double* scale, hipStream_t st);
// out[perm[k]] = in[k] * (scale ? scale[k] : 1)      (back to the user numbering)
void launch_scatter_perm(const DevPlan& P, const double* in, double* out, const double* scale, hipStream_t st);

// Residual of LiftedKKT (hy = 0) or of K1 (hy = 1) with K unassembled,
// plus the componentwise backward error per instance (omega_bits, as
// uint64 of nonnegative doubles, must be zeroed first) and max |res|.
void launch_residual(const DevPlan& P, const SysVals& v, const double* d, const double* x,
                     const double* y, const double* rhs1, const double* rhs2, double* res1,
                     double* res2, double* tbuf, double* tabuf, unsigned long long* omega_bits,
                     unsigned long long* resmax_bits, hipStream_t st);
void launch_zero_u64(unsigned long long* p, int count, hipStream_t st);
void launch_maxabs(int n, const double* x, unsigned long long* bits, hipStream_t st);  // atomic max of |x|
// Augmented system K2 (delta_c = 0) over the slack rows of the plan; f is the
// right-hand side of K2 d = f, split like d into (f1: n, f2: slack rows,
// f3: equality rows (HyKKT), f4: slack rows).
void launch_k2_condense(const DevPlan& P, const SysVals& v, const double* d, const double* f1, const double* f2,
                        const double* f4, double* u, double* rb1, hipStream_t st);  // rb1 = f1 + H^T (E f4 - f2)
void launch_k2_recover(const DevPlan& P, const SysVals& v, const double* d, const double* f2, const double* f4,
                       const double* dx, double* ds, double* dz, hipStream_t st);
// R = -r - K2 d blockwise with the componentwise backward error (atomic max)
void launch_k2_residual(const DevPlan& P, const SysVals& v, const double* d, const double* r1, const double* r2,
                        const double* r3, const double* r4, const double* dx, const double* ds, const double* dy,
                        const double* dz, double* R1, double* R2, double* R3, double* R4,
                        unsigned long long* omega_bits, unsigned long long* resmax_bits, hipStream_t st);
void launch_bound_dual(int64_t count, const double* s, const double* v, double mu, const double* ds, double* dv,
                       hipStream_t st);  // dv = -(v ds - mu) / s - v
// Split dense rows (Woodbury around the factor of K_s): J_d from the J values;
// the capacitance C = D_d^{-1} + J_d Z and its Cholesky factor (status gets
// column n on a non-positive pivot); x -= Z C^{-1} (J_d x).
void launch_dense_setup_gather(const DevPlan& P, const SysVals& v, const int32_t* rows, int k, double* jd,
                               hipStream_t st);
void launch_dense_setup_cap(int n, int k, const int32_t* rows, const double* d, const double* jd, const double* z,
                            double* cpart, double* cap, int32_t* status, hipStream_t st);
void launch_dense_correct(int n, int k, const double* jd, const double* z, const double* cap, double* part,
                          double* u, double* x, hipStream_t st);

// Vector kernels
void launch_axpy(int n, double alpha, const double* x, double* y, hipStream_t st);  // y += a x
// y += x on the variables of the instances whose omega_bits entry exceeds tol
void launch_masked_axpy(const DevPlan& P, const unsigned long long* omega_bits, double tol, const double* x,
                        double* y, hipStream_t st);
void launch_copy(int n, const double* x, double* y, hipStream_t st);
void launch_fill(int n, double v, double* y, hipStream_t st);
void launch_shift_copy(int n, const double* x, double delta, double* y, hipStream_t st);  // y = x + delta
void launch_scale(int n, double alpha, double* y, hipStream_t st);                     // y = alpha y
// out_i = base_i + scale * (G^T y)_i   (base may be null)
void launch_gt(const DevPlan& P, const SysVals& v, const double* base, double scale, const double* y,
               double* out, hipStream_t st);
// out_r = (G x)_r - sub_r   (sub may be null)
void launch_g(const DevPlan& P, const SysVals& v, const double* x, const double* sub, double* out,
              hipStream_t st);

// Deterministic dot product into *result (device); partial buffer of
// kDotBlocks doubles.
constexpr int kDotBlocks = 256;
constexpr int kMaxDenseRows = 64;  // rows of J split off the condensed matrix at most
constexpr int kDenseChunkBuf = 64;  // chunks per split row in the partial-sum buffers (kernels' kDenseChunks)
constexpr int kAnalyzeThreads = 16;  // host threads of a batch analysis (orderings of the instances)
void launch_dot(int n, const double* a, const double* b, double* partial, double* result, hipStream_t st);

// CG helpers with device-resident scalars.  sc[0] = rr, sc[1] = pq,
// sc[2] = alpha, sc[3] = rr_new, sc[4] = beta.
void launch_cg_alpha(double* sc, hipStream_t st);                       // alpha = rr / pq
void launch_cg_update(int m, const double* sc, const double* p, const double* q, double* y, double* r,
                      hipStream_t st);                                  // y += a p, r -= a q
void launch_cg_beta(double* sc, hipStream_t st);                        // beta = rr_new / rr, rr = rr_new
void launch_cg_direction(int m, const double* sc, const double* r, double* p, hipStream_t st);  // p = r + b p
void launch_axpy_dev(int n, const double* sc, int idx, double sign, const double* x, double* y,
                     hipStream_t st);                                   // y += sign * sc[idx] * x

// Jacobi scale s_k = 1/sqrt(K_kk) over the factor numbering (FP32 path).
void launch_diag_scale(const DevPlan& P, const double* K, double* scale, hipStream_t st);

// ---- learned diagonal preconditioner (kernels_mlp.hip)
constexpr int kMlpF = 8, kMlpH = 64;
constexpr int kMlpNParam = kMlpH * kMlpF + kMlpH + kMlpH * kMlpH + kMlpH + kMlpH + 1;
void launch_kdiag(const DevPlan& P, const SysVals& v, const double* d, double* kd, hipStream_t st);
void launch_features(const DevPlan& P, const double* sx_new, const double* d_new, const double* kd_new,
                     const double* sx_old, const double* d_old, const double* kd_old, float* feat, hipStream_t st);
void launch_mlp_forward(int64_t n, const float* feat, const float* prm, float* out, float* cache, hipStream_t st);
size_t mlp_workspace_bytes(int64_t n);
// rows of the allocation-free backward; its scratch is a static device array
constexpr int64_t kMlpNoAllocRows = 32768;
// device address of that array on the current device (looked up once per
// device); null with *err set when the lookup fails
void* mlp_noalloc_scratch(hipError_t* err);
void launch_mlp_backward(int64_t n, const float* feat, const float* prm, const float* cache, const float* g_o,
                         float* grad, void* ws, hipStream_t st);
void launch_adam(int np, float* prm, const float* g, float* m, float* v, int step, float lr, hipStream_t st);
void launch_dscale(int n, const float* o, const double* x, double* out, hipStream_t st);
void launch_train_err(int n, const float* o, const double* y, const double* x, double* e, hipStream_t st);
void launch_train_gzD(int n, const float* o, const double* e, const double* sc, double* out, hipStream_t st);
void launch_train_go(int n, const float* o, const double* e, const double* y, const double* b, const double* w,
                     const double* sc, float* g_o, hipStream_t st);

}  // namespace ckkt
