// HIP kernels for gfx950: condensed assembly, multifrontal supernodal
// Cholesky, supernodal triangular sweeps and the FP64 vector work of the
// refinement and CG loops.
//
// Data layout in HBM (all in the caller-bound workspace):
//  * K (or K_gamma) values: lower triangle, CSC in the factor numbering, FP64.
//  * factor arena (FP64 or FP32): per supernode s a column-major panel of
//    f_s x w_s (leading dimension f_s = front order) followed by its r_s x r_s
//    update (Schur) matrix; fronts larger than the LDS limit keep the whole
//    f_s x f_s front there (panel = first w_s columns, update = trailing block).
//  * uvec: one FP64 update vector per supernode for the forward sweep,
//    indexed like the front row lists.
// Every reduction is a fixed-order tree and every scatter has a single
// writer, so results are bitwise reproducible run to run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <climits>
#include <cmath>
#include <cstdint>
#include <type_traits>

#include "device.hpp"

namespace ckkt {

namespace {

constexpr int kWave = 64;

__device__ __forceinline__ double jval(const SysVals& v, int64_t nnzg, int32_t a) {
    return a < nnzg ? v.g_val[a] : v.h_val[a - nnzg];
}

__device__ __forceinline__ double wave_sum(double x) {
    for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
    return x;
}

__device__ __forceinline__ double wave_max(double x) {
    for (int o = kWave / 2; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, kWave));
    return x;
}

__device__ __forceinline__ double nan_to_inf(double x) { return (x == x) ? x : INFINITY; }
// Value of lane k (k the same in every lane: a register read, no LDS trip).
template <typename T>
__device__ __forceinline__ T bcast(T x, int k);
template <>
__device__ __forceinline__ double bcast<double>(double x, int k) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), k);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), k);
    return __hiloint2double(hi, lo);
}
template <>
__device__ __forceinline__ float bcast<float>(float x, int k) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), k));
}

// x, opaque to the optimizer: lane comparisons made from it inside a loop
// are not hoisted out of it (64 lane masks kept across a loop would not fit
// in scalar registers).  Emits no instruction.
__device__ __forceinline__ int opaque(int x) {
    asm volatile("" : "+v"(x));
    return x;
}
// Completes the load that produced x here (the empty asm reads x, so the
// wait for it is placed before it), and leaves x as a value that is no
// longer a pending load: later uses inside loops then wait for nothing,
// in particular not for younger loads still in flight.
__device__ __forceinline__ double settle(double x) {
    asm volatile("" : "+v"(x));
    return x;
}

// Per-block maxima of (ratio, |res|) pushed with one atomic each when the
// whole block belongs to one instance, else one atomic per element.  The
// block must be 256 threads and every thread must call it.
// atomicMax on the bits of a non-negative double, skipped when the word
// already holds at least v (most blocks find a larger maximum there, so the
// atomics on one address stay few)
__device__ __forceinline__ void max_bits(unsigned long long* p, double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    if (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < b) atomicMax(p, b);
}

__device__ void block_max_push(bool active, int inst, double ratio, double num,
                               unsigned long long* omega_bits, unsigned long long* resmax_bits) {
    __shared__ int s_inst0, s_mixed;
    __shared__ double s_r[256 / kWave], s_n[256 / kWave];
    if (threadIdx.x == 0) { s_inst0 = inst; s_mixed = 0; }
    __syncthreads();
    if (active && inst != s_inst0) s_mixed = 1;
    __syncthreads();
    if (!active) { ratio = 0.0; num = 0.0; }
    ratio = nan_to_inf(ratio);
    num = nan_to_inf(num);
    if (s_mixed) {
        if (active) {
            max_bits(omega_bits + inst, ratio);
            max_bits(resmax_bits, num);
        }
        return;
    }
    ratio = wave_max(ratio);
    num = wave_max(num);
    if (threadIdx.x % kWave == 0) { s_r[threadIdx.x / kWave] = ratio; s_n[threadIdx.x / kWave] = num; }
    __syncthreads();
    if (threadIdx.x == 0 && s_inst0 >= 0) {
        double r = 0.0, nm = 0.0;
        for (int t = 0; t < (int)(blockDim.x / kWave); ++t) { r = fmax(r, s_r[t]); nm = fmax(nm, s_n[t]); }
        max_bits(omega_bits + s_inst0, r);
        max_bits(resmax_bits, nm);
    }
}

// ---------------------------------------------------------------- assembly

__global__ void k_row_weights(DevPlan P, SysVals v, double* __restrict__ d) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= P.m) return;
    if (P.hy) d[r] = (r < P.m_eq) ? v.gamma : v.sigma_s[r - P.m_eq];
    else d[r] = v.sigma_s[r];
}

// K[t] = W + [diag] sigma_x + sum_r d_r J_ra J_rb, gathered per slot
// (Sec. 2.2 K1: K = W + delta_w I + H^T D_H H; Sec. 3.1 K_gamma; Sec. 3.2 K_tau).
// One K slot per thread; a slot that is not finite (NaN or Inf in an input
// that reaches it) sets *nonfinite.
__global__ void k_assemble(DevPlan P, SysVals v, const double* __restrict__ d, double* __restrict__ K,
                           int32_t* nonfinite) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= P.nnzk) return;
    double acc = 0.0;
    int ws = P.k_wsrc[t];
    if (ws >= 0) acc = v.w_val[ws];
    int dg = P.k_diag[t];
    if (dg >= 0) acc += v.sigma_x[dg];
    int q1 = P.prod_ptr[t + 1];
    for (int q = P.prod_ptr[t]; q < q1; ++q) {
        int r = P.prod_r[q];
        acc += d[r] * (jval(v, P.nnzg, P.prod_a[q]) * jval(v, P.nnzg, P.prod_b[q]));
    }
    K[t] = acc;
    if (!(fabs(acc) <= DBL_MAX)) atomicOr(nonfinite, 1);
}

// status: [0] failing column, [1] FP32 pivot floors, [2] sweep wait failure,
// [3] non-finite assembled entry (kept when `keep_inputs`: same K)
__global__ void k_init_status(int32_t* status, int keep_inputs) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        status[0] = INT_MAX;
        status[1] = 0;
        status[2] = 0;
        if (!keep_inputs) status[3] = 0;
    }
}

__global__ void k_diag_scale(DevPlan P, const double* __restrict__ K, double* __restrict__ scale) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P.n) return;
    double dk = K[P.kcolptr[k]];
    scale[k] = dk > 0.0 ? 1.0 / sqrt(dk) : 1.0;
}

// --------------------------------------------------------- factorization

// Pivot handling.  FP64: a non-positive pivot records its column and the
// factorization is reported as failed.  FP32 (factor of the Jacobi-scaled
// matrix, unit diagonal): pivots below a floor are raised to it (static
// pivoting); the count is recorded and the factor serves as a
// preconditioner for the FP64 refinement.  Both return the pivot sqrt(d)
// and its reciprocal, from the hardware reciprocal square root refined by
// Newton's iteration y <- y (3 - d y^2) / 2 (two steps for FP64, one for
// FP32), which keeps the square root and the division off the chain.
template <typename T>
__device__ __forceinline__ T pivot_root(T d, int col, int32_t* status, bool report, T& rinv);

template <>
__device__ __forceinline__ double pivot_root<double>(double d, int col, int32_t* status, bool report,
                                                     double& rinv) {
    if (!(d > 0.0)) {
        if (report && status) atomicMin(status, col);
        rinv = 1.0;
        return 1.0;
    }
    double y = __builtin_amdgcn_rsq(d);
    const double hd = 0.5 * d;
    y = y * fma(-hd * y, y, 1.5);
    y = y * fma(-hd * y, y, 1.5);
    rinv = y;
    return d * y;
}

template <>
__device__ __forceinline__ float pivot_root<float>(float d, int col, int32_t* status, bool report, float& rinv) {
    const float floor_ = 1e-5f;
    if (!(d > floor_)) {
        if (report && status) atomicAdd(status + 1, 1);
        d = floor_;
    }
    float y = __builtin_amdgcn_rsqf(d);
    y = y * fmaf(-0.5f * d * y, y, 1.5f);
    rinv = y;
    return d * y;
}

// Pivot of the branch-free register Cholesky forms: as pivot_root, with the failure
// (FP64: d not positive; FP32: d below the floor) returned instead of
// reported, so that the column loop holds no branch.
template <typename T>
__device__ __forceinline__ T pivot_select(T d, T& rinv, bool& fail);
template <>
__device__ __forceinline__ double pivot_select<double>(double d, double& rinv, bool& fail) {
    fail = !(d > 0.0);
    d = fail ? 1.0 : d;
    double y = __builtin_amdgcn_rsq(d);
    y = y * fma(-0.5 * d * y, y, 1.5);
    y = y * fma(-0.5 * d * y, y, 1.5);
    rinv = y;
    return d * y;
}
template <>
__device__ __forceinline__ float pivot_select<float>(float d, float& rinv, bool& fail) {
    const float floor_ = 1e-5f;
    fail = !(d > floor_);
    d = fail ? floor_ : d;
    float y = __builtin_amdgcn_rsqf(d);
    y = y * fmaf(-0.5f * d * y, y, 1.5f);
    rinv = y;
    return d * y;
}

constexpr int kDiag = 16;  // diagonal block of the blocked front factorization
constexpr int kMaxChildBatch = 64;  // children whose metadata is staged at once

// sum_{t < n} x[t * ldx] * y[t * ldy] over LDS operands, eight products per
// step with all sixteen loads issued first (their latencies overlap), the
// rest in steps of four, two and one; two partial sums.
template <typename T>
__device__ __forceinline__ T row_dot(const T* x, const T* y, int ldx, int ldy, int n) {
    T acc0 = T(0), acc1 = T(0);
    int t = 0;
    for (; t + 8 <= n; t += 8) {
        T a[8], b[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            a[u] = x[(t + u) * ldx];
            b[u] = y[(t + u) * ldy];
        }
#pragma unroll
        for (int u = 0; u < 8; u += 2) {
            acc0 += a[u] * b[u];
            acc1 += a[u + 1] * b[u + 1];
        }
    }
    if (t + 4 <= n) {
        const T a0 = x[t * ldx], a1 = x[(t + 1) * ldx], a2 = x[(t + 2) * ldx], a3 = x[(t + 3) * ldx];
        const T b0 = y[t * ldy], b1 = y[(t + 1) * ldy], b2 = y[(t + 2) * ldy], b3 = y[(t + 3) * ldy];
        acc0 += a0 * b0;
        acc1 += a1 * b1;
        acc0 += a2 * b2;
        acc1 += a3 * b3;
        t += 4;
    }
    if (t + 2 <= n) {
        const T a0 = x[t * ldx], a1 = x[(t + 1) * ldx];
        const T b0 = y[t * ldy], b1 = y[(t + 1) * ldy];
        acc0 += a0 * b0;
        acc1 += a1 * b1;
        t += 2;
    }
    if (t < n) acc0 += x[t * ldx] * y[t * ldy];
    return acc0 + acc1;
}

// One wave factors the nb x nb diagonal block at A (LDS, column-major,
// leading dimension ld) in place and leaves the reciprocal pivots in
// rdiag[0, nb).  Left-looking: at step j lane i (i >= j) forms
// A(i, j) - sum_{t<j} L(i, t) L(j, t) from its own finished row and row j
// (an LDS broadcast), the pivot comes from lane j by a register broadcast,
// and the column is scaled.  No read-modify-write chains through LDS, and
// the loops stay rolled (small code).  Rows written by other lanes in
// earlier steps are visible because one wave's LDS operations complete in
// order.  The caller synchronises before and after.
template <typename T>
__device__ void wave_potrf(T* A, int ld, int nb, int col0, int32_t* status, T* rdiag) {
    const int lane = threadIdx.x % kWave;
    for (int j = 0; j < nb; ++j) {
        const bool act = lane < nb && lane >= j;
        const int ri = act ? lane : j;  // inactive lanes read a valid row and discard it
        const T d = A[ri + j * ld] - row_dot<T>(A + ri, A + j, ld, ld, j);
        const T djj = bcast(d, j);
        T r;
        const T ljj = pivot_root<T>(djj, col0 + j, status, lane == j, r);
        if (act) A[lane + j * ld] = (lane == j) ? ljj : d * r;
        if (lane == j) rdiag[j] = r;
    }
}

// Rows [i0, i1) of B (column-major, leading dimension ld) times D^{-T} in
// place, D the factored nb x nb diagonal block (leading dimension ldd) with
// reciprocal pivots rdiag; one thread per row, left-looking (x_j from the
// already solved x_t, t < j, and row j of D by LDS broadcast).
template <typename T>
__device__ void rows_trsm(T* B, int ld, const T* D, int ldd, int nb, int i0, int i1, const T* rdiag) {
    for (int i = i0 + (int)threadIdx.x; i < i1; i += blockDim.x) {
        for (int j = 0; j < nb; ++j)
            B[i + j * ld] = (B[i + j * ld] - row_dot<T>(B + i, D + j, ld, ldd, j)) * rdiag[j];
    }
}

// Full kDiag-column diagonal block of an LDS front (leading dimension ld),
// right-looking with row i in the registers of lane i (lanes 0..kDiag-1
// call it).  As k_big_panel_fused: select pivots (a failure is recorded after
// the loop as pivot_root records it), the column store writes back the old
// value above the diagonal (one store per lane, no branch), and a
// scheduling barrier per column keeps each column's updates in that
// column instead of letting them sink in front of the next pivot.
template <typename T>
__device__ __forceinline__ void potrf_diag_reg(T* A, int ld, int col0, int32_t* status, T* rdiag) {
    constexpr int NB = kDiag;
    const int lane = threadIdx.x % kWave;
    T a[NB];
#pragma unroll
    for (int t = 0; t < NB; ++t) a[t] = t <= lane ? A[lane + t * ld] : T(0);
    int first_bad = INT_MAX, n_bad = 0;
    // as k_big_panel_fused: the next column's entry takes its multiplier by a
    // lane read, the others one column late from LDS (loaded while the next
    // pivot is computed), in the same order of operations
    T m[NB];
    T lprev = T(0);
#pragma unroll
    for (int t = 0; t < NB; ++t) m[t] = T(0);
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const T old = A[lane + j * ld];
        T r;
        bool fail;
        const T ljj = pivot_select<T>(bcast<T>(a[j], j), r, fail);
        if (j >= 1) {
#pragma unroll
            for (int k = j + 1; k < NB; ++k) a[k] = fma(-lprev, m[k], a[k]);
        }
        first_bad = (fail && first_bad == INT_MAX) ? j : first_bad;
        n_bad += fail ? 1 : 0;
        const T lij = lane == j ? ljj : a[j] * r;
        A[lane + j * ld] = lane >= j ? lij : old;
        rdiag[j] = r;
        if (j + 1 < NB) a[j + 1] = fma(-lij, bcast<T>(lij, j + 1), a[j + 1]);
#pragma unroll
        for (int k = j + 2; k < NB; ++k) m[k] = A[k + j * ld];
        lprev = lij;
        __builtin_amdgcn_sched_barrier(0);
    }
    if (status && lane == 0) {
        if (std::is_same<T, double>::value) {
            if (first_bad != INT_MAX) atomicMin(status, col0 + first_bad);
        } else if (n_bad > 0) {
            atomicAdd(status + 1, n_bad);
        }
    }
}

// Rows [i0, i1) of B times the inverse transpose of a factored full
// kDiag-column block D, one row per thread in registers, right-looking.
template <typename T>
__device__ __forceinline__ void rows_trsm_diag_reg(T* B, int ld, const T* D, int ldd, int i0, int i1,
                                                   const T* rdiag) {
    constexpr int NB = kDiag;
    for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        T x[NB];
#pragma unroll
        for (int t = 0; t < NB; ++t) x[t] = B[i + t * ld];
        // the next column's multipliers are loaded while the current
        // column's are applied
        T dc[NB], dn[NB];
        T rc = rdiag[0];
#pragma unroll
        for (int k = 1; k < NB; ++k) dc[k] = D[k];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            T rn = T(0);
            if (j + 1 < NB) {
                rn = rdiag[j + 1];
#pragma unroll
                for (int k = j + 2; k < NB; ++k) dn[k] = D[k + (j + 1) * ldd];
            }
            x[j] *= rc;
#pragma unroll
            for (int k = j + 1; k < NB; ++k) x[k] = fma(-x[j], dc[k], x[k]);
#pragma unroll
            for (int k = j + 2; k < NB; ++k) dc[k] = dn[k];
            rc = rn;
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int t = 0; t < NB; ++t) B[i + t * ld] = x[t];
    }
}

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

// The 16 x 16 x 4 matrix-core step of each factor precision: acc += A B
// with lane l supplying A(l % 16, l / 16) and B(l / 16, l % 16); the
// output row of accumulator register r in lane l differs between the two
// instructions (FP64: 4 r + l / 16; FP32: 4 (l / 16) + r; column l % 16).
template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
    typedef dbl4 acc;
    static __device__ __forceinline__ acc zero() { return dbl4{0.0, 0.0, 0.0, 0.0}; }
    static __device__ __forceinline__ acc step(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int r, int lk) { return 4 * r + lk; }
};
template <>
struct Mfma<float> {
    typedef flt4 acc;
    static __device__ __forceinline__ acc zero() { return flt4{0.f, 0.f, 0.f, 0.f}; }
    static __device__ __forceinline__ acc step(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int r, int lk) { return 4 * lk + r; }
};

// Lower-triangular rank-k update on the matrix cores (FP64):
//   out(i, j, (P P^T)_ij)  for i in [i0, i1), j in [j0, j1), i >= j,
// where P holds columns [t0, t1) of the LDS front F (leading dimension f).
// One 32 x 32 output block (2 x 2 tiles of 16 x 16) per wave at a time, K
// in steps of 4 with v_mfma_f64_16x16x4f64: lane l supplies A(l % 16, l / 16)
// and B(l / 16, l % 16) and receives D(4 r + l / 16, l % 16) in register r.
// Blocks entirely above the diagonal are skipped (wave-uniform), so every
// matrix instruction runs with all lanes active.
template <typename T, typename Out>
__device__ __forceinline__ void syrk_mfma(const T* F, int f, int i0, int i1, int j0, int j1, int t0, int t1,
                                          Out out) {
    using M = Mfma<T>;
    // 32 x 32 blocks per wave: 2 x 2 MFMA tiles, four independent
    // accumulators sharing each K step's operand loads
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave, nw = blockDim.x / kWave;
    const int li = lane % 16, lk = lane / 16;
    const int ni = (i1 - i0 + 31) / 32, nj = (j1 - j0 + 31) / 32;
    for (int q = wid; q < ni * nj; q += nw) {
        const int ib = i0 + 32 * (q % ni), jb = j0 + 32 * (q / ni);
        if (ib + 31 < jb) continue;
        bool ai[2], bj[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            ai[a] = ib + 16 * a + li < i1;
            bj[a] = jb + 16 * a + li < j1;
        }
        typename M::acc c[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) c[a][b] = M::zero();
#pragma unroll 2
        for (int t = t0; t < t1; t += 4) {
            const int tk = t + lk;
            const bool kin = tk < t1;
            T av[2], bv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                av[a] = (ai[a] && kin) ? F[ib + 16 * a + li + tk * f] : T(0);
                bv[a] = (bj[a] && kin) ? F[jb + 16 * a + li + tk * f] : T(0);
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) c[a][b] = M::step(av[a], bv[b], c[a][b]);
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = ib + 16 * a + M::row(r, lk), j = jb + 16 * b + li;
                    if (i < i1 && j < j1 && i >= j) out(i, j, c[a][b][r]);
                }
    }
}

// Fronts that fit in LDS (f^2 elements <= 160 KiB): one workgroup per front.
// Assemble (K columns + extend-add of the children's update matrices in
// child order), blocked partial Cholesky of the first w columns (kDiag-
// column diagonal blocks factored by one wave, parallel row solves and
// panel updates), store the panel, and form the update matrix
// U = F22 - L21 L21^T in one parallel pass (multifrontal method).  REG:
// the large class (256 threads, one front per CU), whose full FP64 diagonal
// blocks use the register forms (potrf_diag_reg, rows_trsm_diag_reg); the
// compact class keeps the left-looking LDS forms (fewer registers, several
// workgroups per CU).
template <typename T, bool REG>
__global__ void __launch_bounds__(256)
k_factor_small(DevPlan P, const double* __restrict__ K, T* __restrict__ arena, int list_begin,
               int32_t* status, const double* __restrict__ scale) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* F = reinterpret_cast<T*>(smem_raw);
    const int s = P.lvl_small[list_begin + blockIdx.x];
    const int c0 = P.sn_start[s], c1 = P.sn_start[s + 1], w = c1 - c0;
    const int ro = P.sn_rowptr[s], f = P.sn_rowptr[s + 1] - ro, r = f - w;
    const int tid = threadIdx.x, nt = blockDim.x;
    // An FP64 factorization that has met a non-positive pivot is not
    // finished: every later front returns at once (the decision is taken
    // from one read by thread 0, so the whole workgroup leaves together).
    __shared__ int s_failed;
    if (sizeof(T) == 8 && tid == 0) s_failed = *reinterpret_cast<volatile const int32_t*>(status) != INT_MAX;
    for (int i = tid; i < f * f; i += nt) F[i] = T(0);
    __syncthreads();
    if (sizeof(T) == 8 && s_failed) return;
    // K entries of the w columns: one contiguous slot range (four entries
    // per thread in flight)
    {
        const int t0 = P.kcolptr[c0], t1 = P.kcolptr[c1];
        for (int base = t0; base < t1; base += 4 * nt) {
            int pr[4], j[4];
            double val[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int t = base + u * nt + tid;
                const bool in = t < t1;
                pr[u] = in ? P.kmap[t] : 0;
                j[u] = in ? P.kcol[t] : c0;
                val[u] = in ? K[t] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (base + u * nt + tid < t1) {
                    double x = val[u];
                    if (scale) x *= scale[j[u]] * scale[P.sn_rows[ro + pr[u]]];
                    F[pr[u] + (j[u] - c0) * f] = (T)x;
                }
            }
        }
    }
    __syncthreads();
    // extend-add, one child after the other (fixed order), each child's
    // lower update entries column by column: every wave takes columns
    // wid, wid + nw, ... kCols at a time, lane l rows b + l, b + 64 + l, ...
    // (kChunks of them, the rest in a tail loop), so that kCols x kChunks
    // entries per lane (with their row map entries) are loaded before they
    // are added; child metadata prefetched
    {
        __shared__ int64_t c_uoff[kMaxChildBatch];
        __shared__ int c_rel[kMaxChildBatch], c_rc[kMaxChildBatch], c_ld[kMaxChildBatch];
        const int q0 = P.child_ptr[s], nch = P.child_ptr[s + 1] - q0;
        const int lane = tid % kWave, wid = tid / kWave, nw = nt / kWave;
        for (int base = 0; base < nch; base += kMaxChildBatch) {
            const int nb_ch = min(kMaxChildBatch, nch - base);
            if (tid < nb_ch) {
                const int c = P.child_list[q0 + base + tid];
                const int wc = P.sn_start[c + 1] - P.sn_start[c];
                const int roc = P.sn_rowptr[c];
                c_rel[tid] = roc + wc;
                c_rc[tid] = P.sn_rowptr[c + 1] - roc - wc;
                c_uoff[tid] = P.u_off[c];
                c_ld[tid] = P.u_ld[c];
            }
            __syncthreads();
            for (int q = 0; q < nb_ch; ++q) {
                const int rc = c_rc[q], ld = c_ld[q];
                const int* rel = P.relmap + c_rel[q];
                const T* U = arena + c_uoff[q];
                constexpr int kChunks = REG ? 2 : 1, kCols = REG ? 8 : 4;
                for (int b0 = wid; b0 < rc; b0 += kCols * nw) {
                    T u[kCols][kChunks];
                    int ra[kCols][kChunks], rb[kCols];
#pragma unroll
                    for (int k = 0; k < kCols; ++k) {
                        const int b = b0 + k * nw;
                        const bool vb = b < rc;
                        rb[k] = vb ? rel[b] : 0;
#pragma unroll
                        for (int c = 0; c < kChunks; ++c) {
                            const int a = b + c * kWave + lane;
                            const bool in = vb && a < rc;
                            u[k][c] = in ? U[a + (int64_t)b * ld] : T(0);
                            ra[k][c] = in ? rel[a] : -1;
                        }
                    }
#pragma unroll
                    for (int k = 0; k < kCols; ++k)
#pragma unroll
                        for (int c = 0; c < kChunks; ++c)
                            if (ra[k][c] >= 0) F[ra[k][c] + rb[k] * f] += u[k][c];
#pragma unroll
                    for (int k = 0; k < kCols; ++k) {
                        const int b = b0 + k * nw;
                        for (int a = b + kChunks * kWave + lane; b < rc && a < rc; a += kWave)
                            F[rel[a] + rb[k] * f] += U[a + (int64_t)b * ld];
                    }
                }
                __syncthreads();
            }
        }
    }
    __shared__ T s_rdiag[kDiag];
    for (int kb = 0; kb < w; kb += kDiag) {
        const int nb = min(kDiag, w - kb);
        T* Dg = F + kb + kb * f;
        if (REG && sizeof(T) == 8 && nb == kDiag) {  // large class, FP64, full block
            if (tid < kDiag) potrf_diag_reg<T>(Dg, f, c0 + kb, status, s_rdiag);
            __syncthreads();
            rows_trsm_diag_reg<T>(F + kb * f, f, Dg, f, kb + nb, f, s_rdiag);
        } else {
            if (tid < kWave) wave_potrf<T>(Dg, f, nb, c0 + kb, status, s_rdiag);
            __syncthreads();
            rows_trsm<T>(F + kb * f, f, Dg, f, nb, kb + nb, f, s_rdiag);
        }
        __syncthreads();
        // remaining panel columns [kb+nb, w), rows >= column
        const int j0 = kb + nb, mc = w - j0;
        if (mc > 0) syrk_mfma<T>(F, f, j0, f, j0, w, kb, kb + nb, [&](int i, int j, T v) { F[i + j * f] -= v; });
        __syncthreads();
    }
    T* L = arena + P.l_off[s];
    for (int idx = tid; idx < f * w; idx += nt) L[idx] = F[idx];
    T* U = arena + P.u_off[s];
    if (r > 0)
        syrk_mfma<T>(F, f, w, f, w, f, 0, w,
                     [&](int i, int j, T v) { U[(i - w) + (int64_t)(j - w) * r] = F[i + j * f] - v; });
}

// Large fronts, step 1: one workgroup per 64-column tile of a front kept in
// the arena.  Zero the lower part of the tile, scatter the K entries of its
// columns, then add every child's update entries whose destination column
// lies in the tile (children in fixed order; each entry has one writer).
// When the tile fits in LDS (lds_rows >= f) it is assembled there, child by
// child with eight loads per thread in flight, and written out once;
// otherwise it is assembled in place in the arena column by column.
template <typename T>
__global__ void __launch_bounds__(256)
k_big_init(DevPlan P, const double* __restrict__ K, T* __restrict__ arena, int tile_begin,
           const double* __restrict__ scale, int lds_rows) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int tix = tile_begin + blockIdx.x;
    const int s = P.big_tile_sn[tix], col0 = P.big_tile_col[tix];
    const int c0 = P.sn_start[s], w = P.sn_start[s + 1] - c0;
    const int ro = P.sn_rowptr[s], f = P.sn_rowptr[s + 1] - ro;
    const int col1 = min(col0 + kBigTile, f);
    T* F = arena + P.l_off[s];
    const int tid = threadIdx.x, nt = blockDim.x;
    if (f <= lds_rows) {
        T* Tl = reinterpret_cast<T*>(smem_raw);  // tile column j - col0 at (j - col0) * f
        const int nc = col1 - col0;
        for (int i = tid; i < nc * f; i += nt) Tl[i] = T(0);
        __syncthreads();
        if (col0 < w) {
            const int ce = c0 + min(col1, w);
            for (int t = P.kcolptr[c0 + col0] + tid; t < P.kcolptr[ce]; t += nt) {
                const int pr = P.kmap[t], j = P.kcol[t];
                double val = K[t];
                if (scale) val *= scale[j] * scale[P.sn_rows[ro + pr]];
                Tl[pr + (j - c0 - col0) * f] = (T)val;
            }
        }
        __syncthreads();
        __shared__ int s_b[2];
        for (int q = P.child_ptr[s]; q < P.child_ptr[s + 1]; ++q) {
            const int c = P.child_list[q];
            const int wc = P.sn_start[c + 1] - P.sn_start[c];
            const int roc = P.sn_rowptr[c], rc = P.sn_rowptr[c + 1] - roc - wc;
            const int* rel = P.relmap + roc + wc;
            const T* U = arena + P.u_off[c];
            const int ld = P.u_ld[c];
            // child columns landing in the tile: a contiguous range (rel increases)
            if (tid == 0) { s_b[0] = rc; s_b[1] = 0; }
            __syncthreads();
            for (int b2 = tid; b2 < rc; b2 += nt) {
                const int d = rel[b2];
                if (d >= col0 && d < col1) { atomicMin(&s_b[0], b2); atomicMax(&s_b[1], b2 + 1); }
            }
            __syncthreads();
            const int b0 = s_b[0], nbc = s_b[1] - s_b[0];
            const int tot = nbc > 0 ? nbc * rc : 0;
            for (int base = 0; base < tot; base += 8 * nt) {
                T u8[8];
                int dr[8], dc[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int idx = base + u * nt + tid;
                    const int a2 = idx % rc, b2 = b0 + idx / rc;
                    const bool in = idx < tot && a2 >= b2;
                    u8[u] = in ? U[a2 + (int64_t)b2 * ld] : T(0);
                    dr[u] = in ? rel[a2] : -1;
                    dc[u] = in ? rel[b2] : 0;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (dr[u] >= 0) Tl[dr[u] + (dc[u] - col0) * f] += u8[u];
            }
            __syncthreads();
        }
        for (int i = tid; i < nc * f; i += nt) {
            const int r = i % f, jj = i / f;
            if (r >= col0 + jj) F[r + (int64_t)(col0 + jj) * f] = Tl[i];
        }
        return;
    }
    for (int j = col0; j < col1; ++j)
        for (int i = j + tid; i < f; i += nt) F[i + (int64_t)j * f] = T(0);
    __syncthreads();
    if (col0 < w) {
        const int ce = c0 + min(col1, w);
        for (int t = P.kcolptr[c0 + col0] + tid; t < P.kcolptr[ce]; t += nt) {
            const int pr = P.kmap[t], j = P.kcol[t];
            double val = K[t];
            if (scale) val *= scale[j] * scale[P.sn_rows[ro + pr]];
            F[pr + (int64_t)(j - c0) * f] = (T)val;
        }
    }
    __syncthreads();
    // one wave per column; a child's column lands on distinct rows, so the
    // eight entries of a batch are loaded, added and stored together
    const int lane = tid % kWave, wid = tid / kWave, nw = nt / kWave;
    for (int j = col0 + wid; j < col1; j += nw) {
        T* Fj = F + (int64_t)j * f;
        const int q1 = P.cb_ptr[ro + j + 1];
        for (int q = P.cb_ptr[ro + j]; q < q1; ++q) {
            const int src = P.cb_src[q], len = P.cb_len[q];
            const T* Ucol = arena + P.cb_uoff[q];
            const int* rel = P.relmap + src;
            for (int a0 = 0; a0 < len; a0 += 8 * kWave) {
                int r[8];
                T u[8], fv[8];
#pragma unroll
                for (int v = 0; v < 8; ++v) {
                    const int a = a0 + v * kWave + lane;
                    r[v] = a < len ? rel[a] : -1;
                    u[v] = a < len ? Ucol[a] : T(0);
                }
#pragma unroll
                for (int v = 0; v < 8; ++v) fv[v] = r[v] >= 0 ? Fj[r[v]] : T(0);
#pragma unroll
                for (int v = 0; v < 8; ++v)
                    if (r[v] >= 0) Fj[r[v]] = fv[v] + u[v];
            }
        }
    }
}

// Large fronts, step 1, for fronts of at most kInitColRows rows: one wave
// per front column, assembled in LDS.  The column is zeroed from the
// diagonal down, the K entries of the supernode's own columns are stored,
// the children's update columns landing on it are added in child order
// (the same order, so the same sums, as k_big_init), and the column is
// written to the arena once.  Every wave works on its own column buffer and
// a wave's LDS operations complete in issue order, so no barrier is needed;
// the child metadata of up to kWave contributions is fetched by the lanes
// at once and broadcast.  Grid (tile, kBigTile / 4), 256 threads: block y
// takes columns 4 y .. 4 y + 3 of the tile, one per wave.
template <typename T>
__global__ void __launch_bounds__(256)
k_big_init_cols(DevPlan P, const double* __restrict__ K, T* __restrict__ arena, int tile_begin,
                const double* __restrict__ scale, int lds_rows) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    const int tix = tile_begin + blockIdx.x;
    const int s = P.big_tile_sn[tix];
    const int j = P.big_tile_col[tix] + 4 * (int)blockIdx.y + wid;  // front column of this wave
    const int ro = P.sn_rowptr[s], f = P.sn_rowptr[s + 1] - ro;
    if (j >= f) return;  // wave-uniform; no workgroup barrier follows
    const int c0 = P.sn_start[s], w = P.sn_start[s + 1] - c0;
    T* col = reinterpret_cast<T*>(smem_raw) + (size_t)wid * lds_rows;
    // metadata of the contributions to this column (one per lane), issued
    // with the K entries' loads
    const int q0 = P.cb_ptr[ro + j], nq = P.cb_ptr[ro + j + 1] - q0;
    int m_src = 0, m_len = 0;
    int64_t m_off = 0;
    if (lane < nq) {
        m_src = P.cb_src[q0 + lane];
        m_len = P.cb_len[q0 + lane];
        m_off = P.cb_uoff[q0 + lane];
    }
    for (int i = j + lane; i < f; i += kWave) col[i] = T(0);
    if (j < w) {
        const int t0 = P.kcolptr[c0 + j], t1 = P.kcolptr[c0 + j + 1];
        const double sj = scale ? scale[c0 + j] : 1.0;
        for (int t = t0 + lane; t < t1; t += kWave) {
            const int pr = P.kmap[t];
            double v = K[t];
            if (scale) v *= sj * scale[P.sn_rows[ro + pr]];
            col[pr] = (T)v;
        }
    }
    for (int q = 0; q < nq; ++q) {
        int src, len;
        int64_t off;
        if (q < kWave) {
            src = __builtin_amdgcn_readlane(m_src, q);
            len = __builtin_amdgcn_readlane(m_len, q);
            off = ((int64_t)__builtin_amdgcn_readlane((int)(m_off >> 32), q) << 32) |
                  (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)m_off, q);
        } else {
            src = P.cb_src[q0 + q];
            len = P.cb_len[q0 + q];
            off = P.cb_uoff[q0 + q];
        }
        const T* U = arena + off;
        const int* rel = P.relmap + src;
        for (int a0 = 0; a0 < len; a0 += 8 * kWave) {
            int r[8];
            T u[8];
#pragma unroll
            for (int v = 0; v < 8; ++v) {
                const int a = a0 + v * kWave + lane;
                r[v] = a < len ? rel[a] : -1;
                u[v] = a < len ? U[a] : T(0);
            }
#pragma unroll
            for (int v = 0; v < 8; ++v)
                if (r[v] >= 0) col[r[v]] += u[v];
        }
    }
    T* Fj = arena + P.l_off[s] + (int64_t)j * f;
    for (int i = j + lane; i < f; i += kWave) Fj[i] = col[i];
}

// Cholesky of the nb x nb (nb <= 32) lower triangle D (LDS, leading
// dimension kPanelLd) by one wave (the FP32 panels), right-looking with the
// rows in registers: lane i keeps row i; per column j the pivot comes from
// lane j, the column is scaled and written back to LDS, and every lane
// subtracts l_ij l_kj from its entries k > j, reading l_kj as LDS
// broadcasts (one address for the whole wave).
template <typename T>
__device__ __forceinline__ void potrf32_reg(T* D, int nb, int col0, int32_t* status, T* rdiag) {
    const int lane = threadIdx.x % kWave;
    const bool act = lane < nb;
    T a[kPanelNB];
#pragma unroll
    for (int t = 0; t < kPanelNB; ++t) a[t] = (act && t <= lane && t < nb) ? D[lane + t * kPanelLd] : T(0);
#pragma unroll
    for (int j = 0; j < kPanelNB; ++j) {
        if (j < nb) {
            T r;
            const T ljj = pivot_root<T>(bcast<T>(a[j], j), col0 + j, status, lane == j, r);
            const T lij = lane == j ? ljj : a[j] * r;
            if (act && lane >= j) D[lane + j * kPanelLd] = lij;
            if (lane == j) rdiag[j] = r;
#pragma unroll
            for (int k = j + 1; k < kPanelNB; ++k)
                if (k < nb) a[k] = fma(-lij, D[k + j * kPanelLd], a[k]);
        }
    }
}

// Large fronts, step 2 in FP32 (per block column kb), grid (row chunk,
// front): every workgroup stages the diagonal block (nb x nb, nb <= 32), one
// wave factors it (the same arithmetic in every workgroup) while the
// workgroup's rows are loaded, and each thread then solves its row of the
// chunk (kPanelRows rows below the block) in registers, right-looking, with
// the factored block read as LDS broadcasts.  With one chunk the factored
// block is written back in place; with several, chunk 0 leaves it in dscr
// (another chunk may still be reading the original block) and the
// trailing-update launch copies it into the front.  (FP64 panels:
// k_big_panel_fused.)
template <typename T>
__global__ void __launch_bounds__(256)
k_big_panel(DevPlan P, T* __restrict__ arena, int list_begin, int kb, int32_t* status, T* __restrict__ dscr) {
    static_assert(kPanelRows == 256, "one row per thread");
    static_assert(sizeof(T) == 4, "the FP32 panel");
    __shared__ T D[kPanelLd * kPanelNB];
    __shared__ T s_rdiag[kPanelNB];
    const int s = P.lvl_big[list_begin + blockIdx.y];
    const int c0 = P.sn_start[s], w = P.sn_start[s + 1] - c0;
    const int f = P.sn_rowptr[s + 1] - P.sn_rowptr[s];
    if (kb >= w) return;
    const int nb = min(kPanelNB, w - kb);
    T* F = arena + P.l_off[s];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int r0 = kb + nb + blockIdx.x * kPanelRows;
    if (blockIdx.x > 0 && r0 >= f) return;
    const int nr = r0 < f ? min(kPanelRows, f - r0) : 0;
    // the diagonal block's loads and this thread's row are issued together
    T t4[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int idx = u * nt + tid;
        const int i = idx % nb, j = idx / nb;
        t4[u] = (idx < nb * nb && i >= j) ? F[(kb + i) + (int64_t)(kb + j) * f] : T(0);
    }
    const bool row = tid < nr;
    T* Fr = F + (row ? r0 + tid : kb) + (int64_t)kb * f;
    T x[kPanelNB];
#pragma unroll
    for (int t = 0; t < kPanelNB; ++t) x[t] = (row && t < nb) ? Fr[(int64_t)t * f] : T(0);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int idx = u * nt + tid;
        if (idx < nb * nb) D[idx % nb + (idx / nb) * kPanelLd] = t4[u];
    }
    __syncthreads();
    if (tid < kWave) potrf32_reg<T>(D, nb, c0 + kb, blockIdx.x == 0 ? status : nullptr, s_rdiag);
    __syncthreads();
    if (blockIdx.x == 0) {
        T* dst = gridDim.x == 1 ? F + kb + (int64_t)kb * f : dscr + (size_t)blockIdx.y * kPanelNB * kPanelNB;
        const int64_t ld = gridDim.x == 1 ? f : kPanelNB;
        for (int idx = tid; idx < nb * nb; idx += nt) {
            const int i = idx % nb, j = idx / nb;
            if (i >= j) dst[i + j * ld] = D[i + j * kPanelLd];
        }
    }
    if (!row) return;
#pragma unroll
    for (int j = 0; j < kPanelNB; ++j) {
        if (j < nb) {
            x[j] *= s_rdiag[j];
#pragma unroll
            for (int k = j + 1; k < kPanelNB; ++k)
                if (k < nb) x[k] = fma(-x[j], D[k + j * kPanelLd], x[k]);
        }
    }
#pragma unroll
    for (int t = 0; t < kPanelNB; ++t)
        if (t < nb) Fr[(int64_t)t * f] = x[t];
}

// Large fronts, step 2 in FP64: the diagonal Cholesky and the row solves
// in one right-looking pass.  In every wave, lanes 0..31 hold the rows of
// the 32 x 32 diagonal block (padded with an identity when narrower: unit
// pivots, zero multipliers) and lanes 32..63 hold 32 rows below it; per
// column j the pivot comes from lane j and every lane scales its entry j by
// the pivot's reciprocal and subtracts l_ij l_kj from its entries k > j, so
// that a row below the block is solved by exactly the steps that factor the
// block's own rows.  Each wave factors the block itself (no LDS staging, no
// barrier before the solves).  The columns are one basic block: pivots by
// select (a failed pivot is recorded after the loop exactly as pivot_root
// records it), every lane stores its column entry to the wave's LDS slice
// (kPanelLd x kPanelNB doubles; lanes 32..63 land in the padding), the next
// column's entry takes its multiplier by a lane read and the others take
// theirs one column late from LDS (loaded while the next pivot is
// computed), and a scheduling barrier per column keeps each column's
// updates in that column (left to the scheduler they sink to the next
// pivot and put a chain of up to 31 dependent FMAs in front of it).  Every
// entry sees the operations of a column-by-column Cholesky of the block and
// a forward substitution of each row against it, in the same order.  Grid
// (row chunk of kFusedPanelRows rows, front), 256 threads.  With one chunk
// the factored block is written back in place (after a barrier: every wave
// has read it); with several, chunk 0 leaves it in dscr and the
// trailing-update launch copies it into the front.
__global__ void __launch_bounds__(256)
k_big_panel_fused(DevPlan P, BigOne one, double* __restrict__ arena, int list_begin, int kb, int32_t* status,
                  double* __restrict__ dscr) {
    constexpr int NB = kPanelNB;
    static_assert(2 * NB == kWave && kFusedPanelRows == 4 * NB, "block rows and chunk rows share each wave");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    int c0, w, f;
    int64_t loff;
    if (one.loff >= 0) {
        c0 = one.c0, w = one.w, f = one.f, loff = one.loff;
    } else {
        const int s = P.lvl_big[list_begin + blockIdx.y];
        c0 = P.sn_start[s], w = P.sn_start[s + 1] - c0;
        f = P.sn_rowptr[s + 1] - P.sn_rowptr[s], loff = P.l_off[s];
    }
    if (kb >= w) return;  // workgroup-uniform
    const int nb = min(NB, w - kb);
    double* F = arena + loff;
    const int tid = threadIdx.x, lane = tid % kWave, wid = tid / kWave;
    const int r0 = kb + nb + blockIdx.x * kFusedPanelRows;
    if (blockIdx.x > 0 && r0 >= f) return;  // workgroup-uniform
    const bool blk = lane < NB;              // a row of the diagonal block
    const int rr = r0 + wid * NB + (lane - NB);  // (lanes 32..63) row of the front
    const bool row = !blk && rr < f;
    // the lane's row, from clamped addresses (every load in bounds, no
    // branches between the loads).  The block's padding is selected to an
    // exact identity (its pivots are reported); a row's entries past nb,
    // and the entries of lanes without a row, keep whatever they loaded:
    // they only ever reach entries that are not stored.
    const int ri = blk ? kb + (lane < nb ? lane : 0) : (row ? rr : kb);
    double* Fl = F + ri + (int64_t)kb * f;
    double a[NB];
#pragma unroll
    for (int t = 0; t < NB; ++t) {
        const int tc = (t < nb && (!blk || t <= lane)) ? t : 0;
        a[t] = Fl[(int64_t)tc * f];
    }
#pragma unroll
    for (int t = 0; t < NB; ++t)
        if (blk) a[t] = (lane < nb && t <= lane) ? a[t] : (lane == t ? 1.0 : 0.0);
    double* Dx = reinterpret_cast<double*>(smem_raw) + wid * (kPanelLd * NB);
    double m[NB];
    double lprev = 0.0, dn = 0.0;
#pragma unroll
    for (int t = 0; t < NB; ++t) m[t] = 0.0;
    int first_bad = INT_MAX;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        double r;
        bool fail;
        const double ljj = pivot_select<double>(bcast<double>(j == 0 ? a[0] : dn, j), r, fail);
        if (j >= 1) {
#pragma unroll
            for (int k = j + 1; k < NB; ++k) a[k] = fma(-lprev, m[k], a[k]);
        }
        first_bad = (fail && first_bad == INT_MAX) ? j : first_bad;
        const double lij = lane == j ? ljj : a[j] * r;
        Dx[lane + j * kPanelLd] = lij;  // (lanes 32..63 land in the slice's padding)
        a[j] = lij;
        if (j + 1 < NB) {
            // the next pivot's entry, formed in its own lane (its multiplier
            // is its own l_ij: the same value as the broadcast, one lane
            // read shorter on the pivot chain)
            dn = fma(-lij, lij, a[j + 1]);
            a[j + 1] = fma(-lij, bcast<double>(lij, j + 1), a[j + 1]);
        }
#pragma unroll
        for (int k = j + 2; k < NB; ++k) m[k] = Dx[k + j * kPanelLd];
        lprev = lij;
        __builtin_amdgcn_sched_barrier(0);
    }
    // every wave has consumed its loads of the block before it is
    // overwritten in place
    __syncthreads();
    const int tn = opaque(nb);  // (kept out of the column loop's registers)
    if (blk) {
        if (blockIdx.x != 0 || wid != 0) return;
        if (status && lane == 0 && first_bad != INT_MAX) atomicMin(status, c0 + kb + first_bad);
        double* dst = gridDim.x == 1 ? F + kb + (int64_t)kb * f : dscr + (size_t)blockIdx.y * NB * NB;
        const int64_t ld = gridDim.x == 1 ? f : NB;
#pragma unroll
        for (int j = 0; j < NB; ++j)
            if (j < tn && j <= lane && lane < tn) dst[lane + j * ld] = a[j];
        return;
    }
    if (!row) return;
    if (nb == NB) {
#pragma unroll
        for (int t = 0; t < NB; ++t) Fl[(int64_t)t * f] = a[t];
    } else {
#pragma unroll
        for (int t = 0; t < NB; ++t)
            if (t < tn) Fl[(int64_t)t * f] = a[t];
    }
}

// Large fronts, step 3: trailing update C -= P P^T of the lower triangle
// below the panel, one 64 x 64 tile per workgroup (grid: tile row, tile
// column, front); only columns below col_end are updated (the rest of a
// wide panel when the trailing part gets one wide update later).
template <typename T, int PW>
__global__ void __launch_bounds__(256)
k_big_update(DevPlan P, BigOne one, T* __restrict__ arena, int list_begin, int kb, const T* __restrict__ dscr,
             int copy_d, int col_end) {
    int w, f;
    int64_t loff;
    if (one.loff >= 0) {
        w = one.w, f = one.f, loff = one.loff;
    } else {
        const int s = P.lvl_big[list_begin + blockIdx.z];
        w = P.sn_start[s + 1] - P.sn_start[s], f = P.sn_rowptr[s + 1] - P.sn_rowptr[s], loff = P.l_off[s];
    }
    if (kb >= w) return;
    if (copy_d && blockIdx.x == 0 && blockIdx.y == 0) {
        // the factored diagonal block left by a multi-chunk panel launch
        const int nb = min(PW, w - kb);
        const T* src = dscr + (size_t)blockIdx.z * PW * PW;
        T* F = arena + loff;
        for (int idx = threadIdx.x; idx < nb * nb; idx += blockDim.x) {
            const int i = idx % nb, j = idx / nb;
            if (i >= j) F[(kb + i) + (int64_t)(kb + j) * f] = src[i + j * PW];
        }
    }
    const int ti = blockIdx.x, tj = blockIdx.y;
    if (tj > ti) return;
    const int nb = min(PW, w - kb);
    const int base = kb + nb;
    const int i0 = base + ti * 64, j0 = base + tj * 64;
    if (i0 >= f || j0 >= col_end) return;
    T* F = arena + loff;
    const int tid = threadIdx.x;
    const int cmax = min(f, col_end);
    using M = Mfma<T>;
    const int lane = tid % kWave, wv = tid / kWave;
    const int qi = wv % 2, qj = wv / 2;
    const int li = lane % 16, lk = lane / 16;
    const bool quad = !(ti == tj && qj > qi);  // quadrant on or below the diagonal (wave-uniform)
    // the tile's old values, loaded first so that their latency overlaps the
    // panel loads and the matrix-core steps
    T old[2][2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = i0 + qi * 32 + a * 16 + M::row(r, lk), col = j0 + qj * 32 + b * 16 + li;
                old[a][b][r] = (quad && row < f && col < cmax && row >= col) ? F[row + (int64_t)col * f] : T(0);
            }
    // four waves, one 32 x 32 quadrant each, 2 x 2 MFMA tiles of 16 x 16:
    // each wave loads its own operands of every step straight from the
    // front (the rows of its quadrant, four panel columns per step), all
    // issued before the first matrix-core step
    if (!quad) return;  // quadrant above the diagonal (wave-uniform)
    {
        constexpr int kSteps = PW / 4;
        T av[kSteps][2], bv[kSteps][2];
#pragma unroll
        for (int u = 0; u < kSteps; ++u) {
            const int t = 4 * u + lk;
            const int64_t col = (int64_t)(kb + (t < nb ? t : 0)) * f;
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const int gi = i0 + qi * 32 + a * 16 + li;
                av[u][a] = (gi < f && t < nb) ? F[gi + col] : T(0);
            }
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int gj = j0 + qj * 32 + b * 16 + li;
                bv[u][b] = (gj < f && t < nb) ? F[gj + col] : T(0);
            }
        }
        typename M::acc c[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) c[a][b] = M::zero();
#pragma unroll
        for (int u = 0; u < kSteps; ++u) {
            if (4 * u < nb) {
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b) c[a][b] = M::step(av[u][a], bv[u][b], c[a][b]);
            }
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = i0 + qi * 32 + a * 16 + M::row(r, lk), col = j0 + qj * 32 + b * 16 + li;
                    if (row < f && col < cmax && row >= col) F[row + (int64_t)col * f] = old[a][b][r] - c[a][b][r];
                }
    }
}

// Large fronts, wide trailing update: C -= P P^T on the lower triangle
// of the columns from kb + kWideRank on, P the (up to) kWideRank factored
// columns from kb (rank-kWideRank instead of rank-kPanelNB updates, so the
// trailing matrix is read and written a quarter as often).  One 64 x 64
// tile per workgroup of four waves, each a 32 x 32 quadrant of 16 x 16
// matrix-core tiles (v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32).  P's rows come through LDS in 32-column
// chunks stored column by column (the sixteen lanes that read one MFMA
// operand column touch sixteen consecutive doubles), the next chunk's loads
// in flight during the current chunk's MFMAs; the tile's old values are
// loaded first.  The lower-triangle tiles of a front are numbered column by
// column and a launch takes the tiles [lin0, lin1) (a run of whole tile
// columns).  Grid (lin1 - lin0, front), 256 threads.
template <typename T>
__global__ void __launch_bounds__(256)
k_big_update_wide(DevPlan P, T* __restrict__ arena, int list_begin, int kb, int nt, int lin0, int lin1) {
    using M = Mfma<T>;
    constexpr int kT = kWideTile, kThreads = 256, kMA = 2, KC = kPanelNB;
    __shared__ T A[KC][kT];
    __shared__ T B[KC][kT];
    const int s = P.lvl_big[list_begin + blockIdx.y];
    const int w = P.sn_start[s + 1] - P.sn_start[s];
    const int f = P.sn_rowptr[s + 1] - P.sn_rowptr[s];
    if (kb >= w) return;
    // lower-triangle tiles of a front with nt tile rows, column by column:
    // column tj holds tiles (tj .. nt - 1, tj) and starts at
    // S(tj) = tj nt - tj (tj - 1) / 2
    const int lin = lin0 + blockIdx.x;
    if (lin >= lin1) return;
    auto col_start = [&](int c) { return c * nt - c * (c - 1) / 2; };
    const double q = 2.0 * nt + 1.0;
    int tj = (int)((q - sqrt(q * q - 8.0 * lin)) * 0.5);
    tj = max(0, min(tj, nt - 1));
    while (tj > 0 && col_start(tj) > lin) --tj;
    while (tj + 1 < nt && col_start(tj + 1) <= lin) ++tj;
    const int ti = tj + (lin - col_start(tj));
    const int base = kb + kWideRank;
    const int i0 = base + ti * kT, j0 = base + tj * kT;
    if (i0 >= f) return;
    T* F = arena + P.l_off[s];
    const int rank = min(kWideRank, w - kb);
    const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
    const int qi = wv % 2, qj = wv / 2;  // rows qi * TILE / 2, columns qj * 32 of the tile
    const bool idle = ti == tj && qj * 32 >= (qi + 1) * (kT / 2);  // block above the diagonal (wave-uniform)
    const int li = lane % 16, lk = lane / 16;
    // the tile's old values, loaded first so that their latency overlaps
    // the MFMAs
    T cv[kMA][2][4];
#pragma unroll
    for (int a = 0; a < kMA; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = i0 + qi * (kT / 2) + a * 16 + M::row(r, lk), col = j0 + qj * 32 + b * 16 + li;
                cv[a][b][r] = (!idle && row < f && col < f && row >= col) ? F[row + (int64_t)col * f] : T(0);
            }
    constexpr int kPer = kT * KC / kThreads;
    T ta[kPer], tb[kPer];
    auto load_chunk = [&](int t0) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int idx = u * kThreads + tid;
            const int ii = idx % kT, t = idx / kT;
            const int gi = i0 + ii, gj = j0 + ii;
            const bool tin = t0 + t < rank;
            ta[u] = (gi < f && tin) ? F[gi + (int64_t)(kb + t0 + t) * f] : T(0);
            tb[u] = (gj < f && tin) ? F[gj + (int64_t)(kb + t0 + t) * f] : T(0);
        }
    };
    load_chunk(0);
    typename M::acc c[kMA][2];
#pragma unroll
    for (int a = 0; a < kMA; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) c[a][b] = M::zero();
    for (int t0 = 0; t0 < rank; t0 += KC) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int idx = u * kThreads + tid;
            A[idx / kT][idx % kT] = ta[u];
            B[idx / kT][idx % kT] = tb[u];
        }
        __syncthreads();
        if (t0 + KC < rank) load_chunk(t0 + KC);
        const int kc = min(KC, rank - t0);
        if (!idle) {
            for (int t = 0; t < kc; t += 4) {
                T av[kMA], bv[2];
#pragma unroll
                for (int a = 0; a < kMA; ++a) av[a] = A[t + lk][qi * (kT / 2) + a * 16 + li];
#pragma unroll
                for (int b = 0; b < 2; ++b) bv[b] = B[t + lk][qj * 32 + b * 16 + li];
#pragma unroll
                for (int a = 0; a < kMA; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
                        c[a][b] = M::step(av[a], bv[b], c[a][b]);
            }
        }
        __syncthreads();
    }
    if (idle) return;
#pragma unroll
    for (int a = 0; a < kMA; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = i0 + qi * (kT / 2) + a * 16 + M::row(r, lk), col = j0 + qj * 32 + b * 16 + li;
                if (row < f && col < f && row >= col) F[row + (int64_t)col * f] = cv[a][b][r] - c[a][b][r];
            }
}

// ---------------------------------------------------------------- sweeps

// Wave-uniform broadcast of lane k's value (k must be the same in every lane).
__device__ __forceinline__ double lane_bcast(double x, int k) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), k);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), k);
    return __hiloint2double(hi, lo);
}

// Completion flags of the dependency-driven sweeps.  A producer makes its
// stores visible at device scope before raising its flag; a consumer that
// saw the flag orders its later loads after it.
__device__ __forceinline__ unsigned flag_load(const unsigned* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void flag_store(unsigned* p, unsigned v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void release_device() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ __forceinline__ void acquire_device() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

// Bounded wait for *flag == want.  Gives up after `ticks` of the constant
// wall clock, or as soon as another wait has given up, and then records
// the failure in *err; the caller carries on, so every wave still exits.
__device__ void wait_flag(const unsigned* flag, unsigned want, int32_t* err, unsigned long long ticks) {
    if (flag_load(flag) == want) return;
    const unsigned long long t0 = wall_clock64();
    for (;;) {
        __builtin_amdgcn_s_sleep(1);
        if (flag_load(flag) == want) return;
        if (wall_clock64() - t0 > ticks || flag_load(reinterpret_cast<unsigned*>(err)) != 0u) {
            flag_store(reinterpret_cast<unsigned*>(err), 1u);
            return;
        }
    }
}

// Stage the nb x nb lower triangle of the diagonal block at src (leading
// dimension f) into D[r + c * ldd] (ldd odd,
// sweep_diag_ld: the backward solves read a row of D across the lanes, and
// an odd stride spreads it over the LDS banks); eight loads per
// thread are issued before their LDS stores so that their latencies overlap.
template <typename T>
__device__ __forceinline__ void stage_diag_block(const T* __restrict__ src, int f, int nb, double* D, int ldd) {
    const int tid = threadIdx.x, nt = blockDim.x, tot = nb * nb;
    for (int base = 0; base < tot; base += 8 * nt) {
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = base + u * nt + tid;
            const int i = idx % nb, k = idx / nb;
            t[u] = (idx < tot && i >= k) ? (double)src[i + (int64_t)k * f] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = base + u * nt + tid;
            if (idx < tot) {
                const int i = idx % nb, k = idx / nb;
                D[i + k * ldd] = t[u];
            }
        }
    }
}

// Triangular solves of a staged diagonal block by one wave (D: the block's
// lower triangle, leading dimension ldd, raw pivots on the diagonal; lane
// r < nb holds entry r, lanes from nb on keep their value).  Each lane of
// the block carries its value scaled by its reciprocal pivot, so that lane
// k's value is the k-th unknown once the earlier steps are applied, and
// takes step k as s -= (d / pivot) x_k with its multiplier zero unless it
// is updated by step k: one broadcast and one fma per step on the
// dependency chain.  The entries of D are read eight steps ahead.
__device__ __forceinline__ double wave_fwd_tri(double vi, const double* D, int ldd, int nb) {
    const int lane = threadIdx.x % kWave, lr = lane < nb ? lane : 0;
    const bool own = lane < nb;
    const double rdl = 1.0 / D[lr + lr * ldd];
    double sv = own ? vi * rdl : vi;
    int k = 0;
    for (; k + 8 <= nb; k += 8) {
        double dk[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) dk[u] = D[lr + (k + u) * ldd];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double m = (own && lane > k + u) ? dk[u] * rdl : 0.0;
            sv = fma(-m, lane_bcast(sv, k + u), sv);
        }
    }
    for (; k < nb; ++k) {
        const double m = (own && lane > k) ? D[lr + k * ldd] * rdl : 0.0;
        sv = fma(-m, lane_bcast(sv, k), sv);
    }
    return sv;
}
__device__ __forceinline__ double wave_bwd_tri(double ri, const double* D, int ldd, int nb) {
    const int lane = threadIdx.x % kWave, lr = lane < nb ? lane : 0;
    const bool own = lane < nb;
    const double rdl = 1.0 / D[lr + lr * ldd];
    double sv = own ? ri * rdl : ri;
    int k = nb - 1;
    for (; k >= 7; k -= 8) {
        double dk[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) dk[u] = D[(k - u) + lr * ldd];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double m = (own && lane < k - u) ? dk[u] * rdl : 0.0;
            sv = fma(-m, lane_bcast(sv, k - u), sv);
        }
    }
    for (; k >= 0; --k) {
        const double m = (own && lane < k) ? D[k + lr * ldd] * rdl : 0.0;
        sv = fma(-m, lane_bcast(sv, k), sv);
    }
    return sv;
}

// Forward sweep of one supernode by a workgroup: v (LDS, f entries) holds
// the gathered right-hand side on entry; per block of 64 columns one wave
// solves the diagonal block (staged in LDS with reciprocal pivots) with
// lane broadcasts and the workgroup applies the block to every row below
// it (one thread per row, loads in batches of 16).  Rows beyond the
// supernode's own columns end up holding this front's update vector.
template <typename T>
__device__ void fwd_front(const T* __restrict__ L, int w, int f, int ldd, double* v, double* D,
                          bool first_staged = false) {
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid % kWave, wid = tid / kWave;
    for (int kb = 0; kb < w; kb += kWave) {
        const int nb = min(kWave, w - kb);
        if (kb > 0 || !first_staged) stage_diag_block(L + kb + (int64_t)kb * f, f, nb, D, ldd);
        __syncthreads();
        if (wid == 0) {
            const double vi = wave_fwd_tri(lane < nb ? v[kb + lane] : 0.0, D, ldd, nb);
            if (lane < nb) v[kb + lane] = vi;
        }
        __syncthreads();
        for (int i = kb + nb + tid; i < f; i += nt) {
            const T* Li = L + i + (int64_t)kb * f;
            double acc = 0.0;
            int k = 0;
            for (; k + 32 <= nb; k += 32) {
                // 32 loads in flight, then their products in column order
                T l[32];
#pragma unroll
                for (int u = 0; u < 32; ++u) l[u] = Li[(int64_t)(k + u) * f];
#pragma unroll
                for (int u = 0; u < 32; ++u) acc = fma((double)l[u], v[kb + k + u], acc);
            }
            for (; k < nb; ++k) acc = fma((double)Li[(int64_t)k * f], v[kb + k], acc);
            v[i] -= acc;
        }
        __syncthreads();
    }
}

// The nb x nb lower triangle of the diagonal block at src (leading
// dimension f) in registers: entry idx = tid + u nt (row idx % nb, column
// idx / nb) for u < kDiagRegs; store_diag_regs writes them to
// D[r + c * ldd] and stages any entries beyond
// kDiagRegs * nt directly (fewer than 256 threads).  Together they are
// stage_diag_block with the loads issued earlier.
constexpr int kDiagRegs = 16;
template <typename T>
__device__ __forceinline__ void load_diag_regs(T (&d)[kDiagRegs], const T* __restrict__ src, int f, int nb) {
    const int tid = threadIdx.x, nt = blockDim.x, tot = nb * nb;
#pragma unroll
    for (int u = 0; u < kDiagRegs; ++u) {
        const int idx = u * nt + tid, i = idx % nb, k = idx / nb;
        d[u] = (idx < tot && i >= k) ? src[i + (int64_t)k * f] : T(0);
    }
}
template <typename T>
__device__ __forceinline__ void store_diag_regs(const T (&d)[kDiagRegs], const T* __restrict__ src, int f, int nb,
                                                double* D, int ldd) {
    const int tid = threadIdx.x, nt = blockDim.x, tot = nb * nb;
#pragma unroll
    for (int u = 0; u < kDiagRegs; ++u) {
        const int idx = u * nt + tid, i = idx % nb, k = idx / nb;
        if (idx < tot) D[i + k * ldd] = (double)d[u];
    }
    for (int idx = kDiagRegs * nt + tid; idx < tot; idx += nt) {
        const int i = idx % nb, k = idx / nb;
        D[i + k * ldd] = i >= k ? (double)src[i + (int64_t)k * f] : 0.0;
    }
}

// Backward sweep of one supernode by a workgroup: z (LDS, f entries) holds
// y on the own columns and the solved x on the rows below; per block of 64
// columns (last block first) the entries of the diagonal block are loaded
// into registers (unless the caller staged the last block in D:
// last_staged), each wave forms the dot products of its columns (two
// groups of eight at a time) with everything solved so far, the block is
// stored to D and one wave back-substitutes it.
template <typename T>
__device__ void bwd_front(const T* __restrict__ L, int w, int f, int ldd, double* z, double* D, double* tb,
                          bool last_staged = false) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int nw = nt / kWave, lane = tid % kWave, wid = tid / kWave;
    const int nblk = (w + kWave - 1) / kWave;
    T dreg[kDiagRegs];
    for (int b = nblk - 1; b >= 0; --b) {
        const int kb = b * kWave, nb = min(kWave, w - kb), r0 = kb + nb;
        const T* Lb = L + kb + (int64_t)kb * f;
        const bool staged = b == nblk - 1 && last_staged;
        if (!staged) load_diag_regs(dreg, Lb, f, nb);
        for (int k0 = wid * 8; k0 < nb; k0 += 2 * nw * 8) {
            // column groups k0 and k1 = k0 + 8 nw (when below nb); each
            // lane sums its rows r0 + lane + 64 m in row order, four rows of
            // both groups per step (64 loads in flight)
            const int k1 = k0 + nw * 8;
            const bool g1 = k1 < nb;
            double pa[8], pb[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) pa[c] = pb[c] = 0.0;
            int i = r0 + lane;
            for (; i + 3 * kWave < f; i += 4 * kWave) {
                double zm[4];
                T la[4][8], lb[4][8];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    zm[m] = z[i + m * kWave];
#pragma unroll
                    for (int c = 0; c < 8; ++c) {
                        la[m][c] = (k0 + c < nb) ? L[i + m * kWave + (int64_t)(kb + k0 + c) * f] : T(0);
                        lb[m][c] = (g1 && k1 + c < nb) ? L[i + m * kWave + (int64_t)(kb + k1 + c) * f] : T(0);
                    }
                }
#pragma unroll
                for (int m = 0; m < 4; ++m)
#pragma unroll
                    for (int c = 0; c < 8; ++c) {
                        pa[c] = fma((double)la[m][c], zm[m], pa[c]);
                        pb[c] = fma((double)lb[m][c], zm[m], pb[c]);
                    }
            }
            for (; i < f; i += kWave) {
                const double zi = z[i];
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    pa[c] = fma((k0 + c < nb) ? (double)L[i + (int64_t)(kb + k0 + c) * f] : 0.0, zi, pa[c]);
                    pb[c] = fma((g1 && k1 + c < nb) ? (double)L[i + (int64_t)(kb + k1 + c) * f] : 0.0, zi, pb[c]);
                }
            }
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const double sa = wave_sum(pa[c]);
                if (lane == 0 && k0 + c < nb) tb[k0 + c] = sa;
            }
            if (g1) {
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const double sb = wave_sum(pb[c]);
                    if (lane == 0 && k1 + c < nb) tb[k1 + c] = sb;
                }
            }
        }
        if (!staged) store_diag_regs(dreg, Lb, f, nb, D, ldd);
        __syncthreads();
        if (wid == 0) {
            const double ri = wave_bwd_tri(lane < nb ? z[kb + lane] - tb[lane] : 0.0, D, ldd, nb);
            if (lane < nb) z[kb + lane] = ri;
        }
        __syncthreads();
    }
}

// Level-synchronous forward sweep: one workgroup per supernode of a level.
template <typename T>
__global__ void __launch_bounds__(256)
k_fwd(DevPlan P, const T* __restrict__ arena, int list_begin, int ldd, int skip_f, double* __restrict__ v_perm,
      double* __restrict__ uvec) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* v = reinterpret_cast<double*>(smem_raw);
    const int s = P.lvl_all[list_begin + blockIdx.x];
    const int c0 = P.sn_start[s], w = P.sn_start[s + 1] - c0;
    const int ro = P.sn_rowptr[s], f = P.sn_rowptr[s + 1] - ro;
    if (f >= skip_f) return;  // swept by the tiled kernels
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int i = tid; i < f; i += nt) {
        double acc = (i < w) ? v_perm[c0 + i] : 0.0;
        const int q1 = P.cb_ptr[ro + i + 1];
        for (int q = P.cb_ptr[ro + i]; q < q1; ++q) acc += uvec[P.cb_src[q]];
        v[i] = acc;
    }
    __syncthreads();
    fwd_front(arena + P.l_off[s], w, f, ldd, v, v + ((f + 1) & ~1));
    for (int i = tid; i < f; i += nt) {
        if (i < w) v_perm[c0 + i] = v[i];
        else uvec[ro + i] = v[i];
    }
}

// Level-synchronous backward sweep (levels root to leaves).
template <typename T>
__global__ void __launch_bounds__(256)
k_bwd(DevPlan P, const T* __restrict__ arena, int list_begin, int ldd, int skip_f, double* __restrict__ x_perm) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* z = reinterpret_cast<double*>(smem_raw);
    __shared__ double tb[kWave];
    const int s = P.lvl_all[list_begin + blockIdx.x];
    const int c0 = P.sn_start[s], w = P.sn_start[s + 1] - c0;
    const int ro = P.sn_rowptr[s], f = P.sn_rowptr[s + 1] - ro;
    if (f >= skip_f) return;  // swept by the tiled kernels
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int i = tid; i < f; i += nt) z[i] = x_perm[P.sn_rows[ro + i]];
    __syncthreads();
    bwd_front(arena + P.l_off[s], w, f, ldd, z, z + ((f + 1) & ~1), tb);
    for (int i = tid; i < w; i += nt) x_perm[c0 + i] = z[i];
}

// ---------------------------------------------------------------- tiled sweeps of large fronts
//
// A front with at least kSweepTiledFront rows (the default size) is swept
// by many workgroups, one launch per 64-column block of its panel, instead
// of by one workgroup.
// Between launches the front vector lives in global memory: entry i is
// v_perm[c0 + i] for the own columns (i < w) and this front's update slot
// uvec[ro + i] below them, so no flags are needed (launch order on the
// stream orders the blocks).  Every sum runs in a fixed order.

// Forward gather: entry i = own right-hand side (i < w) plus the children's
// contributions, written to its global slot.  Grid (row tiles, big list).
__global__ void __launch_bounds__(256)
k_fwd_tiled_gather(DevPlan P, int list_begin, int min_f, double* __restrict__ v_perm, double* __restrict__ uvec) {
    const int s = P.lvl_big[list_begin + blockIdx.y];
    const int c0 = P.sn_start[s], w = P.sn_start[s + 1] - c0;
    const int ro = P.sn_rowptr[s], f = P.sn_rowptr[s + 1] - ro;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (f < min_f || i >= f) return;
    double acc = (i < w) ? v_perm[c0 + i] : 0.0;
    const int q1 = P.cb_ptr[ro + i + 1];
    for (int q = P.cb_ptr[ro + i]; q < q1; ++q) acc += uvec[P.cb_src[q]];
    if (i < w) v_perm[c0 + i] = acc;
    else uvec[ro + i] = acc;
}

// Forward step j of the tiled fronts (j = 0 .. number of column blocks):
// each workgroup takes 64 rows from row min(64 j, w) on, subtracts the
// contribution of block j - 1 (already solved; its four waves take 16 of
// its columns each and their partial sums are added in wave order), and
// the first workgroup then solves diagonal block j on its rows.  Grid
// (row tiles, big list), 256 threads.
template <typename T>
__global__ void __launch_bounds__(256)
k_fwd_tiled_step(DevPlan P, const T* __restrict__ arena, int list_begin, int min_f, int j,
                 double* __restrict__ v_perm, double* __restrict__ uvec) {
    __shared__ double D[kWave * kWave];
    __shared__ double yb[kWave];
    __shared__ double red[4][kWave];
    const int s = P.lvl_big[list_begin + blockIdx.y];
    const int c0 = P.sn_start[s], w = P.sn_start[s + 1] - c0;
    const int ro = P.sn_rowptr[s], f = P.sn_rowptr[s + 1] - ro;
    const int nblk = (w + kWave - 1) / kWave;
    if (f < min_f || j > nblk) return;
    const int r0 = min(j * kWave, w) + blockIdx.x * kWave;
    if (r0 >= f) return;
    const T* L = arena + P.l_off[s];
    const int tid = threadIdx.x, lane = tid % kWave, wid = tid / kWave;
    const bool solve = blockIdx.x == 0 && j < nblk;
    const int kb = j * kWave, nb = min(kWave, w - kb);
    const int pk = (j - 1) * kWave, pnb = j > 0 ? min(kWave, w - pk) : 0;
    if (solve) stage_diag_block(L + kb + (int64_t)kb * f, f, nb, D, kWave);
    if (tid < pnb) yb[tid] = v_perm[c0 + pk + tid];
    __syncthreads();
    const int i = r0 + lane;
    const bool row = i < f;
    double acc = 0.0;
    if (pnb > 0) {
        const int k0 = wid * 16;
        const T* Li = L + (row ? i : r0) + (int64_t)(pk + k0) * f;
        double l[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) l[u] = (row && k0 + u < pnb) ? (double)Li[(int64_t)u * f] : 0.0;
#pragma unroll
        for (int u = 0; u < 16; ++u) acc = fma(l[u], (k0 + u < pnb) ? yb[k0 + u] : 0.0, acc);
    }
    red[wid][lane] = acc;
    __syncthreads();
    if (wid != 0) return;
    double vi = 0.0;
    if (row) vi = ((i < w) ? v_perm[c0 + i] : uvec[ro + i]) - (((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane]);
    if (solve) vi = wave_fwd_tri(vi, D, kWave, nb);
    if (row) {
        if (i < w) v_perm[c0 + i] = vi;
        else uvec[ro + i] = vi;
    }
}

// Backward, part below the diagonal blocks: for every own column c of a
// tiled front, x_perm[c0 + c] -= sum over rows i >= w of L[i, c] x_i (the
// rows below are ancestors' columns, already solved).  One workgroup per
// eight columns; its four waves split the rows and their sums are added in
// wave order.  Grid (column groups, big list).
template <typename T>
__global__ void __launch_bounds__(256)
k_bwd_tiled_rect(DevPlan P, const T* __restrict__ arena, int list_begin, int min_f, double* __restrict__ x_perm) {
    __shared__ double red[4][8];
    const int s = P.lvl_big[list_begin + blockIdx.y];
    const int c0 = P.sn_start[s], w = P.sn_start[s + 1] - c0;
    const int ro = P.sn_rowptr[s], f = P.sn_rowptr[s + 1] - ro;
    const int cb = blockIdx.x * 8;
    if (f < min_f || f == w || cb >= w) return;
    const int nc = min(8, w - cb);
    const T* L = arena + P.l_off[s] + (int64_t)cb * f;
    const int tid = threadIdx.x, lane = tid % kWave, wid = tid / kWave;
    double part[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) part[c] = 0.0;
    for (int i0 = w + wid * kWave; i0 < f; i0 += 8 * kWave) {
        const int ia = i0 + lane, ib = i0 + 4 * kWave + lane;
        const bool va = ia < f, vb = ib < f;
        const int ra = va ? P.sn_rows[ro + ia] : 0, rb = vb ? P.sn_rows[ro + ib] : 0;
        double la[8], lb[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            la[c] = (va && c < nc) ? (double)L[ia + (int64_t)c * f] : 0.0;
            lb[c] = (vb && c < nc) ? (double)L[ib + (int64_t)c * f] : 0.0;
        }
        const double xa = va ? x_perm[ra] : 0.0, xb = vb ? x_perm[rb] : 0.0;
#pragma unroll
        for (int c = 0; c < 8; ++c) part[c] = fma(lb[c], xb, fma(la[c], xa, part[c]));
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const double sc = wave_sum(part[c]);
        if (lane == 0) red[wid][c] = sc;
    }
    __syncthreads();
    if (tid < nc) x_perm[c0 + cb + tid] -= ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
}

// Backward step b of the tiled fronts (b = last column block .. 0): the
// workgroup of column tile t <= b subtracts from its 64 columns the
// contribution of block b + 1 (solved by the previous step): lanes take
// the block's rows, the products go through LDS and four threads per
// column add 16 rows each, in a fixed order.  The workgroup of tile b
// then back-substitutes diagonal block b.  Grid (b + 1, big list).
template <typename T>
__global__ void __launch_bounds__(256)
k_bwd_tiled_step(DevPlan P, const T* __restrict__ arena, int list_begin, int min_f, int b,
                 double* __restrict__ x_perm) {
    __shared__ double D[kWave * (kWave + 1)];
    __shared__ double S[kWave * (kWave + 1)];
    __shared__ double tb[kWave];
    const int s = P.lvl_big[list_begin + blockIdx.y];
    const int c0 = P.sn_start[s], w = P.sn_start[s + 1] - c0;
    const int ro = P.sn_rowptr[s], f = P.sn_rowptr[s + 1] - ro;
    const int nblk = (w + kWave - 1) / kWave;
    const int t = blockIdx.x;
    if (f < min_f || b >= nblk || t > b) return;
    (void)ro;
    const T* L = arena + P.l_off[s];
    const int tid = threadIdx.x, lane = tid % kWave, wid = tid / kWave;
    const bool solve = t == b;
    const int kb = b * kWave, nb = min(kWave, w - kb);
    const int ct = t * kWave, tnb = min(kWave, w - ct);
    const int q = kb + kWave, qnb = b + 1 < nblk ? min(kWave, w - q) : 0;
    if (solve) stage_diag_block(L + kb + (int64_t)kb * f, f, nb, D, kWave + 1);
    if (qnb > 0) {
        const bool r = lane < qnb;
        const double xr = r ? x_perm[c0 + q + lane] : 0.0;
        const int k0 = wid * 16;
        const T* Lr = L + (r ? q + lane : q) + (int64_t)(ct + k0) * f;
        double l[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) l[u] = (r && k0 + u < tnb) ? (double)Lr[(int64_t)u * f] : 0.0;
#pragma unroll
        for (int u = 0; u < 16; ++u) S[(k0 + u) * (kWave + 1) + lane] = l[u] * xr;
        __syncthreads();
        const int c = tid >> 2, rq = tid & 3;
        double sum = 0.0;
#pragma unroll
        for (int u = 0; u < 16; ++u) sum += S[c * (kWave + 1) + rq * 16 + u];
        sum += __shfl_xor(sum, 1, kWave);
        sum += __shfl_xor(sum, 2, kWave);
        if (rq == 0) tb[c] = sum;
    } else if (tid < kWave) {
        tb[tid] = 0.0;
    }
    __syncthreads();
    if (wid != 0) return;
    double ri = lane < tnb ? x_perm[c0 + ct + lane] - tb[lane] : 0.0;
    if (solve) ri = wave_bwd_tri(ri, D, kWave + 1, nb);
    if (lane < tnb) x_perm[c0 + ct + lane] = ri;
}

// Forward step of one supernode with f <= 64 by one wave: lane i holds
// row i of the panel in registers (loaded before the gather, so the two
// overlap), gathers row i of the front, and one pass over the columns
// solves the diagonal block and forms the update vector (lane k broadcasts
// y_k, rows below subtract their multiple).
template <typename T, int MW>
__device__ __forceinline__ void fwd_wave_front(const DevPlan& P, const T* __restrict__ arena, int s,
                                               double* __restrict__ v_perm, double* __restrict__ uvec) {
    const int lane = threadIdx.x % kWave;
    const int c0 = P.sn_start[s], w = P.sn_start[s + 1] - c0;
    const int ro = P.sn_rowptr[s], f = P.sn_rowptr[s + 1] - ro;
    const T* L = arena + P.l_off[s];
    const bool act = lane < f;
    double lr[MW];
#pragma unroll
    for (int k = 0; k < MW; ++k) lr[k] = (k < w && act) ? (double)L[lane + (int64_t)k * f] : 0.0;
    const double rd = lane < w ? 1.0 / (double)L[lane + (int64_t)lane * f] : 0.0;
    double vi = 0.0;
    if (act) {
        vi = lane < w ? v_perm[c0 + lane] : 0.0;
        const int q1 = P.cb_ptr[ro + lane + 1];
        for (int q = P.cb_ptr[ro + lane]; q < q1; ++q) vi += uvec[P.cb_src[q]];
    }
#pragma unroll
    for (int k = 0; k < MW; ++k) {
        if (k < w) {
            const double yk = lane_bcast(vi, k) * lane_bcast(rd, k);
            if (lane == k) vi = yk;
            else if (lane > k) vi = fma(-lr[k], yk, vi);
        }
    }
    if (lane < w) v_perm[c0 + lane] = vi;
    else if (act) uvec[ro + lane] = vi;
}

// Backward step of one supernode with f <= 64 by one wave: lane j holds
// column j of the panel, forms the product with the solved rows below and
// back-substitutes the diagonal block with lane broadcasts.
template <typename T, int MF>
__device__ __forceinline__ void bwd_wave_front(const DevPlan& P, const T* __restrict__ arena, int s,
                                               double* __restrict__ x_perm) {
    const int lane = threadIdx.x % kWave;
    const int c0 = P.sn_start[s], w = P.sn_start[s + 1] - c0;
    const int ro = P.sn_rowptr[s], f = P.sn_rowptr[s + 1] - ro;
    const T* Lc = arena + P.l_off[s] + (int64_t)lane * f;
    const bool act = lane < f, own = lane < w;
    double lc[MF];
#pragma unroll
    for (int k = 0; k < MF; ++k) lc[k] = (k < f && own) ? (double)Lc[k] : 0.0;
    const double rd = own ? 1.0 / (double)Lc[lane] : 0.0;
    const double z = act ? x_perm[P.sn_rows[ro + lane]] : 0.0;
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < MF; ++k)
        if (k >= w && k < f) acc = fma(lc[k], lane_bcast(z, k), acc);
    double ri = own ? z - acc : 0.0;
#pragma unroll
    for (int k = MF - 1; k >= 0; --k) {
        if (k < w) {
            const double xk = lane_bcast(ri, k) * lane_bcast(rd, k);
            if (lane == k) ri = xk;
            else if (lane < k) ri = fma(-lc[k], xk, ri);
        }
    }
    if (own) x_perm[c0 + lane] = ri;
}

// Forward step of one supernode with f <= 128 and w <= 64 by two waves
// (threads 128 p .. 128 p + 127 of the workgroup, pair p): lane l of wave h
// holds row 64 h + l of the panel in registers and gathers that row of the
// front; wave 0 solves the diagonal block as fwd_wave_front does (its rows
// below take their updates in the same pass) and leaves the solution in
// y (LDS); wave 1 then applies it to rows 64 .. f - 1 in the same column
// order.  Every thread of the workgroup calls it (valid == false: no work,
// the barrier only).
template <typename T, int MW>
__device__ __forceinline__ void fwd_pair_front(const DevPlan& P, const T* __restrict__ arena, int s, bool valid,
                                               double* __restrict__ v_perm, double* __restrict__ uvec, double* y) {
    const int lane = threadIdx.x % kWave, h = (threadIdx.x / kWave) & 1;
    int c0 = 0, w = 0, ro = 0, f = 0;
    if (valid) {
        c0 = P.sn_start[s];
        w = P.sn_start[s + 1] - c0;
        ro = P.sn_rowptr[s];
        f = P.sn_rowptr[s + 1] - ro;
    }
    const int r = h * kWave + lane;
    const bool act = r < f;
    const T* L = arena + (valid ? P.l_off[s] : 0);
    double lr[MW];
#pragma unroll
    for (int k = 0; k < MW; ++k) lr[k] = (k < w && act) ? (double)L[r + (int64_t)k * f] : 0.0;
    const double rd = (h == 0 && lane < w) ? 1.0 / (double)L[lane + (int64_t)lane * f] : 0.0;
    double vi = 0.0;
    if (act) {
        vi = r < w ? v_perm[c0 + r] : 0.0;
        const int q1 = P.cb_ptr[ro + r + 1];
        for (int q = P.cb_ptr[ro + r]; q < q1; ++q) vi += uvec[P.cb_src[q]];
    }
    if (h == 0) {
#pragma unroll
        for (int k = 0; k < MW; ++k) {
            if (k < w) {
                const double yk = lane_bcast(vi, k) * lane_bcast(rd, k);
                if (lane == k) vi = yk;
                else if (lane > k) vi = fma(-lr[k], yk, vi);
            }
        }
        if (lane < w) y[lane] = vi;
    }
    __syncthreads();
    if (h == 1) {
#pragma unroll
        for (int k = 0; k < MW; ++k)
            if (k < w) vi = fma(-lr[k], y[k], vi);
    }
    if (r < w) v_perm[c0 + r] = vi;
    else if (act) uvec[ro + r] = vi;
}

// Backward step of one supernode with f <= 128 and w <= 64 by two waves:
// lane j of wave h holds rows 64 h .. 64 h + 63 of panel column j; wave 1
// forms its part of the product with the solved rows below (rows 64 and
// on) into part (LDS), wave 0 adds its own part (rows w .. 63) and
// back-substitutes the diagonal block with lane broadcasts.
template <typename T>
__device__ __forceinline__ void bwd_pair_front(const DevPlan& P, const T* __restrict__ arena, int s, bool valid,
                                               double* __restrict__ x_perm, double* part) {
    const int lane = threadIdx.x % kWave, h = (threadIdx.x / kWave) & 1;
    int c0 = 0, w = 0, ro = 0, f = 0;
    if (valid) {
        c0 = P.sn_start[s];
        w = P.sn_start[s + 1] - c0;
        ro = P.sn_rowptr[s];
        f = P.sn_rowptr[s + 1] - ro;
    }
    const int r0 = h * kWave;
    const bool own = lane < w;
    const T* Lc = arena + (valid ? P.l_off[s] : 0) + (int64_t)lane * f + r0;
    double lc[kWave];
#pragma unroll
    for (int k = 0; k < kWave; ++k) lc[k] = (own && r0 + k < f) ? (double)Lc[k] : 0.0;
    const double rd = (h == 0 && own) ? 1.0 / (double)Lc[lane] : 0.0;
    const int r = r0 + lane;
    const double z = r < f ? x_perm[P.sn_rows[ro + r]] : 0.0;
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < kWave; ++k)
        if (r0 + k >= w && r0 + k < f) acc = fma(lc[k], lane_bcast(z, k), acc);
    if (h == 1) part[lane] = acc;
    __syncthreads();
    if (h == 1 || !own) return;
    if (f > kWave) acc += part[lane];
    double ri = z - acc;
#pragma unroll
    for (int k = kWave - 1; k >= 0; --k) {
        if (k < w) {
            const double xk = lane_bcast(ri, k) * lane_bcast(rd, k);
            if (lane == k) ri = xk;
            else if (lane < k) ri = fma(-lc[k], xk, ri);
        }
    }
    x_perm[c0 + lane] = ri;
}

// Level-synchronous sweeps for levels whose fronts have order <= 128 and
// width <= 64 (the larger ones of the small-front levels): two supernodes
// per 256-thread workgroup, two waves each.
template <typename T, int MW>
__global__ void __launch_bounds__(256)
k_fwd_pairs(DevPlan P, const T* __restrict__ arena, int list_begin, int count, double* __restrict__ v_perm,
            double* __restrict__ uvec) {
    __shared__ double y[2][kWave];
    const int pr = threadIdx.x / (2 * kWave);
    const int t = blockIdx.x * 2 + pr;
    const bool valid = t < count;
    fwd_pair_front<T, MW>(P, arena, valid ? P.lvl_all[list_begin + t] : 0, valid, v_perm, uvec, y[pr]);
}

template <typename T>
__global__ void __launch_bounds__(256)
k_bwd_pairs(DevPlan P, const T* __restrict__ arena, int list_begin, int count, double* __restrict__ x_perm) {
    __shared__ double part[2][kWave];
    const int pr = threadIdx.x / (2 * kWave);
    const int t = blockIdx.x * 2 + pr;
    const bool valid = t < count;
    bwd_pair_front(P, arena, valid ? P.lvl_all[list_begin + t] : 0, valid, x_perm, part[pr]);
}

// Level-synchronous sweeps for levels whose fronts all have order <= 64:
// four supernodes per 256-thread workgroup, one per wave.
// MW (forward) bounds the level's supernode widths, MF (backward) its
// front orders: the panel row or column a lane holds is that many
// registers, so narrow levels keep more waves in flight.
template <typename T, int MW>
__global__ void __launch_bounds__(256)
k_fwd_waves(DevPlan P, const T* __restrict__ arena, int list_begin, int count, double* __restrict__ v_perm,
            double* __restrict__ uvec) {
    const int t = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (t >= count) return;
    fwd_wave_front<T, MW>(P, arena, P.lvl_all[list_begin + t], v_perm, uvec);
}

template <typename T, int MF>
__global__ void __launch_bounds__(256)
k_bwd_waves(DevPlan P, const T* __restrict__ arena, int list_begin, int count, double* __restrict__ x_perm) {
    const int t = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (t >= count) return;
    bwd_wave_front<T, MF>(P, arena, P.lvl_all[list_begin + t], x_perm);
}

// Control words of the dependency-driven sweeps (one array per handle):
// four ticket counters and the sweep epoch.  A supernode's flag holds
// 2*epoch after its forward step and 2*epoch+1 after its backward step.
enum { kCtlFwdWave = 0, kCtlFwdGroup = 1, kCtlBwdGroup = 2, kCtlBwdWave = 3, kCtlEpoch = 4, kCtlFwdRows = 5 };

__global__ void k_sweep_prep(unsigned* ctl) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctl[kCtlFwdWave] = ctl[kCtlFwdGroup] = ctl[kCtlBwdGroup] = ctl[kCtlBwdWave] = ctl[kCtlFwdRows] = 0u;
        ctl[kCtlEpoch] = ctl[kCtlEpoch] + 1u;
    }
}

// Dependency-driven forward sweep over the supernodes lvl_all[t0, t1)
// (whole levels from the leaves up, every front of order <= 64) by
// one-wave workgroups: each takes the next supernode in level order from a
// ticket counter (read through LDS after a barrier, so that every lane of
// the wave sees the same ticket), so every
// child of its supernode is held by a wave that started earlier and the
// oldest unfinished ticket can always proceed.  The wave loads its lane's
// row of the panel, the reciprocal pivot and the gather positions before
// it waits for the children; then lane i gathers row i of the front and
// one pass over the columns solves the diagonal block and forms the update
// vector (lane k broadcasts y_k, rows below subtract their multiple).
template <typename T>
__global__ void __launch_bounds__(64)
k_fwd_wave(DevPlan P, const T* __restrict__ arena, int t0, int t1, double* __restrict__ v_perm,
           double* __restrict__ uvec, unsigned* ctl, unsigned* done, int32_t* err, unsigned long long ticks) {
    __shared__ int s_ticket[2];
    const int lane = threadIdx.x;
    const unsigned want = 2u * ctl[kCtlEpoch];
    if (lane == 0) s_ticket[0] = (int)atomicAdd(&ctl[kCtlFwdWave], 1u);
    __syncthreads();
    for (int it = 0;; ++it) {
        const int t = s_ticket[it & 1] + t0;
        if (t >= t1) break;
        if (lane == 0) s_ticket[(it + 1) & 1] = (int)atomicAdd(&ctl[kCtlFwdWave], 1u);
        const int s = P.lvl_all[t];
        const int c0 = P.sn_start[s], w = P.sn_start[s + 1] - c0;
        const int ro = P.sn_rowptr[s], f = P.sn_rowptr[s + 1] - ro;
        const T* L = arena + P.l_off[s];
        const bool act = lane < f;
        double lr[kWave];
#pragma unroll
        for (int k = 0; k < kWave; ++k) lr[k] = (k < w && act) ? (double)L[lane + (int64_t)k * f] : 0.0;
        const double rd = lane < w ? 1.0 / (double)L[lane + (int64_t)lane * f] : 0.0;
        int q0 = 0, q1 = 0;
        if (act) { q0 = P.cb_ptr[ro + lane]; q1 = P.cb_ptr[ro + lane + 1]; }
        const int src0 = q0 < q1 ? P.cb_src[q0] : -1;
        const int src1 = q0 + 1 < q1 ? P.cb_src[q0 + 1] : -1;
        double vi = lane < w ? v_perm[c0 + lane] : 0.0;
        for (int c = P.child_ptr[s] + lane; c < P.child_ptr[s + 1]; c += kWave)
            wait_flag(&done[P.child_list[c]], want, err, ticks);
        __syncthreads();
        acquire_device();
        if (src0 >= 0) vi += uvec[src0];
        if (src1 >= 0) vi += uvec[src1];
        for (int q = q0 + 2; q < q1; ++q) vi += uvec[P.cb_src[q]];
#pragma unroll
        for (int k = 0; k < kWave; ++k) {
            if (k < w) {
                const double yk = lane_bcast(vi, k) * lane_bcast(rd, k);
                if (lane == k) vi = yk;
                else if (lane > k) vi = fma(-lr[k], yk, vi);
            }
        }
        if (lane < w) v_perm[c0 + lane] = vi;
        else if (act) uvec[ro + lane] = vi;
        release_device();
        __syncthreads();
        if (lane == 0) flag_store(&done[s], want);
    }
}

// Dependency-driven backward sweep over lvl_all[t0, t1) (fronts of order
// <= 64), tickets handed out root side first.  Lane j holds column j of
// the panel; after the parent's flag (when the parent is in the range) it
// forms the product with the solved rows below and back-substitutes the
// diagonal block with lane broadcasts.
template <typename T>
__global__ void __launch_bounds__(64)
k_bwd_wave(DevPlan P, const T* __restrict__ arena, int t0, int t1, int lvl_hi, double* __restrict__ x_perm,
           unsigned* ctl, unsigned* done, int32_t* err, unsigned long long ticks) {
    __shared__ int s_ticket[2];
    const int lane = threadIdx.x;
    const unsigned want = 2u * ctl[kCtlEpoch] + 1u;
    if (lane == 0) s_ticket[0] = (int)atomicAdd(&ctl[kCtlBwdWave], 1u);
    __syncthreads();
    for (int it = 0;; ++it) {
        const int t = t1 - 1 - s_ticket[it & 1];
        if (t < t0) break;
        if (lane == 0) s_ticket[(it + 1) & 1] = (int)atomicAdd(&ctl[kCtlBwdWave], 1u);
        const int s = P.lvl_all[t];
        const int c0 = P.sn_start[s], w = P.sn_start[s + 1] - c0;
        const int ro = P.sn_rowptr[s], f = P.sn_rowptr[s + 1] - ro;
        const T* L = arena + P.l_off[s];
        const bool act = lane < f, own = lane < w;
        double lc[kWave];
        const T* Lc = L + (int64_t)lane * f;
#pragma unroll
        for (int k = 0; k < kWave; ++k) lc[k] = (k < f && own) ? (double)Lc[k] : 0.0;
        const double rd = own ? 1.0 / (double)Lc[lane] : 0.0;
        const int row = act ? P.sn_rows[ro + lane] : 0;
        const int par = P.sn_parent[s];
        if (lane == 0 && par >= 0 && P.sn_level[par] < lvl_hi) wait_flag(&done[par], want, err, ticks);
        __syncthreads();
        acquire_device();
        const double z = act ? x_perm[row] : 0.0;
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < kWave; ++k)
            if (k >= w && k < f) acc = fma(lc[k], lane_bcast(z, k), acc);
        double ri = own ? z - acc : 0.0;
#pragma unroll
        for (int k = kWave - 1; k >= 0; --k) {
            if (k < w) {
                const double xk = lane_bcast(ri, k) * lane_bcast(rd, k);
                if (lane == k) ri = xk;
                else if (lane < k) ri = fma(-lc[k], xk, ri);
            }
        }
        if (own) x_perm[c0 + lane] = ri;
        release_device();
        __syncthreads();
        if (lane == 0) flag_store(&done[s], want);
    }
}

// Row r of columns c .. c + 63 of a column-major panel with leading
// dimension f: l[k] = L[r + (c + k) f] for k < n when ok.  A wave none of
// whose lanes has ok loads nothing (l = 0); otherwise, in groups of eight
// columns, loads stop after the group holding column n - 1, columns from n
// on inside that group re-read column c + n - 1 and a lane with ok false
// reads L[0], so every load is from inside the panel; callers use only
// k < n of rows with ok.  The offset is a per-thread 32-bit value that
// advances by f per column.
template <typename T>
__device__ __forceinline__ void load_panel_row(T (&l)[kWave], const T* __restrict__ L, int r, int c, int f, int n,
                                               bool ok) {
    if (__ballot(ok) == 0) {
#pragma unroll
        for (int k = 0; k < kWave; ++k) l[k] = T(0);
        return;
    }
    int off = ok ? r + c * f : 0;
    const int step = ok ? f : 0;
#pragma unroll
    for (int k0 = 0; k0 < kWave; k0 += 8) {
        if (k0 < n) {
#pragma unroll
            for (int k = k0; k < k0 + 8; ++k) {
                l[k] = L[off];
                off += (k + 1 < n) ? step : 0;
            }
        } else {
#pragma unroll
            for (int k = k0; k < k0 + 8; ++k) l[k] = T(0);
        }
    }
}

// Forward sweep of one supernode with f <= blockDim.x, one row per thread:
// thread i holds v_i (vi), the reciprocal of its pivot when i < w (rd) and
// its row of the panel in the current 64-column block (l; the caller loads
// block 0).  Per block the wave that holds the block's rows solves it with
// lane broadcasts from registers (rows scaled by their reciprocal pivots)
// and leaves y in LDS (two buffers, so one barrier per block suffices);
// every row below then subtracts its products in column order (as
// fwd_front does) and loads its row of the next block.
template <typename T>
__device__ __forceinline__ void fwd_rows(const T* __restrict__ L, int w, int f, double& vi, T (&l)[kWave],
                                         double rd, double* ybuf) {
    const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
    const int nblk = (w + kWave - 1) / kWave;
    for (int b = 0; b < nblk; ++b) {
        const int kb = b * kWave, nb = min(kWave, w - kb);
        double* y = ybuf + (b & 1) * kWave;
        if (wv == b) {
            // each row of the block carries s = v / pivot (s_k = y_k once
            // the rows above are applied) and takes the update of row k as
            // s -= (l_k / pivot) y_k, its multiplier zero unless the row is
            // below k in the block: one broadcast and one fma per step on
            // the dependency chain.  Steps in groups of eight (one branch
            // per group); rows below the block (lanes >= nb) keep v.
            const int ln = opaque(lane);
            const bool own = ln < nb;
            double sv = own ? vi * rd : vi;
#pragma unroll
            for (int k0 = 0; k0 < kWave; k0 += 8) {
                if (k0 < nb) {
#pragma unroll
                    for (int k = k0; k < k0 + 8; ++k) {
                        const double m = (own && ln > k) ? (double)l[k] * rd : 0.0;
                        sv = fma(-m, lane_bcast(sv, k), sv);
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            vi = sv;
            if (own) y[lane] = vi;
        }
        __syncthreads();
        if (tid >= kb + nb && tid < f) {
            // y read from LDS 8 entries at a time (bounded register use);
            // products of columns k >= nb are not added
            double acc = 0.0;
#pragma unroll
            for (int k0 = 0; k0 < kWave; k0 += 8) {
                if (k0 < nb) {
#pragma unroll
                    for (int k = k0; k < k0 + 8; ++k) {
                        const double a = fma((double)l[k], y[k], acc);
                        acc = k < nb ? a : acc;
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            vi -= acc;
        }
        if (b + 1 < nblk) {
            const int kn = kb + kWave;
            load_panel_row(l, L, tid, kn, f, min(kWave, w - kn), tid >= kn && tid < f);
        }
    }
}

// Dependency-driven forward sweep by workgroups of kGroupThreads threads
// when every front of lvl_all[t0, t1) has at most that many rows: each
// front is held one row per thread (fwd_rows), its first block row loaded
// before the wait on the children; otherwise as k_fwd_group.
template <typename T>
__global__ void __launch_bounds__(kGroupThreads)
k_fwd_group_rows(DevPlan P, const T* __restrict__ arena, int t0, int t1, int lvl_lo, double* __restrict__ v_perm,
                 double* __restrict__ uvec, unsigned* ctl, unsigned* done, int32_t* err, unsigned long long ticks) {
    __shared__ double ybuf[2 * kWave];
    __shared__ int s_ticket[2];
    const int tid = threadIdx.x, nt = blockDim.x;
    const unsigned want = 2u * ctl[kCtlEpoch];
    if (tid == 0) s_ticket[0] = (int)atomicAdd(&ctl[kCtlFwdRows], 1u);
    __syncthreads();
    for (int it = 0;; ++it) {
        const int t = s_ticket[it & 1] + t0;
        if (t >= t1) break;
        if (tid == 0) s_ticket[(it + 1) & 1] = (int)atomicAdd(&ctl[kCtlFwdRows], 1u);
        const int s = P.lvl_all[t];
        const int c0 = P.sn_start[s], w = P.sn_start[s + 1] - c0;
        const int ro = P.sn_rowptr[s], f = P.sn_rowptr[s + 1] - ro;
        const T* Ls = arena + P.l_off[s];
        // work that does not depend on the children, issued before the
        // wait: this thread's row of the first column block and its pivot,
        // its own right-hand side entry and its first contribution indices
        T l[kWave];
        const bool r0 = tid < f;
        load_panel_row(l, Ls, tid, 0, f, min(kWave, w), r0);
        double rd = tid < w ? 1.0 / (double)Ls[tid + (int64_t)tid * f] : 0.0;
        constexpr int kPre = 4;
        double vi = (r0 && tid < w) ? v_perm[c0 + tid] : 0.0;
        const int qa = r0 ? P.cb_ptr[ro + tid] : 0, qb = r0 ? P.cb_ptr[ro + tid + 1] : 0;
        int src[kPre];
#pragma unroll
        for (int k = 0; k < kPre; ++k) src[k] = qa + k < qb ? P.cb_src[qa + k] : -1;
        for (int c = P.child_ptr[s] + tid; c < P.child_ptr[s + 1]; c += nt) {
            const int ch = P.child_list[c];
            if (P.sn_level[ch] >= lvl_lo) wait_flag(&done[ch], want, err, ticks);
        }
        __syncthreads();
        acquire_device();
#pragma unroll
        for (int k = 0; k < kPre; ++k)
            if (src[k] >= 0) vi += uvec[src[k]];
        for (int q = qa + kPre; q < qb; ++q) vi += uvec[P.cb_src[q]];
        vi = settle(vi);
        rd = settle(rd);
        fwd_rows(Ls, w, f, vi, l, rd, ybuf);
        if (tid < w) v_perm[c0 + tid] = vi;
        else if (r0) uvec[ro + tid] = vi;
        release_device();
        __syncthreads();
        if (tid == 0) flag_store(&done[s], want);
    }
}

// Dependency-driven forward sweep by workgroups over lvl_all[t0, t1)
// (levels from lvl_lo up); children below lvl_lo were finished by an
// earlier launch.  The next ticket is fetched while the current supernode
// is processed.
template <typename T>
__global__ void __launch_bounds__(256)
k_fwd_group(DevPlan P, const T* __restrict__ arena, int t0, int t1, int lvl_lo, int ldd,
            double* __restrict__ v_perm, double* __restrict__ uvec, unsigned* ctl, unsigned* done, int32_t* err,
            unsigned long long ticks) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* v = reinterpret_cast<double*>(smem_raw);
    __shared__ int s_ticket[2];
    const int tid = threadIdx.x, nt = blockDim.x;
    const unsigned want = 2u * ctl[kCtlEpoch];
    if (tid == 0) s_ticket[0] = (int)atomicAdd(&ctl[kCtlFwdGroup], 1u);
    __syncthreads();
    for (int it = 0;; ++it) {
        const int t = s_ticket[it & 1] + t0;
        if (t >= t1) break;
        if (tid == 0) s_ticket[(it + 1) & 1] = (int)atomicAdd(&ctl[kCtlFwdGroup], 1u);
        const int s = P.lvl_all[t];
        const int c0 = P.sn_start[s], w = P.sn_start[s + 1] - c0;
        const int ro = P.sn_rowptr[s], f = P.sn_rowptr[s + 1] - ro;
        const T* Ls = arena + P.l_off[s];
        // work that does not depend on the children, issued before the
        // wait: the first diagonal block, this thread's first row's own
        // right-hand side and its first contribution indices
        stage_diag_block(Ls, f, min(kWave, w), v + ((f + 1) & ~1), ldd);
        constexpr int kPre = 4;
        const bool r0 = tid < f;
        double own = (r0 && tid < w) ? v_perm[c0 + tid] : 0.0;
        int qa = r0 ? P.cb_ptr[ro + tid] : 0, qb = r0 ? P.cb_ptr[ro + tid + 1] : 0;
        int src[kPre];
#pragma unroll
        for (int k = 0; k < kPre; ++k) src[k] = qa + k < qb ? P.cb_src[qa + k] : -1;
        // a front with one diagonal block and at most one row below per
        // thread: this thread's panel row below the block, loaded now
        const bool single = w <= kWave && f - w <= nt;
        double lrow[kWave];
        {
            const bool hr = single && tid < f - w;
            const T* Li = Ls + (hr ? w + tid : 0);
#pragma unroll
            for (int k = 0; k < kWave; ++k) lrow[k] = (hr && k < w) ? (double)Li[(int64_t)k * f] : 0.0;
        }
        for (int c = P.child_ptr[s] + tid; c < P.child_ptr[s + 1]; c += nt) {
            const int ch = P.child_list[c];
            if (P.sn_level[ch] >= lvl_lo) wait_flag(&done[ch], want, err, ticks);
        }
        __syncthreads();
        acquire_device();
        if (r0) {
            double acc = own;
#pragma unroll
            for (int k = 0; k < kPre; ++k)
                if (src[k] >= 0) acc += uvec[src[k]];
            for (int q = qa + kPre; q < qb; ++q) acc += uvec[P.cb_src[q]];
            v[tid] = acc;
        }
        for (int i = tid + nt; i < f; i += nt) {
            double acc = (i < w) ? v_perm[c0 + i] : 0.0;
            const int q1 = P.cb_ptr[ro + i + 1];
            for (int q = P.cb_ptr[ro + i]; q < q1; ++q) acc += uvec[P.cb_src[q]];
            v[i] = acc;
        }
        __syncthreads();
        if (single) {
            // one diagonal block: its solve, then the rows below from the
            // panel rows loaded before the wait (same order of operations
            // as fwd_front, so the result is the same)
            double* D = v + ((f + 1) & ~1);
            const int lane = tid % kWave;
            if (tid < kWave) {
                const double vi = wave_fwd_tri(lane < w ? v[lane] : 0.0, D, ldd, w);
                if (lane < w) v[lane] = vi;
            }
            __syncthreads();
            if (tid < f - w) {
                double acc = 0.0;
#pragma unroll
                for (int k = 0; k < kWave; ++k)
                    if (k < w) acc = fma(lrow[k], v[k], acc);
                v[w + tid] -= acc;
            }
            __syncthreads();
        } else {
            fwd_front(Ls, w, f, ldd, v, v + ((f + 1) & ~1), true);
        }
        for (int i = tid; i < f; i += nt) {
            if (i < w) v_perm[c0 + i] = v[i];
            else uvec[ro + i] = v[i];
        }
        release_device();
        __syncthreads();
        if (tid == 0) flag_store(&done[s], want);
    }
}

// Dependency-driven backward sweep by workgroups over lvl_all[t0, t1),
// root side first; the whole range is above every level a later launch
// handles, so the parent is always inside it (or is a root).
template <typename T>
__global__ void __launch_bounds__(256)
k_bwd_group(DevPlan P, const T* __restrict__ arena, int t0, int t1, int ldd, double* __restrict__ x_perm,
            unsigned* ctl, unsigned* done, int32_t* err, unsigned long long ticks) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* z = reinterpret_cast<double*>(smem_raw);
    __shared__ double tb[kWave];
    __shared__ int s_ticket[2];
    const int tid = threadIdx.x, nt = blockDim.x;
    const unsigned want = 2u * ctl[kCtlEpoch] + 1u;
    if (tid == 0) s_ticket[0] = (int)atomicAdd(&ctl[kCtlBwdGroup], 1u);
    __syncthreads();
    for (int it = 0;; ++it) {
        const int t = t1 - 1 - s_ticket[it & 1];
        if (t < t0) break;
        if (tid == 0) s_ticket[(it + 1) & 1] = (int)atomicAdd(&ctl[kCtlBwdGroup], 1u);
        const int s = P.lvl_all[t];
        const int c0 = P.sn_start[s], w = P.sn_start[s + 1] - c0;
        const int ro = P.sn_rowptr[s], f = P.sn_rowptr[s + 1] - ro;
        const int par = P.sn_parent[s];
        const T* Ls = arena + P.l_off[s];
        // issued before the wait: the last diagonal block (the first one
        // solved) and this thread's first row index
        const int nblk = (w + kWave - 1) / kWave, kbl = (nblk - 1) * kWave;
        stage_diag_block(Ls + kbl + (int64_t)kbl * f, f, w - kbl, z + ((f + 1) & ~1), ldd);
        const int row0 = tid < f ? P.sn_rows[ro + tid] : 0;
        // a front with one diagonal block and at most 4 x 64 rows below:
        // the panel entries of the dot products, loaded now (the products
        // then run in bwd_front's order)
        const int lane = tid % kWave, wid = tid / kWave;
        const bool single = w <= kWave && f - w <= 4 * kWave && nt == 4 * kWave;
        double lp[2][4][8];
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const int k = wid * 8 + p * 32 + c, i = w + lane + m * kWave;
                    lp[p][m][c] = (single && k < w && i < f) ? (double)Ls[i + (int64_t)k * f] : 0.0;
                }
        if (tid == 0 && par >= 0) wait_flag(&done[par], want, err, ticks);
        __syncthreads();
        acquire_device();
        if (tid < f) z[tid] = x_perm[row0];
        for (int i = tid + nt; i < f; i += nt) z[i] = x_perm[P.sn_rows[ro + i]];
        __syncthreads();
        if (single) {
            double* D = z + ((f + 1) & ~1);
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                const int k0 = wid * 8 + p * 32;
                if (k0 < w) {
                    double part[8];
#pragma unroll
                    for (int c = 0; c < 8; ++c) part[c] = 0.0;
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        const int i = w + lane + m * kWave;
                        if (i < f) {
                            const double zi = z[i];
#pragma unroll
                            for (int c = 0; c < 8; ++c) part[c] = fma(lp[p][m][c], zi, part[c]);
                        }
                    }
#pragma unroll
                    for (int c = 0; c < 8; ++c) {
                        const double sc = wave_sum(part[c]);
                        if (lane == 0 && k0 + c < w) tb[k0 + c] = sc;
                    }
                }
            }
            __syncthreads();
            if (wid == 0) {
                const double ri = wave_bwd_tri(lane < w ? z[lane] - tb[lane] : 0.0, D, ldd, w);
                if (lane < w) z[lane] = ri;
            }
            __syncthreads();
        } else {
            bwd_front(Ls, w, f, ldd, z, z + ((f + 1) & ~1), tb, true);
        }
        for (int i = tid; i < w; i += nt) x_perm[c0 + i] = z[i];
        release_device();
        __syncthreads();
        if (tid == 0) flag_store(&done[s], want);
    }
}

// ---------------------------------------------------------------- vectors

__global__ void k_gather_perm(DevPlan P, const double* __restrict__ in, double* __restrict__ out,
                              const double* __restrict__ scale) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P.n) return;
    double v = in[P.perm[k]];
    out[k] = scale ? v * scale[k] : v;
}

__global__ void k_scatter_perm(DevPlan P, const double* __restrict__ in, double* __restrict__ out,
                               const double* __restrict__ scale) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P.n) return;
    double v = in[k];
    out[P.perm[k]] = scale ? v * scale[k] : v;
}

// (J x)_r and (|J||x|)_r.  A row split off K (long) is read from the values
// k_dense_rowdot left for this x; the others are summed here, in CSR order.
__device__ __forceinline__ void row_jx(const DevPlan& P, const SysVals& v, int r, const double* __restrict__ x,
                                       double& acc, double& mag) {
    const int a0 = P.j_ptr[r], a1 = P.j_ptr[r + 1];
    if (P.dense_min > 0 && a1 - a0 >= P.dense_min) {
        int b = 0;
        while (b < P.ndense && P.drows[b] != r) ++b;
        if (b < P.ndense) {
            acc = P.drowdot[2 * b];
            mag = P.drowdot[2 * b + 1];
            return;
        }
    }
    acc = 0.0;
    mag = 0.0;
    // four entries at a time: column indices, then values, then the terms
    // added in order
    for (int a = a0; a < a1; a += 4) {
        int ci[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) ci[u] = a + u < a1 ? P.j_col[a + u] : 0;
        double jv[4], xv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const bool ok = a + u < a1;
            jv[u] = ok ? jval(v, P.nnzg, a + u) : 0.0;
            xv[u] = ok ? x[ci[u]] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (a + u < a1) {
                const double p = jv[u] * xv[u];
                acc += p;
                mag += fabs(p);
            }
    }
}

// Residual, pass 1 (one thread per constraint row): for rows weighted by d
// (LiftedKKT all rows; HyKKT rows of H) t = d (J x) and ta = |d| (|J||x|);
// for HyKKT rows of G the K1 second-block residual rhs2 - (G x - delta_c y)
// and its componentwise ratio.
__global__ void __launch_bounds__(256)
k_resid_rows(DevPlan P, SysVals v, const double* __restrict__ d, const double* __restrict__ x,
             const double* __restrict__ y, const double* __restrict__ rhs2, double* __restrict__ res2,
             double* __restrict__ t, double* __restrict__ ta, unsigned long long* omega_bits,
             unsigned long long* resmax_bits) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = r < P.m;
    double acc = 0.0, mag = 0.0;
    if (in) row_jx(P, v, r, x, acc, mag);
    const bool eq = in && P.hy && r < P.m_eq;
    double ratio = 0.0, num = 0.0;
    int inst = -1;
    if (eq) {
        if (v.delta_c != 0.0) {
            const double q = v.delta_c * y[r];
            acc -= q;
            mag += fabs(q);
        }
        double res = rhs2[r] - acc;
        res2[r] = res;
        num = fabs(res);
        double den = mag + fabs(rhs2[r]);
        ratio = den > 0.0 ? num / den : (num == 0.0 ? 0.0 : INFINITY);  // NaN -> INFINITY
        inst = P.inst_of_eqrow[r];
    } else if (in) {
        double dr = d[r];
        t[r] = dr * acc;
        ta[r] = fabs(dr) * mag;
    }
    if (P.hy && P.m_eq > 0) {
        // only blocks that contain equality rows report
        if (__syncthreads_or(eq)) block_max_push(eq, inst, ratio, num, omega_bits, resmax_bits);
    }
}

// Residual, pass 2 (one thread per variable): res1 = rhs1 - (W x + sigma_x x
// + sum_{weighted rows} J^T t [+ G^T y]) and the componentwise ratio
// |res1| / (|W||x| + |sigma_x x| + |J|^T ta [+ |G|^T |y|] + |rhs1|).
__global__ void __launch_bounds__(256)
k_resid_vars(DevPlan P, SysVals v, const double* __restrict__ x, const double* __restrict__ y,
             const double* __restrict__ rhs1, const double* __restrict__ t, const double* __restrict__ ta,
             double* __restrict__ res1, unsigned long long* omega_bits, unsigned long long* resmax_bits) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = i < P.n;
    double ratio = 0.0, num = 0.0;
    int inst = -1;
    if (in) {
        // the entries of each sum four at a time: their index loads issued
        // together, then their value loads, then the terms added in order
        // (the same sums as one entry at a time)
        double acc = 0.0, mag = 0.0;
        const int w0 = P.wf_ptr[i], w1 = P.wf_ptr[i + 1];
        for (int k = w0; k < w1; k += 4) {
            int vi[4], ci[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const bool ok = k + u < w1;
                vi[u] = ok ? P.wf_vidx[k + u] : 0;
                ci[u] = ok ? P.wf_col[k + u] : 0;
            }
            double wv[4], xv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const bool ok = k + u < w1;
                wv[u] = ok ? v.w_val[vi[u]] : 0.0;
                xv[u] = ok ? x[ci[u]] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (k + u < w1) {
                    const double p = wv[u] * xv[u];
                    acc += p;
                    mag += fabs(p);
                }
        }
        double px = v.sigma_x[i] * x[i];
        acc += px;
        mag += fabs(px);
        const int gend = P.jt_gend[i], k1 = P.jt_ptr[i + 1];
        int k0 = P.jt_ptr[i];
        if (P.hy) {
            for (int k = k0; k < gend; k += 4) {
                int ai[4], ri[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const bool ok = k + u < gend;
                    ai[u] = ok ? P.jt_vidx[k + u] : 0;
                    ri[u] = ok ? P.jt_row[k + u] : 0;
                }
                double gv[4], yv[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const bool ok = k + u < gend;
                    gv[u] = ok ? jval(v, P.nnzg, ai[u]) : 0.0;
                    yv[u] = ok ? y[ri[u]] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (k + u < gend) {
                        const double p = gv[u] * yv[u];
                        acc += p;
                        mag += fabs(p);
                    }
            }
            k0 = gend;
        }
        for (int k = k0; k < k1; k += 4) {
            int ai[4], ri[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const bool ok = k + u < k1;
                ai[u] = ok ? P.jt_vidx[k + u] : 0;
                ri[u] = ok ? P.jt_row[k + u] : 0;
            }
            double hv[4], tv[4], tav[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const bool ok = k + u < k1;
                hv[u] = ok ? jval(v, P.nnzg, ai[u]) : 0.0;
                tv[u] = ok ? t[ri[u]] : 0.0;
                tav[u] = ok ? ta[ri[u]] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (k + u < k1) {
                    acc += hv[u] * tv[u];
                    mag += fabs(hv[u]) * tav[u];
                }
        }
        const double bi = rhs1 ? rhs1[i] : 0.0;
        double res = bi - acc;
        res1[i] = res;
        num = fabs(res);
        double den = mag + fabs(bi);
        ratio = den > 0.0 ? num / den : (num == 0.0 ? 0.0 : INFINITY);  // NaN -> INFINITY
        inst = P.inst_of_var[i];
    }
    block_max_push(in, inst, ratio, num, omega_bits, resmax_bits);
}

// ------------------------------------------------- augmented system K2
//
// K2 (Sec. 2.2, delta_c = 0) with its slack rows: LiftedKKT every constraint
// row (relaxed equalities), HyKKT the rows of H.  Global row r, slack index
// q = r - s0 with s0 = m_eq for HyKKT and 0 for LiftedKKT; the slack
// diagonal E_r = D_s + delta_w is the row weight d[r] of the condensed
// matrix (D_H = E when delta_c = 0).  The kernels work on K2 d = f.

__device__ __forceinline__ int slack_begin(const DevPlan& P) { return P.hy ? P.m_eq : 0; }

// u_r = E_r f4_q - f2_q on the slack rows (the other entries are not read)
__global__ void k_k2_u(DevPlan P, const double* __restrict__ d, const double* __restrict__ f2,
                       const double* __restrict__ f4, double* __restrict__ u) {
    const int s0 = slack_begin(P);
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= P.m - s0) return;
    const int r = s0 + q;
    u[r] = d[r] * f4[q] - f2[q];
}

// rbar1 = f1 + H^T u over the slack rows (the condensed first block)
__global__ void k_k2_rbar(DevPlan P, SysVals v, const double* __restrict__ f1, const double* __restrict__ u,
                          double* __restrict__ rb1) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    double acc = 0.0;
    for (int k = P.hy ? P.jt_gend[i] : P.jt_ptr[i]; k < P.jt_ptr[i + 1]; ++k)
        acc += jval(v, P.nnzg, P.jt_vidx[k]) * u[P.jt_row[k]];
    rb1[i] = f1[i] + acc;
}

// slack recovery: dz = f2 + E (H dx - f4), ds = (f2 - dz) / E
__global__ void k_k2_recover(DevPlan P, SysVals v, const double* __restrict__ d, const double* __restrict__ f2,
                             const double* __restrict__ f4, const double* __restrict__ dx, double* __restrict__ ds,
                             double* __restrict__ dz) {
    const int s0 = slack_begin(P);
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= P.m - s0) return;
    const int r = s0 + q;
    double hx, hmag;
    row_jx(P, v, r, dx, hx, hmag);
    const double e = d[r];
    const double z = f2[q] + e * (hx - f4[q]);
    dz[q] = z;
    ds[q] = (f2[q] - z) / e;
}

__device__ __forceinline__ double cw_ratio(double num, double den) {
    return den > 0.0 ? num / den : (num == 0.0 ? 0.0 : INFINITY);  // NaN -> INFINITY
}

// K2 residual, constraint rows: R3 = f3 - G dx (HyKKT equality rows);
// R2 = f2 - (E ds + dz) and R4 = f4 - (H dx + ds) (slack rows), with the
// componentwise ratios |R| / (|K2||d| + |f|).  f = -r.
__global__ void __launch_bounds__(256)
k_k2_resid_rows(DevPlan P, SysVals v, const double* __restrict__ d, const double* __restrict__ r2,
                const double* __restrict__ r3, const double* __restrict__ r4, const double* __restrict__ dx,
                const double* __restrict__ ds, const double* __restrict__ dz, double* __restrict__ R2,
                double* __restrict__ R3, double* __restrict__ R4, unsigned long long* omega_bits,
                unsigned long long* resmax_bits) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = r < P.m;
    const int s0 = slack_begin(P);
    double ratio = 0.0, num = 0.0;
    if (in) {
        double jx, mag;
        row_jx(P, v, r, dx, jx, mag);
        if (r < s0) {
            const double res = -r3[r] - jx;
            R3[r] = res;
            num = fabs(res);
            ratio = cw_ratio(num, mag + fabs(r3[r]));
        } else {
            const int q = r - s0;
            const double res4 = -r4[q] - (jx + ds[q]);
            const double es = d[r] * ds[q];
            const double res2 = -r2[q] - (es + dz[q]);
            R2[q] = res2;
            R4[q] = res4;
            num = fmax(fabs(res2), fabs(res4));
            ratio = fmax(cw_ratio(fabs(res4), mag + fabs(ds[q]) + fabs(r4[q])),
                         cw_ratio(fabs(res2), fabs(es) + fabs(dz[q]) + fabs(r2[q])));
        }
    }
    block_max_push(in, 0, ratio, num, omega_bits, resmax_bits);
}

// K2 residual, variables: R1 = f1 - ((W + Sx) dx + G^T dy + H^T dz).
__global__ void __launch_bounds__(256)
k_k2_resid_vars(DevPlan P, SysVals v, const double* __restrict__ r1, const double* __restrict__ dx,
                const double* __restrict__ dy, const double* __restrict__ dz, double* __restrict__ R1,
                unsigned long long* omega_bits, unsigned long long* resmax_bits) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = i < P.n;
    double ratio = 0.0, num = 0.0;
    if (in) {
        double acc = 0.0, mag = 0.0;
        for (int k = P.wf_ptr[i]; k < P.wf_ptr[i + 1]; ++k) {
            const double t = v.w_val[P.wf_vidx[k]] * dx[P.wf_col[k]];
            acc += t;
            mag += fabs(t);
        }
        const double px = v.sigma_x[i] * dx[i];
        acc += px;
        mag += fabs(px);
        const int s0 = slack_begin(P);
        const int gend = P.hy ? P.jt_gend[i] : P.jt_ptr[i];
        for (int k = P.jt_ptr[i]; k < gend; ++k) {
            const double t = jval(v, P.nnzg, P.jt_vidx[k]) * dy[P.jt_row[k]];
            acc += t;
            mag += fabs(t);
        }
        for (int k = gend; k < P.jt_ptr[i + 1]; ++k) {
            const double t = jval(v, P.nnzg, P.jt_vidx[k]) * dz[P.jt_row[k] - s0];
            acc += t;
            mag += fabs(t);
        }
        const double res = -r1[i] - acc;
        R1[i] = res;
        num = fabs(res);
        ratio = cw_ratio(num, mag + fabs(r1[i]));
    }
    block_max_push(in, 0, ratio, num, omega_bits, resmax_bits);
}

// last block row of K3: V ds + S dv = -(S v - mu e)
__global__ void k_bound_dual(int64_t count, const double* __restrict__ s, const double* __restrict__ v, double mu,
                             const double* __restrict__ ds, double* __restrict__ dv) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) dv[i] = -(v[i] * ds[i] - mu) / s[i] - v[i];
}

// ------------------------------------------------------ split dense rows
//
// Rows of J kept out of K: the factor is that of K_s = K - J_d^T D_d J_d and
// K^{-1} b = y - Z C^{-1} (J_d y) with y = K_s^{-1} b, Z = K_s^{-1} J_d^T and
// C = D_d^{-1} + J_d Z (Woodbury).  J_d and Z are k dense rows of length n
// (row-major), C's Cholesky factor is k x k (lower, row-major), k <= 64.

// Long rows are split into kDenseChunks chunks, one workgroup each; sums of
// the chunks' partials are taken in chunk order (deterministic).
constexpr int kDenseChunks = kDenseChunkBuf;

__device__ __forceinline__ void chunk_of(int a0, int a1, int c, int& lo, int& hi) {
    const int cs = (a1 - a0 + kDenseChunks - 1) / kDenseChunks;
    lo = min(a1, a0 + c * cs);
    hi = min(a1, lo + cs);
}

// row b of J_d from the CSR values (J_d cleared beforehand): grid (k, chunks)
__global__ void k_dense_scatter(DevPlan P, SysVals v, const int32_t* __restrict__ rows, double* __restrict__ jd) {
    const int b = blockIdx.x, r = rows[b];
    int lo, hi;
    chunk_of(P.j_ptr[r], P.j_ptr[r + 1], blockIdx.y, lo, hi);
    double* out = jd + (int64_t)b * P.n;
    for (int a = lo + threadIdx.x; a < hi; a += blockDim.x) out[P.j_col[a]] = jval(v, P.nnzg, a);
}

// block sum in a fixed order (256 threads)
__device__ double block_sum256(double x) {
    __shared__ double s_p[256 / kWave];
    x = wave_sum(x);
    if (threadIdx.x % kWave == 0) s_p[threadIdx.x / kWave] = x;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < 256 / kWave; ++w) t += s_p[w];
    __syncthreads();
    return t;
}

// (J x)_r and (|J||x|)_r of the split rows for the row kernels (row_jx):
// chunk partials, grid (k, chunks), then k_dense_rowdot_sum
__global__ void __launch_bounds__(256) k_dense_rowdot(DevPlan P, SysVals v, const double* __restrict__ x) {
    const int b = blockIdx.x, r = P.drows[b];
    int lo, hi;
    chunk_of(P.j_ptr[r], P.j_ptr[r + 1], blockIdx.y, lo, hi);
    double acc = 0.0, mag = 0.0;
    for (int a = lo + threadIdx.x; a < hi; a += 256) {
        const double p = jval(v, P.nnzg, a) * x[P.j_col[a]];
        acc += p;
        mag += fabs(p);
    }
    acc = block_sum256(acc);
    mag = block_sum256(mag);
    if (threadIdx.x == 0) {
        double* out = P.drowpart + 2 * ((int64_t)b * kDenseChunks + blockIdx.y);
        out[0] = acc;
        out[1] = mag;
    }
}

__global__ void k_dense_rowdot_sum(DevPlan P) {
    const int b = threadIdx.x;
    if (b >= P.ndense) return;
    double acc = 0.0, mag = 0.0;
    for (int c = 0; c < kDenseChunks; ++c) {
        acc += P.drowpart[2 * (b * kDenseChunks + c)];
        mag += P.drowpart[2 * (b * kDenseChunks + c) + 1];
    }
    P.drowdot[2 * b] = acc;
    P.drowdot[2 * b + 1] = mag;
}

// chunk partials of the lower triangle of J_d Z: grid (k(k+1)/2, chunks)
__global__ void __launch_bounds__(256)
k_dense_cap(int n, const double* __restrict__ jd, const double* __restrict__ z, double* __restrict__ cpart) {
    int e = blockIdx.x, a = 0;
    while (e > a) { e -= a + 1; ++a; }  // entry (a, e) of the lower triangle, e <= a
    int lo, hi;
    chunk_of(0, n, blockIdx.y, lo, hi);
    const double* ja = jd + (int64_t)a * n;
    const double* zb = z + (int64_t)e * n;
    double acc = 0.0;
    for (int i = lo + threadIdx.x; i < hi; i += 256) acc += ja[i] * zb[i];
    acc = block_sum256(acc);
    if (threadIdx.x == 0) cpart[(int64_t)blockIdx.x * kDenseChunks + blockIdx.y] = acc;
}

// C = D_d^{-1} + J_d Z from the partials (chunk order), then its Cholesky
// factor in place (one workgroup of 64 threads, k <= 64); a non-positive
// pivot reports column n (outside the matrix) through status.
__global__ void __launch_bounds__(64)
k_dense_chol(int n, int k, const int32_t* __restrict__ rows, const double* __restrict__ d,
             const double* __restrict__ cpart, double* __restrict__ cap, int32_t* status) {
    __shared__ double A[64 * 64];
    const int t = threadIdx.x;
    for (int i = 0; i < k; ++i)
        if (t <= i) {
            const int64_t e = (int64_t)i * (i + 1) / 2 + t;
            double acc = 0.0;
            for (int c = 0; c < kDenseChunks; ++c) acc += cpart[e * kDenseChunks + c];
            A[i * 64 + t] = acc + (i == t ? 1.0 / d[rows[i]] : 0.0);
        }
    __syncthreads();
    for (int j = 0; j < k; ++j) {
        if (t == 0) {
            const double dj = A[j * 64 + j];
            if (!(dj > 0.0)) {
                atomicMin(status, n);
                A[j * 64 + j] = 1.0;
            } else {
                A[j * 64 + j] = sqrt(dj);
            }
        }
        __syncthreads();
        const double piv = A[j * 64 + j];
        if (t > j && t < k) A[t * 64 + j] /= piv;
        __syncthreads();
        if (t > j && t < k)
            for (int l = j + 1; l <= t; ++l) A[t * 64 + l] -= A[t * 64 + j] * A[l * 64 + j];
        __syncthreads();
    }
    for (int i = 0; i < k; ++i)
        if (t <= i) cap[i * k + t] = A[i * 64 + t];
}

// partial sums of t_b = J_d[b] . x: grid (kDotBlocks, k)
__global__ void __launch_bounds__(256)
k_dense_dots(int n, const double* __restrict__ jd, const double* __restrict__ x, double* __restrict__ part) {
    const int b = blockIdx.y;
    const double* row = jd + (int64_t)b * n;
    double acc = 0.0;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) acc += row[i] * x[i];
    acc = block_sum256(acc);
    if (threadIdx.x == 0) part[b * gridDim.x + blockIdx.x] = acc;
}

// u = C^{-1} t, t_b summed from the partials by one wave (lane q takes
// partials q, q + 64, ..., then a fixed butterfly), the solve by lane 0
__global__ void __launch_bounds__(64)
k_dense_solve(int k, int nparts, const double* __restrict__ part, const double* __restrict__ cap,
              double* __restrict__ u) {
    __shared__ double tb[64];
    for (int b = 0; b < k; ++b) {
        double acc = 0.0;
        for (int q = threadIdx.x; q < nparts; q += kWave) acc += part[b * nparts + q];
        acc = wave_sum(acc);
        if (threadIdx.x == 0) tb[b] = acc;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double y[64];
    for (int b = 0; b < k; ++b) {
        double t = tb[b];
        for (int l = 0; l < b; ++l) t -= cap[b * k + l] * y[l];
        y[b] = t / cap[b * k + b];
    }
    for (int b = k - 1; b >= 0; --b) {
        double t = y[b];
        for (int l = b + 1; l < k; ++l) t -= cap[l * k + b] * y[l];
        y[b] = t / cap[b * k + b];
    }
    for (int b = 0; b < k; ++b) u[b] = y[b];
}

// x -= Z^T u
__global__ void k_dense_correct(int n, int k, const double* __restrict__ z, const double* __restrict__ u,
                                double* __restrict__ x) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int b = 0; b < k; ++b) acc += z[(int64_t)b * n + i] * u[b];
    x[i] -= acc;
}

// max |x| (NaN as +inf) into *bits: a grid-stride pass (few blocks, so
// that few atomics meet at the one word), one atomic per block
constexpr int kMaxabsBlocks = 128;
__global__ void __launch_bounds__(256) k_maxabs(int n, const double* __restrict__ x, unsigned long long* bits) {
    double a = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        a = fmax(a, nan_to_inf(fabs(x[i])));
    a = wave_max(a);
    __shared__ double s_a[256 / kWave];
    if (threadIdx.x % kWave == 0) s_a[threadIdx.x / kWave] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int t = 0; t < (int)(blockDim.x / kWave); ++t) m = fmax(m, s_a[t]);
        atomicMax(bits, (unsigned long long)__double_as_longlong(m));
    }
}

__global__ void k_zero_u64(unsigned long long* p, int count) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0ull;
}

__global__ void k_axpy(int n, double alpha, const double* __restrict__ x, double* __restrict__ y) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] += alpha * x[i];
}

// y_i += x_i for the variables of the instances whose omega (as uint64 bits
// of a nonnegative double) is still above tol: refinement steps of a batch
// that leave converged instances as they are
__global__ void k_masked_axpy(DevPlan P, const unsigned long long* __restrict__ omega_bits, double tol,
                              const double* __restrict__ x, double* __restrict__ y) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    const double om = __longlong_as_double((long long)omega_bits[P.inst_of_var[i]]);
    if (!(om <= tol)) y[i] += x[i];
}

__global__ void k_copy(int n, const double* __restrict__ x, double* __restrict__ y) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = x[i];
}

__global__ void k_fill(int n, double val, double* __restrict__ y) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = val;
}

__global__ void k_shift_copy(int n, const double* __restrict__ x, double delta, double* __restrict__ y) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = x[i] + delta;
}

__global__ void k_scale(int n, double alpha, double* __restrict__ y) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] *= alpha;
}

// out_i = base_i + scale * sum_{r < m_eq} G_ri y_r
__global__ void k_gt(DevPlan P, SysVals v, const double* __restrict__ base, double scale,
                     const double* __restrict__ y, double* __restrict__ out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    double acc = 0.0;
    for (int k = P.jt_ptr[i]; k < P.jt_gend[i]; ++k) acc += v.g_val[P.jt_vidx[k]] * y[P.jt_row[k]];
    out[i] = (base ? base[i] : 0.0) + scale * acc;
}

// out_r = (G x)_r - sub_r
__global__ void k_g(DevPlan P, SysVals v, const double* __restrict__ x, const double* __restrict__ sub,
                    double* __restrict__ out) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= P.m_eq) return;
    double acc, mag;
    row_jx(P, v, r, x, acc, mag);
    out[r] = sub ? acc - sub[r] : acc;
}

// Deterministic dot product: each of kDotBlocks blocks sums a fixed strided
// subset in a fixed tree; one block then sums the partials in order.
__global__ void __launch_bounds__(256)
k_dot_partial(int n, const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ part) {
    __shared__ double red[256 / kWave];
    double acc = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) acc += a[i] * b[i];
    acc = wave_sum(acc);
    if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int t = 0; t < (int)(blockDim.x / kWave); ++t) s += red[t];
        part[blockIdx.x] = s;
    }
}

__global__ void __launch_bounds__(256) k_dot_final(int nparts, const double* __restrict__ part, double* result) {
    __shared__ double red[256 / kWave];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) acc += part[i];
    acc = wave_sum(acc);
    if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int t = 0; t < (int)(blockDim.x / kWave); ++t) s += red[t];
        *result = s;
    }
}

__global__ void k_cg_alpha(double* sc) {
    if (threadIdx.x == 0) sc[2] = sc[0] / sc[1];
}
__global__ void k_cg_beta(double* sc) {
    if (threadIdx.x == 0) { sc[4] = sc[3] / sc[0]; sc[0] = sc[3]; }
}
__global__ void k_cg_update(int m, const double* __restrict__ sc, const double* __restrict__ p,
                            const double* __restrict__ q, double* __restrict__ y, double* __restrict__ r) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const double a = sc[2];
    y[i] += a * p[i];
    r[i] -= a * q[i];
}
__global__ void k_cg_direction(int m, const double* __restrict__ sc, const double* __restrict__ r,
                               double* __restrict__ p) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) p[i] = r[i] + sc[4] * p[i];
}
__global__ void k_axpy_dev(int n, const double* __restrict__ sc, int idx, double sign,
                           const double* __restrict__ x, double* __restrict__ y) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] += sign * sc[idx] * x[i];
}

inline int nblk(int64_t n, int b = 256) { return (int)((n + b - 1) / b); }

// ---------------------------------------------------------------- tiled sweeps in one launch per level
//
// The same arithmetic as the block-by-block launches of the tiled fronts
// (every row and column receives the same updates in the same order, so
// the results are bitwise equal), in one launch per level: each workgroup
// owns 64 rows (forward) or 64 columns (backward) of one front and waits,
// block by block, on per-block flags raised by the workgroups that solved
// those blocks; the block's panel tile is loaded before the wait.  A
// workgroup only waits on blocks owned by workgroups dispatched before it
// (the front index varies fastest in the grid, then the tile), so the
// launch makes progress whatever the number of resident workgroups.  The
// flags hold the sweep's epoch (2 e + 1 forward, 2 e + 2 backward, e the
// application counter), so they are never reset; every wait is bounded
// (wait_flag) and a timeout is reported in *err.

// Forward: workgroup (front, t) takes rows [64 t, 64 t + 64).  Grid
// (big list, ceil(maxf / 64)), 256 threads.
template <typename T>
__global__ void __launch_bounds__(256)
k_fwd_tiled_level(DevPlan P, const T* __restrict__ arena, int list_begin, int min_f, double* __restrict__ v_perm,
                  double* __restrict__ uvec, const unsigned* ctl, unsigned* flags, int nblk_lvl, int32_t* err,
                  unsigned long long ticks) {
    __shared__ double D[kWave * kWave];
    __shared__ double yb[kWave];
    __shared__ double red[4][kWave];
    const int s = P.lvl_big[list_begin + blockIdx.x];
    const int c0 = P.sn_start[s], w = P.sn_start[s + 1] - c0;
    const int ro = P.sn_rowptr[s], f = P.sn_rowptr[s + 1] - ro;
    const int t = blockIdx.y, r0 = t * kWave;
    if (f < min_f || r0 >= f) return;
    const int nblk = (w + kWave - 1) / kWave;
    const unsigned want = 2u * ctl[kCtlEpoch] + 1u;
    unsigned* fl = flags + (size_t)blockIdx.x * nblk_lvl;
    const T* L = arena + P.l_off[s];
    const int tid = threadIdx.x, lane = tid % kWave, wid = tid / kWave, k0 = wid * 16;
    const int i = r0 + lane;
    const bool row = i < f;
    const bool diag = t < nblk;
    const int nb = diag ? min(kWave, w - r0) : 0;
    if (diag) stage_diag_block(L + r0 + (int64_t)r0 * f, f, nb, D, kWave);
    double vi = 0.0;
    if (wid == 0 && row) vi = (i < w) ? v_perm[c0 + i] : uvec[ro + i];
    // contribution of solved block j to this workgroup's rows
    auto apply = [&](int j) {
        const int pk = j * kWave, pnb = min(kWave, w - pk);
        const T* Li = L + (row ? i : r0) + (int64_t)(pk + k0) * f;
        double l[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) l[u] = (row && k0 + u < pnb) ? (double)Li[(int64_t)u * f] : 0.0;
        if (tid == 0) wait_flag(&fl[j], want, err, ticks);
        __syncthreads();
        acquire_device();
        if (tid < pnb) yb[tid] = v_perm[c0 + pk + tid];
        __syncthreads();
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < 16; ++u) acc = fma(l[u], (k0 + u < pnb) ? yb[k0 + u] : 0.0, acc);
        red[wid][lane] = acc;
        __syncthreads();
        return (((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane]);
    };
    const int J = min(t, nblk);
    for (int j = 0; j < J; ++j) {
        const double sub = apply(j);
        if (wid == 0 && row) vi -= sub;
    }
    if (!diag) {
        if (wid == 0 && row) uvec[ro + i] = vi;
        return;
    }
    __syncthreads();  // D staged
    if (wid == 0) {
        vi = wave_fwd_tri(vi, D, kWave, nb);
        if (lane < nb) v_perm[c0 + i] = vi;
        release_device();
        if (lane == 0) flag_store(&fl[t], want);
    }
    if (r0 + nb < min(f, r0 + kWave)) {
        // rows below the own columns in the last diagonal tile take this
        // block's update too (its flag is already raised, so the wait in
        // apply returns at once)
        const double sub = apply(t);
        if (wid == 0 && row && lane >= nb) uvec[ro + i] = vi - sub;
    }
}

// Backward: workgroup (front, y) takes column tile t = nblk - 1 - y (the
// last blocks first).  Grid (big list, max blocks), 256 threads.
template <typename T>
__global__ void __launch_bounds__(256)
k_bwd_tiled_level(DevPlan P, const T* __restrict__ arena, int list_begin, int min_f, double* __restrict__ x_perm,
                  const unsigned* ctl, unsigned* flags, int nblk_lvl, int32_t* err, unsigned long long ticks) {
    __shared__ double D[kWave * (kWave + 1)];
    __shared__ double S[kWave * (kWave + 1)];
    __shared__ double tb[kWave];
    const int s = P.lvl_big[list_begin + blockIdx.x];
    const int c0 = P.sn_start[s], w = P.sn_start[s + 1] - c0;
    const int f = P.sn_rowptr[s + 1] - P.sn_rowptr[s];
    const int nblk = (w + kWave - 1) / kWave;
    const int t = nblk - 1 - (int)blockIdx.y;
    if (f < min_f || t < 0) return;
    const unsigned want = 2u * ctl[kCtlEpoch] + 2u;
    unsigned* fl = flags + (size_t)blockIdx.x * nblk_lvl;
    const T* L = arena + P.l_off[s];
    const int tid = threadIdx.x, lane = tid % kWave, wid = tid / kWave, k0 = wid * 16;
    const int ct = t * kWave, tnb = min(kWave, w - ct);
    stage_diag_block(L + ct + (int64_t)ct * f, f, tnb, D, kWave + 1);
    double z = (wid == 0 && lane < tnb) ? x_perm[c0 + ct + lane] : 0.0;
    for (int b = nblk - 1; b > t; --b) {
        const int q = b * kWave, qnb = min(kWave, w - q);
        const bool r = lane < qnb;
        const T* Lr = L + (r ? q + lane : q) + (int64_t)(ct + k0) * f;
        double l[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) l[u] = (r && k0 + u < tnb) ? (double)Lr[(int64_t)u * f] : 0.0;
        if (tid == 0) wait_flag(&fl[b], want, err, ticks);
        __syncthreads();
        acquire_device();
        const double xr = r ? x_perm[c0 + q + lane] : 0.0;
#pragma unroll
        for (int u = 0; u < 16; ++u) S[(k0 + u) * (kWave + 1) + lane] = l[u] * xr;
        __syncthreads();
        const int c = tid >> 2, rq = tid & 3;
        double sum = 0.0;
#pragma unroll
        for (int u = 0; u < 16; ++u) sum += S[c * (kWave + 1) + rq * 16 + u];
        sum += __shfl_xor(sum, 1, kWave);
        sum += __shfl_xor(sum, 2, kWave);
        if (rq == 0) tb[c] = sum;
        __syncthreads();
        if (wid == 0 && lane < tnb) z -= tb[lane];
    }
    __syncthreads();  // D staged
    if (wid != 0) return;
    z = wave_bwd_tri(z, D, kWave + 1, tnb);
    if (lane < tnb) x_perm[c0 + ct + lane] = z;
    release_device();
    if (lane == 0) flag_store(&fl[t], want);
}

}  // namespace

// ================================================================ launchers

void launch_row_weights(const DevPlan& P, const SysVals& v, double* d, hipStream_t st) {
    if (P.m == 0) return;
    hipLaunchKernelGGL(k_row_weights, dim3(nblk(P.m)), dim3(256), 0, st, P, v, d);
}

void launch_assemble(const DevPlan& P, const SysVals& v, const double* d, double* K, int32_t* nonfinite,
                     hipStream_t st) {
    if (P.nnzk == 0) return;
    hipLaunchKernelGGL(k_assemble, dim3(nblk(P.nnzk)), dim3(256), 0, st, P, v, d, K, nonfinite);
}

void launch_init_status(int32_t* status, bool keep_inputs, hipStream_t st) {
    hipLaunchKernelGGL(k_init_status, dim3(1), dim3(64), 0, st, status, keep_inputs ? 1 : 0);
}

void launch_diag_scale(const DevPlan& P, const double* K, double* scale, hipStream_t st) {
    if (P.n == 0) return;
    hipLaunchKernelGGL(k_diag_scale, dim3(nblk(P.n)), dim3(256), 0, st, P, K, scale);
}

template <typename T>
bool launch_factor_level(const DevPlan& P, const LevelInfo& L, const double* K, T* arena,
                         int32_t* status, const double* scale, hipStream_t st, const SideStream* side,
                         double* dscr) {
    if ((size_t)L.small_maxf * L.small_maxf * sizeof(T) + kFactorStaticLds > (size_t)kLdsBytes) return false;
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_factor_small<T, true>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes - kFactorStaticLds);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_factor_small<T, false>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes - kFactorStaticLds);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_big_init<T>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes - 1024);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_big_init_cols<T>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 4 * kInitColRows * (int)sizeof(T));
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_big_panel_fused),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, kFusedPanelLds);
        attr_set = true;
    }
    // fronts above the LDS limit run on the side stream, concurrently with
    // the LDS-resident fronts of the same level (both depend only on lower
    // levels and write disjoint arena regions)
    const bool fork = L.big_count > 0 && L.small_count > 0 && side && side->stream;
    hipStream_t sb = st;
    if (fork) {
        (void)hipEventRecord(side->fork, st);
        (void)hipStreamWaitEvent(side->stream, side->fork, 0);
        sb = side->stream;
    }
    if (L.big_count > 0) {
        if (L.big_maxf <= kInitColRows) {
            // one wave per front column
            hipLaunchKernelGGL(k_big_init_cols<T>, dim3(L.tile_count, kBigTile / 4), dim3(256),
                               (size_t)4 * L.big_maxf * sizeof(T), sb, P, K, arena, L.tile_begin, scale, L.big_maxf);
        } else {
            // assemble the tiles in LDS when a whole tile (64 columns x f rows) fits
            const size_t tile_bytes = (size_t)kBigTile * L.big_maxf * sizeof(T);
            const bool lds_tile = tile_bytes + 1024 <= (size_t)kLdsBytes;
            hipLaunchKernelGGL(k_big_init<T>, dim3(L.tile_count), dim3(256), lds_tile ? tile_bytes : 0, sb, P, K,
                               arena, L.tile_begin, scale, lds_tile ? L.big_maxf : 0);
        }
        // levels with large fronts: panels of kWideRank columns, each
        // factored as kPanelNB-column panels whose updates stop at the wide
        // panel's end, then one rank-kWideRank update of the trailing part
        const bool wide = L.big_maxf >= L.wide_front;
        const int step = wide ? kWideRank : kPanelNB;
        for (int kw = 0; kw < L.big_maxw; kw += step) {
            for (int kb = kw; kb < std::min(kw + step, L.big_maxw); kb += kPanelNB) {
                const int below = L.big_maxf - kb - 1;  // upper bound of rows below the block, any front
                const int crows = sizeof(T) == 8 ? kFusedPanelRows : kPanelRows;
                const int chunks = below > 0 ? (below + crows - 1) / crows : 1;
                if constexpr (sizeof(T) == 8) {
                    hipLaunchKernelGGL(k_big_panel_fused, dim3(chunks, L.big_count), dim3(256), kFusedPanelLds,
                                       sb, P, L.big_one, arena, L.big_begin, kb, status, dscr);
                } else {
                    hipLaunchKernelGGL(k_big_panel<T>, dim3(chunks, L.big_count), dim3(256), 0, sb, P, arena,
                                       L.big_begin, kb, status, reinterpret_cast<T*>(dscr));
                }
                // in a wide panel the update stops at the panel's end (after
                // its last panel it only reaches fronts whose own columns end
                // inside the wide panel, for their columns up to its end)
                const int col_end = wide ? kw + step : INT_MAX;
                const int rest = L.big_maxf - kb - 1;  // upper bound of trailing rows
                const int tiles = rest > 0 ? (rest + 63) / 64 : 0;
                // columns: at most up to col_end (a front whose last panel is
                // narrower starts its trailing part up to kPanelNB - 1 earlier)
                const int tcols = wide ? std::min(tiles, (kw + step - kb) / 64 + 1) : tiles;
                if (tiles > 0)
                    hipLaunchKernelGGL((k_big_update<T, kPanelNB>), dim3(tiles, tcols, L.big_count), dim3(256), 0,
                                       sb, P, L.big_one, arena, L.big_begin, kb, reinterpret_cast<const T*>(dscr),
                                       chunks > 1 ? 1 : 0, col_end);
            }
            if (!wide) continue;
            const int rest = L.big_maxf - kw - step;  // upper bound of trailing rows
            if (rest <= 0) continue;
            const int nt = (rest + kWideTile - 1) / kWideTile, ntri = nt * (nt + 1) / 2;
            hipLaunchKernelGGL(k_big_update_wide<T>, dim3(ntri, L.big_count), dim3(256), 0, sb, P, arena, L.big_begin,
                               kw, nt, 0, ntri);
        }
    }
    if (L.small_count > 0) {
        // two LDS size classes so that small fronts keep several workgroups
        // per CU (one wave per front when the class is tiny); when a level
        // holds both classes and few compact fronts, one launch covers all
        // of them so that the classes run concurrently
        const bool d = sizeof(T) == 8;
        const int na = d ? L.small_split : L.small_split32;
        const int fa = d ? L.small_maxf_a : L.small_maxf_a32;
        const int nbig = L.small_count - na;
        if (na > 0 && nbig > 0 && na <= kMergeCompactFronts) {
            size_t lds = (size_t)L.small_maxf * L.small_maxf * sizeof(T);
            hipLaunchKernelGGL((k_factor_small<T, true>), dim3(L.small_count), dim3(256), lds, st, P, K, arena,
                               L.small_begin, status, scale);
        } else {
            if (na > 0)
                hipLaunchKernelGGL((k_factor_small<T, false>), dim3(na), dim3(L.small_threads_a),
                                   (size_t)fa * fa * sizeof(T), st, P, K, arena, L.small_begin, status, scale);
            if (nbig > 0) {
                size_t lds = (size_t)L.small_maxf * L.small_maxf * sizeof(T);
                hipLaunchKernelGGL((k_factor_small<T, true>), dim3(nbig), dim3(256), lds, st, P, K, arena,
                                   L.small_begin + na, status, scale);
            }
        }
    }
    if (fork) {
        (void)hipEventRecord(side->join, side->stream);
        (void)hipStreamWaitEvent(st, side->join, 0);
    }
    return true;
}

template <typename T>
void launch_fwd_level(const DevPlan& P, const LevelInfo& L, const T* arena, double* v_perm,
                      double* uvec, hipStream_t st, const TiledSync* ts) {
    if (L.all_count == 0) return;
    if (L.all_maxf <= kWave) {
        const dim3 g((L.all_count + 3) / 4);
        if (L.all_maxw <= 16)
            hipLaunchKernelGGL((k_fwd_waves<T, 16>), g, dim3(256), 0, st, P, arena, L.all_begin, L.all_count, v_perm,
                               uvec);
        else if (L.all_maxw <= 32)
            hipLaunchKernelGGL((k_fwd_waves<T, 32>), g, dim3(256), 0, st, P, arena, L.all_begin, L.all_count, v_perm,
                               uvec);
        else
            hipLaunchKernelGGL((k_fwd_waves<T, kWave>), g, dim3(256), 0, st, P, arena, L.all_begin, L.all_count,
                               v_perm, uvec);
        return;
    }
    if (L.all_maxf <= 2 * kWave && L.all_maxw <= kWave) {
        const dim3 g((L.all_count + 1) / 2);
        if (L.all_maxw <= 32)
            hipLaunchKernelGGL((k_fwd_pairs<T, 32>), g, dim3(256), 0, st, P, arena, L.all_begin, L.all_count, v_perm,
                               uvec);
        else
            hipLaunchKernelGGL((k_fwd_pairs<T, kWave>), g, dim3(256), 0, st, P, arena, L.all_begin, L.all_count,
                               v_perm, uvec);
        return;
    }
    const int tf = L.sweep_tiled_f;
    const bool tiled = L.big_count > 0 && L.big_maxf >= tf;
    const int skip_f = tiled ? tf : INT_MAX;
    const int maxf = tiled ? std::min(L.all_maxf, tf - 1) : L.all_maxf;
    const int threads = L.sweep_threads;
    const int ldd = sweep_diag_ld(L.all_maxw);
    size_t lds = (size_t)(((maxf + 1) & ~1) + ldd * ldd) * sizeof(double);
    if (!tiled || L.sweep_small_count > 0)
        hipLaunchKernelGGL(k_fwd<T>, dim3(L.all_count), dim3(threads), lds, st, P, arena, L.all_begin, ldd, skip_f,
                           v_perm, uvec);
    if (!tiled) return;
    hipLaunchKernelGGL(k_fwd_tiled_gather, dim3((L.big_maxf + 255) / 256, L.big_count), dim3(256), 0, st, P,
                       L.big_begin, tf, v_perm, uvec);
    const int nblk = (L.big_maxw + kWave - 1) / kWave;
    if (ts) {
        hipLaunchKernelGGL(k_fwd_tiled_level<T>, dim3(L.big_count, (L.big_maxf + kWave - 1) / kWave), dim3(256), 0,
                           st, P, arena, L.big_begin, tf, v_perm, uvec, ts->ctl, ts->flags + L.tflag_off, nblk,
                           ts->err, ts->ticks);
        return;
    }
    for (int j = 0; j <= nblk; ++j) {
        const int rows = L.big_maxf - std::max(0, (j - 1) * kWave);
        hipLaunchKernelGGL(k_fwd_tiled_step<T>, dim3((rows + kWave - 1) / kWave, L.big_count), dim3(256), 0, st,
                           P, arena, L.big_begin, tf, j, v_perm, uvec);
    }
}

template <typename T>
void launch_bwd_level(const DevPlan& P, const LevelInfo& L, const T* arena, double* x_perm,
                      hipStream_t st, const TiledSync* ts) {
    if (L.all_count == 0) return;
    if (L.all_maxf <= kWave) {
        const dim3 g((L.all_count + 3) / 4);
        if (L.all_maxf <= 32)
            hipLaunchKernelGGL((k_bwd_waves<T, 32>), g, dim3(256), 0, st, P, arena, L.all_begin, L.all_count, x_perm);
        else
            hipLaunchKernelGGL((k_bwd_waves<T, kWave>), g, dim3(256), 0, st, P, arena, L.all_begin, L.all_count,
                               x_perm);
        return;
    }
    if (L.all_maxf <= 2 * kWave && L.all_maxw <= kWave) {
        hipLaunchKernelGGL(k_bwd_pairs<T>, dim3((L.all_count + 1) / 2), dim3(256), 0, st, P, arena, L.all_begin,
                           L.all_count, x_perm);
        return;
    }
    const int tf = L.sweep_tiled_f;
    const bool tiled = L.big_count > 0 && L.big_maxf >= tf;
    const int skip_f = tiled ? tf : INT_MAX;
    const int maxf = tiled ? std::min(L.all_maxf, tf - 1) : L.all_maxf;
    const int threads = L.sweep_threads;
    const int ldd = sweep_diag_ld(L.all_maxw);
    size_t lds = (size_t)(((maxf + 1) & ~1) + ldd * ldd) * sizeof(double);
    if (!tiled || L.sweep_small_count > 0)
        hipLaunchKernelGGL(k_bwd<T>, dim3(L.all_count), dim3(threads), lds, st, P, arena, L.all_begin, ldd, skip_f,
                           x_perm);
    if (!tiled) return;
    hipLaunchKernelGGL(k_bwd_tiled_rect<T>, dim3((L.big_maxw + 7) / 8, L.big_count), dim3(256), 0, st, P, arena,
                       L.big_begin, tf, x_perm);
    const int nblk = (L.big_maxw + kWave - 1) / kWave;
    if (ts) {
        hipLaunchKernelGGL(k_bwd_tiled_level<T>, dim3(L.big_count, nblk), dim3(256), 0, st, P, arena, L.big_begin,
                           tf, x_perm, ts->ctl, ts->flags + L.tflag_off, nblk, ts->err, ts->ticks);
        return;
    }
    for (int b = nblk - 1; b >= 0; --b)
        hipLaunchKernelGGL(k_bwd_tiled_step<T>, dim3(b + 1, L.big_count), dim3(256), 0, st, P, arena, L.big_begin,
                           tf, b, x_perm);
}

template bool launch_factor_level<double>(const DevPlan&, const LevelInfo&, const double*, double*, int32_t*,
                                          const double*, hipStream_t, const SideStream*, double*);
template bool launch_factor_level<float>(const DevPlan&, const LevelInfo&, const double*, float*, int32_t*,
                                         const double*, hipStream_t, const SideStream*, double*);
template void launch_fwd_level<double>(const DevPlan&, const LevelInfo&, const double*, double*, double*,
                                       hipStream_t, const TiledSync*);
template void launch_fwd_level<float>(const DevPlan&, const LevelInfo&, const float*, double*, double*,
                                      hipStream_t, const TiledSync*);
template void launch_bwd_level<double>(const DevPlan&, const LevelInfo&, const double*, double*, hipStream_t,
                                       const TiledSync*);
template void launch_bwd_level<float>(const DevPlan&, const LevelInfo&, const float*, double*, hipStream_t,
                                      const TiledSync*);

namespace {
template <typename T>
void set_sweep_attrs() {
    static bool done_once = false;
    if (done_once) return;
    const int cap = kLdsBytes - kSweepStaticLds;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fwd<T>), hipFuncAttributeMaxDynamicSharedMemorySize, cap);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bwd<T>), hipFuncAttributeMaxDynamicSharedMemorySize, cap);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fwd_group<T>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, cap);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bwd_group<T>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, cap);
    done_once = true;
}
}  // namespace

void launch_sweep_prep(unsigned* ctl, hipStream_t st) {
    hipLaunchKernelGGL(k_sweep_prep, dim3(1), dim3(64), 0, st, ctl);
}

template <typename T>
void launch_fwd_sched(const DevPlan& P, const SweepSched& S, const T* arena, double* v_perm, double* uvec,
                      unsigned* ctl, unsigned* done, int32_t* err, hipStream_t st, bool waves) {
    set_sweep_attrs<T>();
    if (waves && S.wave_t1 > 0)
        hipLaunchKernelGGL(k_fwd_wave<T>, dim3(S.wave_grid), dim3(kWave), 0, st, P, arena, 0, S.wave_t1, v_perm, uvec,
                           ctl, done, err, S.ticks);
    const int t0 = waves ? S.wave_t1 : S.pair_t1, lvl0 = waves ? S.wave_lvl : S.pair_lvl;
    // levels below rows_lvl on the LDS kernel, the rest row-held (their
    // children below rows_lvl are finished by the first launch)
    const int ts = S.rows ? std::max(t0, (int)S.rows_t0) : S.ns;
    if (ts > t0)
        hipLaunchKernelGGL(k_fwd_group<T>, dim3(S.group_grid), dim3(256), S.group_lds, st, P, arena, t0, ts, lvl0,
                           S.ldd, v_perm, uvec, ctl, done, err, S.ticks);
    if (S.ns > ts)
        hipLaunchKernelGGL(k_fwd_group_rows<T>, dim3(S.rows_grid), dim3(kGroupThreads), 0, st, P, arena, ts, S.ns,
                           std::max(lvl0, (int)S.rows_lvl), v_perm, uvec, ctl, done, err, S.ticks);
}

template <typename T>
void launch_bwd_sched(const DevPlan& P, const SweepSched& S, const T* arena, double* x_perm, unsigned* ctl,
                      unsigned* done, int32_t* err, hipStream_t st, bool waves) {
    set_sweep_attrs<T>();
    const int t0 = waves ? S.wave_t1 : S.pair_t1;
    if (S.ns > t0)
        hipLaunchKernelGGL(k_bwd_group<T>, dim3(S.group_grid), dim3(256), S.group_lds, st, P, arena, t0, S.ns, S.ldd,
                           x_perm, ctl, done, err, S.ticks);
    if (waves && S.wave_t1 > 0)
        hipLaunchKernelGGL(k_bwd_wave<T>, dim3(S.wave_grid), dim3(kWave), 0, st, P, arena, 0, S.wave_t1, S.wave_lvl,
                           x_perm, ctl, done, err, S.ticks);
}

bool sweep_sched_grids(SweepSched& S, int device) {
    int cus = 0, khz = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0)
        return false;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) != hipSuccess || khz <= 0) return false;
    S.ticks = (unsigned long long)khz * 1000ull * kSweepWaitSeconds;
    set_sweep_attrs<double>();
    set_sweep_attrs<float>();
    auto occ = [&](const void* fn, int threads, size_t lds) {
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, fn, threads, lds) != hipSuccess) return 0;
        return b;
    };
    int ow = std::min({occ(reinterpret_cast<const void*>(&k_fwd_wave<double>), kWave, 0),
                       occ(reinterpret_cast<const void*>(&k_bwd_wave<double>), kWave, 0),
                       occ(reinterpret_cast<const void*>(&k_fwd_wave<float>), kWave, 0),
                       occ(reinterpret_cast<const void*>(&k_bwd_wave<float>), kWave, 0)});
    int og = std::min({occ(reinterpret_cast<const void*>(&k_fwd_group<double>), 256, S.group_lds),
                       occ(reinterpret_cast<const void*>(&k_bwd_group<double>), 256, S.group_lds),
                       occ(reinterpret_cast<const void*>(&k_fwd_group<float>), 256, S.group_lds),
                       occ(reinterpret_cast<const void*>(&k_bwd_group<float>), 256, S.group_lds)});
    int orow = std::min(occ(reinterpret_cast<const void*>(&k_fwd_group_rows<double>), kGroupThreads, 0),
                        occ(reinterpret_cast<const void*>(&k_fwd_group_rows<float>), kGroupThreads, 0));
    (void)hipGetLastError();
    ow = std::max(ow, 1);
    og = std::max(og, 1);
    orow = std::max(orow, 1);
    S.wave_grid = std::max(1, std::min(ow * cus, S.wave_t1));
    S.group_grid = std::max(1, std::min(og * cus, S.ns - S.wave_t1));
    // the row-held launch covers the upper levels (few fronts per level):
    // fewer workgroups, each taking several supernodes, run its code warm
    S.rows_grid = std::max(1, std::min({orow * cus, kRowsMaxGrid, S.ns - std::max(S.wave_t1, S.rows_t0)}));
    return true;
}

template void launch_fwd_sched<double>(const DevPlan&, const SweepSched&, const double*, double*, double*, unsigned*,
                                       unsigned*, int32_t*, hipStream_t, bool);
template void launch_fwd_sched<float>(const DevPlan&, const SweepSched&, const float*, double*, double*, unsigned*,
                                      unsigned*, int32_t*, hipStream_t, bool);
template void launch_bwd_sched<double>(const DevPlan&, const SweepSched&, const double*, double*, unsigned*,
                                       unsigned*, int32_t*, hipStream_t, bool);
template void launch_bwd_sched<float>(const DevPlan&, const SweepSched&, const float*, double*, unsigned*, unsigned*,
                                      int32_t*, hipStream_t, bool);

void launch_gather_perm(const DevPlan& P, const double* in, double* out, const double* scale, hipStream_t st) {
    if (P.n == 0) return;
    hipLaunchKernelGGL(k_gather_perm, dim3(nblk(P.n)), dim3(256), 0, st, P, in, out, scale);
}

void launch_scatter_perm(const DevPlan& P, const double* in, double* out, const double* scale, hipStream_t st) {
    if (P.n == 0) return;
    hipLaunchKernelGGL(k_scatter_perm, dim3(nblk(P.n)), dim3(256), 0, st, P, in, out, scale);
}

void launch_zero_u64(unsigned long long* p, int count, hipStream_t st) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_zero_u64, dim3(nblk(count)), dim3(256), 0, st, p, count);
}

void launch_dense_rowdot(const DevPlan& P, const SysVals& v, const double* x, hipStream_t st) {
    if (P.ndense == 0) return;
    hipLaunchKernelGGL(k_dense_rowdot, dim3(P.ndense, kDenseChunks), dim3(256), 0, st, P, v, x);
    hipLaunchKernelGGL(k_dense_rowdot_sum, dim3(1), dim3(64), 0, st, P);
}
void launch_residual(const DevPlan& P, const SysVals& v, const double* d, const double* x,
                     const double* y, const double* rhs1, const double* rhs2, double* res1,
                     double* res2, double* tbuf, double* tabuf, unsigned long long* omega_bits,
                     unsigned long long* resmax_bits, hipStream_t st) {
    if (P.m > 0) launch_dense_rowdot(P, v, x, st);
    if (P.m > 0)
        hipLaunchKernelGGL(k_resid_rows, dim3(nblk(P.m)), dim3(256), 0, st, P, v, d, x, y, rhs2, res2, tbuf,
                           tabuf, omega_bits, resmax_bits);
    if (P.n > 0)
        hipLaunchKernelGGL(k_resid_vars, dim3(nblk(P.n)), dim3(256), 0, st, P, v, x, y, rhs1, tbuf, tabuf, res1,
                           omega_bits, resmax_bits);
}

void launch_k2_condense(const DevPlan& P, const SysVals& v, const double* d, const double* f1, const double* f2,
                        const double* f4, double* u, double* rb1, hipStream_t st) {
    const int ms = P.m - (P.hy ? P.m_eq : 0);
    if (ms > 0) hipLaunchKernelGGL(k_k2_u, dim3(nblk(ms)), dim3(256), 0, st, P, d, f2, f4, u);
    if (P.n > 0) hipLaunchKernelGGL(k_k2_rbar, dim3(nblk(P.n)), dim3(256), 0, st, P, v, f1, u, rb1);
}
void launch_k2_recover(const DevPlan& P, const SysVals& v, const double* d, const double* f2, const double* f4,
                       const double* dx, double* ds, double* dz, hipStream_t st) {
    const int ms = P.m - (P.hy ? P.m_eq : 0);
    if (ms > 0) launch_dense_rowdot(P, v, dx, st);
    if (ms > 0) hipLaunchKernelGGL(k_k2_recover, dim3(nblk(ms)), dim3(256), 0, st, P, v, d, f2, f4, dx, ds, dz);
}
void launch_k2_residual(const DevPlan& P, const SysVals& v, const double* d, const double* r1, const double* r2,
                        const double* r3, const double* r4, const double* dx, const double* ds, const double* dy,
                        const double* dz, double* R1, double* R2, double* R3, double* R4,
                        unsigned long long* omega_bits, unsigned long long* resmax_bits, hipStream_t st) {
    if (P.m > 0) launch_dense_rowdot(P, v, dx, st);
    if (P.m > 0)
        hipLaunchKernelGGL(k_k2_resid_rows, dim3(nblk(P.m)), dim3(256), 0, st, P, v, d, r2, r3, r4, dx, ds, dz, R2,
                           R3, R4, omega_bits, resmax_bits);
    if (P.n > 0)
        hipLaunchKernelGGL(k_k2_resid_vars, dim3(nblk(P.n)), dim3(256), 0, st, P, v, r1, dx, dy, dz, R1,
                           omega_bits, resmax_bits);
}
void launch_bound_dual(int64_t count, const double* s, const double* v, double mu, const double* ds, double* dv,
                       hipStream_t st) {
    if (count > 0)
        hipLaunchKernelGGL(k_bound_dual, dim3(nblk(count)), dim3(256), 0, st, count, s, v, mu, ds, dv);
}
void launch_dense_setup_gather(const DevPlan& P, const SysVals& v, const int32_t* rows, int k, double* jd,
                               hipStream_t st) {
    if (k <= 0 || P.n <= 0) return;
    launch_fill(k * P.n, 0.0, jd, st);
    hipLaunchKernelGGL(k_dense_scatter, dim3(k, kDenseChunks), dim3(256), 0, st, P, v, rows, jd);
}
void launch_dense_setup_cap(int n, int k, const int32_t* rows, const double* d, const double* jd, const double* z,
                            double* cpart, double* cap, int32_t* status, hipStream_t st) {
    if (k <= 0) return;
    hipLaunchKernelGGL(k_dense_cap, dim3(k * (k + 1) / 2, kDenseChunks), dim3(256), 0, st, n, jd, z, cpart);
    hipLaunchKernelGGL(k_dense_chol, dim3(1), dim3(64), 0, st, n, k, rows, d, cpart, cap, status);
}
void launch_dense_correct(int n, int k, const double* jd, const double* z, const double* cap, double* part,
                          double* u, double* x, hipStream_t st) {
    if (k <= 0 || n <= 0) return;
    hipLaunchKernelGGL(k_dense_dots, dim3(kDotBlocks, k), dim3(256), 0, st, n, jd, x, part);
    hipLaunchKernelGGL(k_dense_solve, dim3(1), dim3(64), 0, st, k, kDotBlocks, part, cap, u);
    hipLaunchKernelGGL(k_dense_correct, dim3(nblk(n)), dim3(256), 0, st, n, k, z, u, x);
}
void launch_maxabs(int n, const double* x, unsigned long long* bits, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_maxabs, dim3(std::min(nblk(n), kMaxabsBlocks)), dim3(256), 0, st, n, x, bits);
}

void launch_masked_axpy(const DevPlan& P, const unsigned long long* omega_bits, double tol, const double* x,
                        double* y, hipStream_t st) {
    if (P.n > 0) hipLaunchKernelGGL(k_masked_axpy, dim3(nblk(P.n)), dim3(256), 0, st, P, omega_bits, tol, x, y);
}

void launch_axpy(int n, double alpha, const double* x, double* y, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_axpy, dim3(nblk(n)), dim3(256), 0, st, n, alpha, x, y);
}
void launch_copy(int n, const double* x, double* y, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_copy, dim3(nblk(n)), dim3(256), 0, st, n, x, y);
}
void launch_fill(int n, double v, double* y, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_fill, dim3(nblk(n)), dim3(256), 0, st, n, v, y);
}
void launch_shift_copy(int n, const double* x, double delta, double* y, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_shift_copy, dim3(nblk(n)), dim3(256), 0, st, n, x, delta, y);
}
void launch_scale(int n, double alpha, double* y, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_scale, dim3(nblk(n)), dim3(256), 0, st, n, alpha, y);
}
void launch_gt(const DevPlan& P, const SysVals& v, const double* base, double scale, const double* y,
               double* out, hipStream_t st) {
    if (P.n > 0) hipLaunchKernelGGL(k_gt, dim3(nblk(P.n)), dim3(256), 0, st, P, v, base, scale, y, out);
}
void launch_g(const DevPlan& P, const SysVals& v, const double* x, const double* sub, double* out,
              hipStream_t st) {
    if (P.m_eq > 0) launch_dense_rowdot(P, v, x, st);
    if (P.m_eq > 0) hipLaunchKernelGGL(k_g, dim3(nblk(P.m_eq)), dim3(256), 0, st, P, v, x, sub, out);
}
void launch_dot(int n, const double* a, const double* b, double* partial, double* result, hipStream_t st) {
    hipLaunchKernelGGL(k_dot_partial, dim3(kDotBlocks), dim3(256), 0, st, n, a, b, partial);
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, st, kDotBlocks, partial, result);
}
void launch_cg_alpha(double* sc, hipStream_t st) { hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(64), 0, st, sc); }
void launch_cg_beta(double* sc, hipStream_t st) { hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(64), 0, st, sc); }
void launch_cg_update(int m, const double* sc, const double* p, const double* q, double* y, double* r,
                      hipStream_t st) {
    if (m > 0) hipLaunchKernelGGL(k_cg_update, dim3(nblk(m)), dim3(256), 0, st, m, sc, p, q, y, r);
}
void launch_cg_direction(int m, const double* sc, const double* r, double* p, hipStream_t st) {
    if (m > 0) hipLaunchKernelGGL(k_cg_direction, dim3(nblk(m)), dim3(256), 0, st, m, sc, r, p);
}
void launch_axpy_dev(int n, const double* sc, int idx, double sign, const double* x, double* y,
                     hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_axpy_dev, dim3(nblk(n)), dim3(256), 0, st, n, sc, idx, sign, x, y);
}

}  // namespace ckkt
