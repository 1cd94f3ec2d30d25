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
#include <climits>
#include <cmath>
#include <cstdint>

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

// Per-block maxima of (ratio, |res|) pushed with one atomic each when the
// whole block belongs to one instance, else one atomic per element.  The
// block must be 256 threads and every thread must call it.
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
            atomicMax(omega_bits + inst, (unsigned long long)__double_as_longlong(ratio));
            atomicMax(resmax_bits, (unsigned long long)__double_as_longlong(num));
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
        atomicMax(omega_bits + s_inst0, (unsigned long long)__double_as_longlong(r));
        atomicMax(resmax_bits, (unsigned long long)__double_as_longlong(nm));
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
__global__ void k_assemble(DevPlan P, SysVals v, const double* __restrict__ d, double* __restrict__ K) {
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
}

__global__ void k_init_status(int32_t* status) {
    if (threadIdx.x == 0 && blockIdx.x == 0) { status[0] = INT_MAX; status[1] = 0; }
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
// preconditioner for the FP64 refinement.
template <typename T>
__device__ __forceinline__ T pivot_root(T d, int col, int32_t* status, bool report);

template <>
__device__ __forceinline__ double pivot_root<double>(double d, int col, int32_t* status, bool report) {
    if (!(d > 0.0)) {
        if (report) atomicMin(status, col);
        return 1.0;
    }
    return sqrt(d);
}

template <>
__device__ __forceinline__ float pivot_root<float>(float d, int col, int32_t* status, bool report) {
    const float floor_ = 1e-5f;
    if (!(d > floor_)) {
        if (report) atomicAdd(status + 1, 1);
        return sqrtf(floor_);
    }
    return sqrtf(d);
}

constexpr int kDiag = 32;  // diagonal block of the blocked front factorization
constexpr int kMaxChildBatch = 64;  // children whose metadata is staged at once

// One wave factors the nb x nb (nb <= 64) diagonal block at A (LDS,
// column-major, leading dimension ld) in place.  Lane i owns row i: it
// reads and writes only its own row, and column k reaches the other lanes
// through shuffles, so no barrier is needed inside.  The caller
// synchronises before and after.
template <typename T>
__device__ void wave_potrf(T* A, int ld, int nb, int col0, int32_t* status) {
    const int lane = threadIdx.x % kWave;
    const bool own = lane < nb;
    for (int k = 0; k < nb; ++k) {
        const T a = (own && lane >= k) ? A[lane + k * ld] : T(0);
        const T akk = __shfl(a, k, kWave);
        const T lkk = pivot_root<T>(akk, col0 + k, status, lane == k);
        const T lik = (lane == k) ? lkk : a / lkk;
        if (own && lane >= k) A[lane + k * ld] = lik;
        for (int j = k + 1; j < nb; ++j) {
            const T ljk = __shfl(lik, j, kWave);
            if (own && lane >= j) A[lane + j * ld] -= lik * ljk;
        }
    }
}

// Rows [i0, i1) of B (column-major, leading dimension ld) times D^{-T} in
// place, D the factored nb x nb diagonal block (leading dimension ldd);
// one thread per row, each thread touching only its own row.
template <typename T>
__device__ void rows_trsm(T* B, int ld, const T* D, int ldd, int nb, int i0, int i1) {
    for (int i = i0 + (int)threadIdx.x; i < i1; i += blockDim.x) {
        for (int j = 0; j < nb; ++j) {
            const T xj = B[i + j * ld] / D[j + j * ldd];
            B[i + j * ld] = xj;
            for (int t = j + 1; t < nb; ++t) B[i + t * ld] -= xj * D[t + j * ldd];
        }
    }
}

// Register variants for wide blocks: the row lives in registers and the
// triangular loops are unrolled, which removes the LDS round trip from every
// step of the dependency chain.  Used for the large-front class only (the
// unrolled code is large).
template <typename T>
__device__ __forceinline__ void wave_potrf_reg(T* A, int ld, int nb, int col0, int32_t* status) {
    const int lane = threadIdx.x % kWave;
    T row[kDiag];
#pragma unroll
    for (int j = 0; j < kDiag; ++j) row[j] = (lane < nb && j < nb && j <= lane) ? A[lane + j * ld] : T(0);
#pragma unroll
    for (int k = 0; k < kDiag; ++k) {
        if (k < nb) {
            const T akk = __shfl(row[k], k, kWave);
            const T lkk = pivot_root<T>(akk, col0 + k, status, lane == k);
            const T lik = (lane == k) ? lkk : row[k] / lkk;
            if (lane >= k) row[k] = lik;
#pragma unroll
            for (int j = k + 1; j < kDiag; ++j) {
                if (j < nb) {
                    const T ljk = __shfl(lik, j, kWave);
                    if (lane >= j) row[j] -= lik * ljk;
                }
            }
        }
    }
    if (lane < nb) {
#pragma unroll
        for (int j = 0; j < kDiag; ++j)
            if (j < nb && j <= lane) A[lane + j * ld] = row[j];
    }
}

template <typename T>
__device__ __forceinline__ void rows_trsm_reg(T* B, int ld, const T* D, int ldd, int nb, int i0, int i1) {
#pragma unroll 1
    for (int i = i0 + (int)threadIdx.x; i < i1; i += blockDim.x) {
        T x[kDiag];
#pragma unroll
        for (int j = 0; j < kDiag; ++j) x[j] = (j < nb) ? B[i + j * ld] : T(0);
#pragma unroll
        for (int j = 0; j < kDiag; ++j) {
            if (j < nb) {
                x[j] /= D[j + j * ldd];
#pragma unroll
                for (int t = j + 1; t < kDiag; ++t)
                    if (t < nb) x[t] -= x[j] * D[t + j * ldd];
            }
        }
#pragma unroll
        for (int j = 0; j < kDiag; ++j)
            if (j < nb) B[i + j * ld] = x[j];
    }
}

// Fronts that fit in LDS (f^2 elements <= 160 KiB): one workgroup per front.
// Assemble (K columns + extend-add of the children's update matrices in
// child order), blocked partial Cholesky of the first w columns (32-column
// diagonal blocks in one wave's registers, parallel row solves and panel
// updates), store the panel, and form the update matrix
// U = F22 - L21 L21^T in one parallel pass (multifrontal method).
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
    for (int i = tid; i < f * f; i += nt) F[i] = T(0);
    __syncthreads();
    // K entries of the w columns: one contiguous slot range
    for (int t = P.kcolptr[c0] + tid; t < P.kcolptr[c1]; t += nt) {
        const int pr = P.kmap[t], j = P.kcol[t];
        double val = K[t];
        if (scale) val *= scale[j] * scale[P.sn_rows[ro + pr]];
        F[pr + (j - c0) * f] = (T)val;
    }
    __syncthreads();
    // extend-add, one child after the other (fixed order), each child's
    // lower update entries in one parallel pass; child metadata prefetched
    {
        __shared__ int64_t c_uoff[kMaxChildBatch];
        __shared__ int c_rel[kMaxChildBatch], c_rc[kMaxChildBatch], c_ld[kMaxChildBatch];
        const int q0 = P.child_ptr[s], nch = P.child_ptr[s + 1] - q0;
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
                for (int idx = tid; idx < rc * rc; idx += nt) {
                    const int a = idx % rc, b = idx / rc;
                    if (a >= b) F[rel[a] + rel[b] * f] += U[a + (int64_t)b * ld];
                }
                __syncthreads();
            }
        }
    }
    for (int kb = 0; kb < w; kb += kDiag) {
        const int nb = min(kDiag, w - kb);
        T* Dg = F + kb + kb * f;
        if (tid < kWave) {
            if (REG) wave_potrf_reg<T>(Dg, f, nb, c0 + kb, status);
            else wave_potrf<T>(Dg, f, nb, c0 + kb, status);
        }
        __syncthreads();
        if (REG) rows_trsm_reg<T>(F + kb * f, f, Dg, f, nb, kb + nb, f);
        else rows_trsm<T>(F + kb * f, f, Dg, f, nb, kb + nb, f);
        __syncthreads();
        // remaining panel columns [kb+nb, w), rows >= column
        const int j0 = kb + nb, mr = f - j0, mc = w - j0;
        for (int idx = tid; idx < mr * mc; idx += nt) {
            const int i = j0 + idx % mr, j = j0 + idx / mr;
            if (i >= j) {
                T acc = F[i + j * f];
                for (int t = 0; t < nb; ++t) acc -= F[i + (kb + t) * f] * F[j + (kb + t) * f];
                F[i + j * f] = acc;
            }
        }
        __syncthreads();
    }
    T* L = arena + P.l_off[s];
    for (int idx = tid; idx < f * w; idx += nt) L[idx] = F[idx];
    T* U = arena + P.u_off[s];
    for (int idx = tid; idx < r * r; idx += nt) {
        const int a = idx % r, b = idx / r;
        if (a >= b) {
            T acc = F[(w + a) + (w + b) * f];
            for (int k = 0; k < w; ++k) acc -= F[(w + a) + k * f] * F[(w + b) + k * f];
            U[idx] = acc;
        }
    }
}

// Large fronts, step 1: one workgroup per 64-column tile of a front kept in
// the arena.  Zero the lower part of the tile, scatter the K entries of its
// columns, then add every child's update entries whose destination column
// lies in the tile (children in fixed order; each entry has one writer).
template <typename T>
__global__ void __launch_bounds__(256)
k_big_init(DevPlan P, const double* __restrict__ K, T* __restrict__ arena, int tile_begin,
           const double* __restrict__ scale) {
    const int tix = tile_begin + blockIdx.x;
    const int s = P.big_tile_sn[tix], col0 = P.big_tile_col[tix];
    const int c0 = P.sn_start[s], w = P.sn_start[s + 1] - c0;
    const int ro = P.sn_rowptr[s], f = P.sn_rowptr[s + 1] - ro;
    const int col1 = min(col0 + kBigTile, f);
    T* F = arena + P.l_off[s];
    const int tid = threadIdx.x, nt = blockDim.x;
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
    const int lane = tid % kWave, wid = tid / kWave, nw = nt / kWave;
    for (int j = col0 + wid; j < col1; j += nw) {
        const int q1 = P.cb_ptr[ro + j + 1];
        for (int q = P.cb_ptr[ro + j]; q < q1; ++q) {
            const int src = P.cb_src[q], len = P.cb_len[q];
            const T* Ucol = arena + P.cb_uoff[q];
            const int* rel = P.relmap + src;
            for (int a = lane; a < len; a += kWave) F[rel[a] + (int64_t)j * f] += Ucol[a];
        }
    }
}

// Large fronts, step 2 (per block column kb): one wave factors the 32 x 32
// diagonal block in LDS, then the rows below are solved in LDS-staged
// chunks of 256 rows (one thread per row).
template <typename T>
__global__ void __launch_bounds__(256)
k_big_panel(DevPlan P, T* __restrict__ arena, int list_begin, int kb, int32_t* status) {
    // one buffer for both, so that the compiler keeps D in LDS instead of
    // hoisting the whole block into registers across the row loop
    __shared__ T buf[kPanelNB * kPanelNB + 256 * kPanelNB];
    T* D = buf;
    T* R = buf + kPanelNB * kPanelNB;
    const int s = P.lvl_big[list_begin + blockIdx.x];
    const int c0 = P.sn_start[s], w = P.sn_start[s + 1] - c0;
    const int f = P.sn_rowptr[s + 1] - P.sn_rowptr[s];
    if (kb >= w) return;
    const int nb = min(kPanelNB, w - kb);
    T* F = arena + P.l_off[s];
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int idx = tid; idx < nb * nb; idx += nt) {
        const int i = idx % nb, j = idx / nb;
        D[i + j * kPanelNB] = (i >= j) ? F[(kb + i) + (int64_t)(kb + j) * f] : T(0);
    }
    __syncthreads();
    if (tid < kWave) wave_potrf_reg<T>(D, kPanelNB, nb, c0 + kb, status);
    __syncthreads();
    for (int idx = tid; idx < nb * nb; idx += nt) {
        const int i = idx % nb, j = idx / nb;
        if (i >= j) F[(kb + i) + (int64_t)(kb + j) * f] = D[i + j * kPanelNB];
    }
#pragma unroll 1
    for (int r0 = kb + nb; r0 < f; r0 += 256) {
        const int nr = min(256, f - r0);
        for (int idx = tid; idx < nr * nb; idx += nt) {
            const int i = idx % nr, j = idx / nr;
            R[i + j * 256] = F[(r0 + i) + (int64_t)(kb + j) * f];
        }
        __syncthreads();
        rows_trsm_reg<T>(R, 256, D, kPanelNB, nb, 0, nr);
        __syncthreads();
        for (int idx = tid; idx < nr * nb; idx += nt) {
            const int i = idx % nr, j = idx / nr;
            F[(r0 + i) + (int64_t)(kb + j) * f] = R[i + j * 256];
        }
        __syncthreads();
    }
}

// Large fronts, step 3: trailing update C -= P P^T of the lower triangle
// below the panel, one 64 x 64 tile per workgroup (grid: tile row, tile
// column, front).
template <typename T>
__global__ void __launch_bounds__(256)
k_big_update(DevPlan P, T* __restrict__ arena, int list_begin, int kb) {
    __shared__ T A[64][kPanelNB + 1];
    __shared__ T B[64][kPanelNB + 1];
    const int s = P.lvl_big[list_begin + blockIdx.z];
    const int w = P.sn_start[s + 1] - P.sn_start[s];
    const int f = P.sn_rowptr[s + 1] - P.sn_rowptr[s];
    if (kb >= w) return;
    const int ti = blockIdx.x, tj = blockIdx.y;
    if (tj > ti) return;
    const int nb = min(kPanelNB, w - kb);
    const int base = kb + nb;
    const int i0 = base + ti * 64, j0 = base + tj * 64;
    if (i0 >= f) return;
    T* F = arena + P.l_off[s];
    const int tid = threadIdx.x;
    for (int idx = tid; idx < 64 * kPanelNB; idx += 256) {
        const int ii = idx % 64, t = idx / 64;
        const int gi = i0 + ii, gj = j0 + ii;
        A[ii][t] = (gi < f && t < nb) ? F[gi + (int64_t)(kb + t) * f] : T(0);
        B[ii][t] = (gj < f && t < nb) ? F[gj + (int64_t)(kb + t) * f] : T(0);
    }
    __syncthreads();
    const int tx = tid % 16, ty = tid / 16;
    T acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = T(0);
    for (int t = 0; t < nb; ++t) {
        T av[4], bv[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) av[a] = A[tx + 16 * a][t];
#pragma unroll
        for (int b = 0; b < 4; ++b) bv[b] = B[ty + 16 * b][t];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] += av[a] * bv[b];
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int col = j0 + ty + 16 * b;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int row = i0 + tx + 16 * a;
            if (row < f && col < f && row >= col) F[row + (int64_t)col * f] -= acc[a][b];
        }
    }
}

// ---------------------------------------------------------------- sweeps

// Forward sweep L y = b, one workgroup per supernode of a level: gather the
// children's update vectors (fixed order), then per block of 64 columns one
// wave solves the diagonal block with lane shuffles and the workgroup
// applies the block to every row below it; rows beyond the supernode's own
// columns end up holding this front's update vector.
template <typename T>
__global__ void __launch_bounds__(256)
k_fwd(DevPlan P, const T* __restrict__ arena, int list_begin, int ldd, double* __restrict__ v_perm,
      double* __restrict__ uvec) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* v = reinterpret_cast<double*>(smem_raw);
    const int s = P.lvl_all[list_begin + blockIdx.x];
    const int c0 = P.sn_start[s], w = P.sn_start[s + 1] - c0;
    const int ro = P.sn_rowptr[s], f = P.sn_rowptr[s + 1] - ro;
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid % kWave, wid = tid / kWave;
    for (int i = tid; i < f; i += nt) {
        double acc = (i < w) ? v_perm[c0 + i] : 0.0;
        const int q1 = P.cb_ptr[ro + i + 1];
        for (int q = P.cb_ptr[ro + i]; q < q1; ++q) acc += uvec[P.cb_src[q]];
        v[i] = acc;
    }
    __syncthreads();
    const T* L = arena + P.l_off[s];
    double* D = v + ((f + 1) & ~1);  // nb x nb diagonal block, column-major, ld kWave
    for (int kb = 0; kb < w; kb += kWave) {
        const int nb = min(kWave, w - kb);
        for (int idx = tid; idx < nb * nb; idx += nt) {
            const int i = idx % nb, k = idx / nb;
            D[i + k * ldd] = (i >= k) ? (double)L[(kb + i) + (int64_t)(kb + k) * f] : 0.0;
        }
        __syncthreads();
        if (wid == 0) {
            double vi = lane < nb ? v[kb + lane] : 0.0;
            for (int k = 0; k < nb; ++k) {
                const double yk = __shfl(vi, k, kWave) / D[k + k * ldd];
                if (lane == k) vi = yk;
                else if (lane > k) vi -= D[lane + k * ldd] * yk;
            }
            if (lane < nb) v[kb + lane] = vi;
        }
        __syncthreads();
        for (int i = kb + nb + tid; i < f; i += nt) {
            double acc = 0.0;
            const T* Li = L + i + (int64_t)kb * f;
            for (int k = 0; k < nb; ++k) acc += (double)Li[(int64_t)k * f] * v[kb + k];
            v[i] -= acc;
        }
        __syncthreads();
    }
    for (int i = tid; i < f; i += nt) {
        if (i < w) v_perm[c0 + i] = v[i];
        else uvec[ro + i] = v[i];
    }
}

// Backward sweep L^T x = y, one workgroup per supernode (levels root to
// leaves): gather the already solved rows below, then per block of 64
// columns (last block first) form the dot products with everything solved
// so far (one wave per column) and back-substitute the diagonal block in
// one wave with lane shuffles.
template <typename T>
__global__ void __launch_bounds__(256)
k_bwd(DevPlan P, const T* __restrict__ arena, int list_begin, int ldd, double* __restrict__ x_perm) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* z = reinterpret_cast<double*>(smem_raw);
    __shared__ double tb[kWave];
    const int s = P.lvl_all[list_begin + blockIdx.x];
    const int c0 = P.sn_start[s], w = P.sn_start[s + 1] - c0;
    const int ro = P.sn_rowptr[s], f = P.sn_rowptr[s + 1] - ro;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int nw = nt / kWave, lane = tid % kWave, wid = tid / kWave;
    double* D = z + ((f + 1) & ~1);
    for (int i = tid; i < f; i += nt) z[i] = x_perm[P.sn_rows[ro + i]];
    __syncthreads();
    const T* L = arena + P.l_off[s];
    const int nblk = (w + kWave - 1) / kWave;
    for (int b = nblk - 1; b >= 0; --b) {
        const int kb = b * kWave, nb = min(kWave, w - kb), r0 = kb + nb;
        for (int k = wid; k < nb; k += nw) {
            const T* col = L + (int64_t)(kb + k) * f;
            double part = 0.0;
            for (int i = r0 + lane; i < f; i += kWave) part += (double)col[i] * z[i];
            part = wave_sum(part);
            if (lane == 0) tb[k] = part;
        }
        __syncthreads();
        // diagonal block, stored transposed: D[k + j * kWave] = L(kb+k, kb+j)
        for (int idx = tid; idx < nb * nb; idx += nt) {
            const int k = idx % nb, j = idx / nb;
            D[k + j * ldd] = (k >= j) ? (double)L[(kb + k) + (int64_t)(kb + j) * f] : 0.0;
        }
        __syncthreads();
        if (wid == 0) {
            double ri = lane < nb ? z[kb + lane] - tb[lane] : 0.0;
            for (int k = nb - 1; k >= 0; --k) {
                const double xk = __shfl(ri, k, kWave) / D[k + k * ldd];
                if (lane == k) ri = xk;
                else if (lane < k) ri -= D[k + lane * ldd] * xk;
            }
            if (lane < nb) z[kb + lane] = ri;
        }
        __syncthreads();
    }
    for (int i = tid; i < w; i += nt) x_perm[c0 + i] = z[i];
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

// Residual, pass 1 (one thread per constraint row): for rows weighted by d
// (LiftedKKT all rows; HyKKT rows of H) t = d (J x) and ta = |d| (|J||x|);
// for HyKKT rows of G the K1 second-block residual rhs2 - G x and its
// componentwise ratio.
__global__ void __launch_bounds__(256)
k_resid_rows(DevPlan P, SysVals v, const double* __restrict__ d, const double* __restrict__ x,
             const double* __restrict__ rhs2, double* __restrict__ res2, double* __restrict__ t,
             double* __restrict__ ta, unsigned long long* omega_bits, unsigned long long* resmax_bits) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = r < P.m;
    double acc = 0.0, mag = 0.0;
    if (in) {
        for (int a = P.j_ptr[r]; a < P.j_ptr[r + 1]; ++a) {
            double p = jval(v, P.nnzg, a) * x[P.j_col[a]];
            acc += p;
            mag += fabs(p);
        }
    }
    const bool eq = in && P.hy && r < P.m_eq;
    double ratio = 0.0, num = 0.0;
    int inst = -1;
    if (eq) {
        double res = rhs2[r] - acc;
        res2[r] = res;
        num = fabs(res);
        double den = mag + fabs(rhs2[r]);
        ratio = den > 0.0 ? num / den : (num > 0.0 ? INFINITY : 0.0);
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
        double acc = 0.0, mag = 0.0;
        for (int k = P.wf_ptr[i]; k < P.wf_ptr[i + 1]; ++k) {
            double p = v.w_val[P.wf_vidx[k]] * x[P.wf_col[k]];
            acc += p;
            mag += fabs(p);
        }
        double px = v.sigma_x[i] * x[i];
        acc += px;
        mag += fabs(px);
        const int gend = P.jt_gend[i];
        int k0 = P.jt_ptr[i];
        if (P.hy) {
            for (int k = k0; k < gend; ++k) {
                double p = jval(v, P.nnzg, P.jt_vidx[k]) * y[P.jt_row[k]];
                acc += p;
                mag += fabs(p);
            }
            k0 = gend;
        }
        for (int k = k0; k < P.jt_ptr[i + 1]; ++k) {
            double h = jval(v, P.nnzg, P.jt_vidx[k]);
            int r = P.jt_row[k];
            acc += h * t[r];
            mag += fabs(h) * ta[r];
        }
        const double bi = rhs1 ? rhs1[i] : 0.0;
        double res = bi - acc;
        res1[i] = res;
        num = fabs(res);
        double den = mag + fabs(bi);
        ratio = den > 0.0 ? num / den : (num > 0.0 ? INFINITY : 0.0);
        inst = P.inst_of_var[i];
    }
    block_max_push(in, inst, ratio, num, omega_bits, resmax_bits);
}

__global__ void __launch_bounds__(256) k_maxabs(int n, const double* __restrict__ x, unsigned long long* bits) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double a = i < n ? nan_to_inf(fabs(x[i])) : 0.0;
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

__global__ void k_copy(int n, const double* __restrict__ x, double* __restrict__ y) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = x[i];
}

__global__ void k_fill(int n, double val, double* __restrict__ y) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = val;
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
    double acc = 0.0;
    for (int a = P.j_ptr[r]; a < P.j_ptr[r + 1]; ++a) acc += v.g_val[a] * x[P.j_col[a]];
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

}  // namespace

// ================================================================ launchers

void launch_row_weights(const DevPlan& P, const SysVals& v, double* d, hipStream_t st) {
    if (P.m == 0) return;
    hipLaunchKernelGGL(k_row_weights, dim3(nblk(P.m)), dim3(256), 0, st, P, v, d);
}

void launch_assemble(const DevPlan& P, const SysVals& v, const double* d, double* K, hipStream_t st) {
    if (P.nnzk == 0) return;
    hipLaunchKernelGGL(k_assemble, dim3(nblk(P.nnzk)), dim3(256), 0, st, P, v, d, K);
}

void launch_init_status(int32_t* status, hipStream_t st) {
    hipLaunchKernelGGL(k_init_status, dim3(1), dim3(64), 0, st, status);
}

void launch_diag_scale(const DevPlan& P, const double* K, double* scale, hipStream_t st) {
    if (P.n == 0) return;
    hipLaunchKernelGGL(k_diag_scale, dim3(nblk(P.n)), dim3(256), 0, st, P, K, scale);
}

template <typename T>
bool launch_factor_level(const DevPlan& P, const LevelInfo& L, const double* K, T* arena,
                         int32_t* status, const double* scale, hipStream_t st) {
    if ((size_t)L.small_maxf * L.small_maxf * sizeof(T) + kFactorStaticLds > (size_t)kLdsBytes) return false;
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_factor_small<T, true>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_factor_small<T, false>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        attr_set = true;
    }
    if (L.small_count > 0) {
        // two LDS size classes so that small fronts keep several workgroups
        // per CU; one wave per front when the class is tiny
        const bool d = sizeof(T) == 8;
        const int na = d ? L.small_split : L.small_split32;
        const int fa = d ? L.small_maxf_a : L.small_maxf_a32;
        const int nbig = L.small_count - na;
        if (na > 0)
            hipLaunchKernelGGL((k_factor_small<T, false>), dim3(na), dim3(L.small_threads_a),
                               (size_t)fa * fa * sizeof(T), st, P, K, arena, L.small_begin, status, scale);
        if (nbig > 0) {
            size_t lds = (size_t)L.small_maxf * L.small_maxf * sizeof(T);
            hipLaunchKernelGGL((k_factor_small<T, true>), dim3(nbig), dim3(256), lds, st, P, K, arena,
                               L.small_begin + na, status, scale);
        }
    }
    if (L.big_count > 0) {
        hipLaunchKernelGGL(k_big_init<T>, dim3(L.tile_count), dim3(256), 0, st, P, K, arena, L.tile_begin,
                           scale);
        for (int kb = 0; kb < L.big_maxw; kb += kPanelNB) {
            hipLaunchKernelGGL(k_big_panel<T>, dim3(L.big_count), dim3(256), 0, st, P, arena, L.big_begin,
                               kb, status);
            int rest = L.big_maxf - kb - 1;  // upper bound of trailing rows
            int tiles = rest > 0 ? (rest + 63) / 64 : 0;
            if (tiles > 0)
                hipLaunchKernelGGL(k_big_update<T>, dim3(tiles, tiles, L.big_count), dim3(256), 0, st, P,
                                   arena, L.big_begin, kb);
        }
    }
    return true;
}

template <typename T>
void launch_fwd_level(const DevPlan& P, const LevelInfo& L, const T* arena, double* v_perm,
                      double* uvec, hipStream_t st) {
    if (L.all_count == 0) return;
    const int threads = L.sweep_threads;
    const int ldd = std::min(kWave, std::max(L.all_maxw, 1));
    size_t lds = (size_t)(((L.all_maxf + 1) & ~1) + ldd * ldd) * sizeof(double);
    hipLaunchKernelGGL(k_fwd<T>, dim3(L.all_count), dim3(threads), lds, st, P, arena, L.all_begin, ldd, v_perm,
                       uvec);
}

template <typename T>
void launch_bwd_level(const DevPlan& P, const LevelInfo& L, const T* arena, double* x_perm,
                      hipStream_t st) {
    if (L.all_count == 0) return;
    const int threads = L.sweep_threads;
    const int ldd = std::min(kWave, std::max(L.all_maxw, 1));
    size_t lds = (size_t)(((L.all_maxf + 1) & ~1) + ldd * ldd) * sizeof(double);
    hipLaunchKernelGGL(k_bwd<T>, dim3(L.all_count), dim3(threads), lds, st, P, arena, L.all_begin, ldd, x_perm);
}

template bool launch_factor_level<double>(const DevPlan&, const LevelInfo&, const double*, double*, int32_t*,
                                          const double*, hipStream_t);
template bool launch_factor_level<float>(const DevPlan&, const LevelInfo&, const double*, float*, int32_t*,
                                         const double*, hipStream_t);
template void launch_fwd_level<double>(const DevPlan&, const LevelInfo&, const double*, double*, double*,
                                       hipStream_t);
template void launch_fwd_level<float>(const DevPlan&, const LevelInfo&, const float*, double*, double*,
                                      hipStream_t);
template void launch_bwd_level<double>(const DevPlan&, const LevelInfo&, const double*, double*, hipStream_t);
template void launch_bwd_level<float>(const DevPlan&, const LevelInfo&, const float*, double*, hipStream_t);

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

void launch_residual(const DevPlan& P, const SysVals& v, const double* d, const double* x,
                     const double* y, const double* rhs1, const double* rhs2, double* res1,
                     double* res2, double* tbuf, double* tabuf, unsigned long long* omega_bits,
                     unsigned long long* resmax_bits, hipStream_t st) {
    if (P.m > 0)
        hipLaunchKernelGGL(k_resid_rows, dim3(nblk(P.m)), dim3(256), 0, st, P, v, d, x, rhs2, res2, tbuf, tabuf,
                           omega_bits, resmax_bits);
    if (P.n > 0)
        hipLaunchKernelGGL(k_resid_vars, dim3(nblk(P.n)), dim3(256), 0, st, P, v, x, y, rhs1, tbuf, tabuf, res1,
                           omega_bits, resmax_bits);
}

void launch_maxabs(int n, const double* x, unsigned long long* bits, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_maxabs, dim3(nblk(n)), dim3(256), 0, st, n, x, bits);
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
void launch_gt(const DevPlan& P, const SysVals& v, const double* base, double scale, const double* y,
               double* out, hipStream_t st) {
    if (P.n > 0) hipLaunchKernelGGL(k_gt, dim3(nblk(P.n)), dim3(256), 0, st, P, v, base, scale, y, out);
}
void launch_g(const DevPlan& P, const SysVals& v, const double* x, const double* sub, double* out,
              hipStream_t st) {
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
