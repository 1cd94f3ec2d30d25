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

#include <climits>
#include <cstdint>

#include "device.hpp"

namespace ckkt {

namespace {

constexpr int kWave = 64;

__device__ __forceinline__ double jval(const SysVals& v, int64_t nnzg, int32_t a) {
    return a < nnzg ? v.g_val[a] : v.h_val[a - nnzg];
}

__device__ __forceinline__ unsigned long long ratio_bits(double num, double den) {
    double q;
    if (den > 0.0) q = num / den;
    else q = (num > 0.0) ? __longlong_as_double(0x7FF0000000000000ll) : 0.0;
    if (!(q == q)) q = __longlong_as_double(0x7FF0000000000000ll);  // NaN -> +inf
    return (unsigned long long)__double_as_longlong(q);
}

__device__ __forceinline__ double wave_sum(double x) {
    for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
    return x;
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
__device__ __forceinline__ T pivot_sqrt(T d, int col, int32_t* status);

template <>
__device__ __forceinline__ double pivot_sqrt<double>(double d, int col, int32_t* status) {
    if (!(d > 0.0)) { atomicMin(status, col); return 1.0; }
    return sqrt(d);
}

template <>
__device__ __forceinline__ float pivot_sqrt<float>(float d, int col, int32_t* status) {
    const float floor_ = 1e-5f;
    if (!(d > floor_)) { atomicAdd(status + 1, 1); return sqrtf(floor_); }
    return sqrtf(d);
}

// Small fronts: one workgroup per front, the whole f x f front in LDS.
// Assemble (K columns + extend-add of the children's update matrices in
// child order), partial right-looking Cholesky of the first w columns, then
// store the panel and the update matrix (multifrontal method).
template <typename T>
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
    for (int j = c0; j < c1; ++j) {
        const int jj = j - c0;
        const int t1 = P.kcolptr[j + 1];
        const double sj = scale ? scale[j] : 1.0;
        for (int t = P.kcolptr[j] + tid; t < t1; t += nt) {
            const int pr = P.kmap[t];
            double val = K[t];
            if (scale) val *= sj * scale[P.sn_rows[ro + pr]];
            F[pr + jj * f] = (T)val;
        }
    }
    __syncthreads();
    for (int q = P.child_ptr[s]; q < P.child_ptr[s + 1]; ++q) {
        const int c = P.child_list[q];
        const int wc = P.sn_start[c + 1] - P.sn_start[c];
        const int roc = P.sn_rowptr[c];
        const int rc = P.sn_rowptr[c + 1] - roc - wc;
        const int* rel = P.relmap + roc + wc;
        const T* U = arena + P.u_off[c];
        const int ld = P.u_ld[c];
        for (int idx = tid; idx < rc * rc; idx += nt) {
            const int a = idx % rc, b = idx / rc;
            if (a >= b) F[rel[a] + rel[b] * f] += U[a + (int64_t)b * ld];
        }
        __syncthreads();
    }
    for (int k = 0; k < w; ++k) {
        if (tid == 0) F[k + k * f] = pivot_sqrt<T>(F[k + k * f], c0 + k, status);
        __syncthreads();
        const T dinv = T(1) / F[k + k * f];
        for (int i = k + 1 + tid; i < f; i += nt) F[i + k * f] *= dinv;
        __syncthreads();
        const int mm = f - k - 1;
        for (int idx = tid; idx < mm * mm; idx += nt) {
            const int i = k + 1 + idx % mm, j = k + 1 + idx / mm;
            if (i >= j) F[i + j * f] -= F[i + k * f] * F[j + k * f];
        }
        __syncthreads();
    }
    T* L = arena + P.l_off[s];
    for (int idx = tid; idx < f * w; idx += nt) L[idx] = F[idx];
    T* U = arena + P.u_off[s];
    for (int idx = tid; idx < r * r; idx += nt) {
        const int a = idx % r, b = idx / r;
        if (a >= b) U[idx] = F[(w + a) + (w + b) * f];
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
    for (int j = col0; j < min(col1, w); ++j) {
        const int gj = c0 + j;
        const double sj = scale ? scale[gj] : 1.0;
        for (int t = P.kcolptr[gj] + tid; t < P.kcolptr[gj + 1]; t += nt) {
            const int pr = P.kmap[t];
            double val = K[t];
            if (scale) val *= sj * scale[P.sn_rows[ro + pr]];
            F[pr + (int64_t)j * f] = (T)val;
        }
    }
    __syncthreads();
    for (int q = P.child_ptr[s]; q < P.child_ptr[s + 1]; ++q) {
        const int c = P.child_list[q];
        const int wc = P.sn_start[c + 1] - P.sn_start[c];
        const int roc = P.sn_rowptr[c];
        const int rc = P.sn_rowptr[c + 1] - roc - wc;
        const int* rel = P.relmap + roc + wc;
        // contiguous range of child columns landing in [col0, col1)
        int lo = 0, hi = rc;
        while (lo < hi) { int mid = (lo + hi) >> 1; if (rel[mid] < col0) lo = mid + 1; else hi = mid; }
        const int b0 = lo;
        hi = rc;
        while (lo < hi) { int mid = (lo + hi) >> 1; if (rel[mid] < col1) lo = mid + 1; else hi = mid; }
        const int b1 = lo;
        const int nbc = b1 - b0;
        if (nbc > 0) {
            const T* U = arena + P.u_off[c];
            const int ld = P.u_ld[c];
            for (int idx = tid; idx < nbc * rc; idx += nt) {
                const int b = b0 + idx / rc, a = idx % rc;
                if (a >= b) F[rel[a] + (int64_t)rel[b] * f] += U[a + (int64_t)b * ld];
            }
        }
        __syncthreads();
    }
}

// Large fronts, step 2 (per block column kb): Cholesky of the nb x nb
// diagonal block in LDS, then the triangular solve of the panel below it.
template <typename T>
__global__ void __launch_bounds__(256)
k_big_panel(DevPlan P, T* __restrict__ arena, int list_begin, int kb, int32_t* status) {
    __shared__ T D[kPanelNB * kPanelNB];
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
    for (int k = 0; k < nb; ++k) {
        if (tid == 0) D[k + k * kPanelNB] = pivot_sqrt<T>(D[k + k * kPanelNB], c0 + kb + k, status);
        __syncthreads();
        const T dinv = T(1) / D[k + k * kPanelNB];
        for (int i = k + 1 + tid; i < nb; i += nt) D[i + k * kPanelNB] *= dinv;
        __syncthreads();
        const int mm = nb - k - 1;
        for (int idx = tid; idx < mm * mm; idx += nt) {
            const int i = k + 1 + idx % mm, j = k + 1 + idx / mm;
            if (i >= j) D[i + j * kPanelNB] -= D[i + k * kPanelNB] * D[j + k * kPanelNB];
        }
        __syncthreads();
    }
    for (int idx = tid; idx < nb * nb; idx += nt) {
        const int i = idx % nb, j = idx / nb;
        if (i >= j) F[(kb + i) + (int64_t)(kb + j) * f] = D[i + j * kPanelNB];
    }
    // rows below: X D^T = B
    for (int i = kb + nb + tid; i < f; i += nt) {
        T x[kPanelNB];
#pragma unroll
        for (int j = 0; j < kPanelNB; ++j) x[j] = (j < nb) ? F[i + (int64_t)(kb + j) * f] : T(0);
#pragma unroll
        for (int j = 0; j < kPanelNB; ++j) {
            if (j < nb) {
                x[j] /= D[j + j * kPanelNB];
#pragma unroll
                for (int t = j + 1; t < kPanelNB; ++t)
                    if (t < nb) x[t] -= x[j] * D[t + j * kPanelNB];
            }
        }
#pragma unroll
        for (int j = 0; j < kPanelNB; ++j)
            if (j < nb) F[i + (int64_t)(kb + j) * f] = x[j];
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
// children's update vectors (fixed order), eliminate the w columns over the
// whole front (which also forms this front's update vector), store y and
// the update vector.
template <typename T>
__global__ void __launch_bounds__(256)
k_fwd(DevPlan P, const T* __restrict__ arena, int list_begin, double* __restrict__ v_perm,
      double* __restrict__ uvec) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* v = reinterpret_cast<double*>(smem_raw);
    const int s = P.lvl_all[list_begin + blockIdx.x];
    const int c0 = P.sn_start[s], w = P.sn_start[s + 1] - c0;
    const int ro = P.sn_rowptr[s], f = P.sn_rowptr[s + 1] - ro;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int i = tid; i < f; i += nt) v[i] = (i < w) ? v_perm[c0 + i] : 0.0;
    __syncthreads();
    for (int q = P.child_ptr[s]; q < P.child_ptr[s + 1]; ++q) {
        const int c = P.child_list[q];
        const int wc = P.sn_start[c + 1] - P.sn_start[c];
        const int roc = P.sn_rowptr[c];
        const int rc = P.sn_rowptr[c + 1] - roc - wc;
        const int* rel = P.relmap + roc + wc;
        const double* uc = uvec + roc + wc;
        for (int a = tid; a < rc; a += nt) v[rel[a]] += uc[a];
        __syncthreads();
    }
    const T* L = arena + P.l_off[s];
    for (int k = 0; k < w; ++k) {
        const double yk = v[k] / (double)L[k + (int64_t)k * f];
        __syncthreads();
        if (tid == 0) v[k] = yk;
        for (int i = k + 1 + tid; i < f; i += nt) v[i] -= (double)L[i + (int64_t)k * f] * yk;
        __syncthreads();
    }
    for (int i = tid; i < f; i += nt) {
        if (i < w) v_perm[c0 + i] = v[i];
        else uvec[ro + i] = v[i];
    }
}

// Backward sweep L^T x = y, one workgroup per supernode (levels root to
// leaves): gather the already solved rows below, then back-substitute the
// diagonal block with a workgroup reduction per column.
template <typename T>
__global__ void __launch_bounds__(256)
k_bwd(DevPlan P, const T* __restrict__ arena, int list_begin, double* __restrict__ x_perm) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* z = reinterpret_cast<double*>(smem_raw);
    __shared__ double red[256 / kWave];
    const int s = P.lvl_all[list_begin + blockIdx.x];
    const int c0 = P.sn_start[s], w = P.sn_start[s + 1] - c0;
    const int ro = P.sn_rowptr[s], f = P.sn_rowptr[s + 1] - ro;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int nw = nt / kWave, lane = tid % kWave, wid = tid / kWave;
    for (int i = tid; i < f; i += nt) z[i] = x_perm[P.sn_rows[ro + i]];
    __syncthreads();
    const T* L = arena + P.l_off[s];
    for (int k = w - 1; k >= 0; --k) {
        double part = 0.0;
        for (int i = k + 1 + tid; i < f; i += nt) part += (double)L[i + (int64_t)k * f] * z[i];
        part = wave_sum(part);
        if (lane == 0) red[wid] = part;
        __syncthreads();
        if (tid == 0) {
            double sum = 0.0;
            for (int t = 0; t < nw; ++t) sum += red[t];
            z[k] = (z[k] - sum) / (double)L[k + (int64_t)k * f];
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
__global__ void k_resid_rows(DevPlan P, SysVals v, const double* __restrict__ d,
                             const double* __restrict__ x, const double* __restrict__ rhs2,
                             double* __restrict__ res2, double* __restrict__ t,
                             double* __restrict__ ta, unsigned long long* omega_bits,
                             unsigned long long* resmax_bits) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= P.m) return;
    double acc = 0.0, mag = 0.0;
    for (int a = P.j_ptr[r]; a < P.j_ptr[r + 1]; ++a) {
        double p = jval(v, P.nnzg, a) * x[P.j_col[a]];
        acc += p;
        mag += fabs(p);
    }
    if (P.hy && r < P.m_eq) {
        double res = rhs2[r] - acc;
        res2[r] = res;
        double num = fabs(res);
        atomicMax(omega_bits + P.inst_of_eqrow[r], ratio_bits(num, mag + fabs(rhs2[r])));
        atomicMax(resmax_bits, (unsigned long long)__double_as_longlong(num == num ? num : INFINITY));
    } else {
        double dr = d[r];
        t[r] = dr * acc;
        ta[r] = fabs(dr) * mag;
    }
}

// Residual, pass 2 (one thread per variable): res1 = rhs1 - (W x + sigma_x x
// + sum_{weighted rows} J^T t [+ G^T y]) and the componentwise ratio
// |res1| / (|W||x| + |sigma_x x| + |J|^T ta [+ |G|^T |y|] + |rhs1|).
__global__ void k_resid_vars(DevPlan P, SysVals v, const double* __restrict__ x,
                             const double* __restrict__ y, const double* __restrict__ rhs1,
                             const double* __restrict__ t, const double* __restrict__ ta,
                             double* __restrict__ res1, unsigned long long* omega_bits,
                             unsigned long long* resmax_bits) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
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
    if (P.hy) {
        for (int k = P.jt_ptr[i]; k < gend; ++k) {
            double g = jval(v, P.nnzg, P.jt_vidx[k]);
            double p = g * y[P.jt_row[k]];
            acc += p;
            mag += fabs(p);
        }
        for (int k = gend; k < P.jt_ptr[i + 1]; ++k) {
            double h = jval(v, P.nnzg, P.jt_vidx[k]);
            int r = P.jt_row[k];
            acc += h * t[r];
            mag += fabs(h) * ta[r];
        }
    } else {
        for (int k = P.jt_ptr[i]; k < P.jt_ptr[i + 1]; ++k) {
            double h = jval(v, P.nnzg, P.jt_vidx[k]);
            int r = P.jt_row[k];
            acc += h * t[r];
            mag += fabs(h) * ta[r];
        }
    }
    const double bi = rhs1 ? rhs1[i] : 0.0;
    double res = bi - acc;
    res1[i] = res;
    double num = fabs(res);
    atomicMax(omega_bits + P.inst_of_var[i], ratio_bits(num, mag + fabs(bi)));
    atomicMax(resmax_bits, (unsigned long long)__double_as_longlong(num == num ? num : INFINITY));
}

__global__ void k_maxabs(int n, const double* __restrict__ x, unsigned long long* bits) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double a = fabs(x[i]);
    if (!(a == a)) a = INFINITY;
    atomicMax(bits, (unsigned long long)__double_as_longlong(a));
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
void launch_factor_level(const DevPlan& P, const LevelInfo& L, const double* K, T* arena,
                         int32_t* status, const double* scale, hipStream_t st) {
    if (L.small_count > 0) {
        int threads = L.small_maxf > 24 ? 256 : 64;
        size_t lds = (size_t)L.small_maxf * L.small_maxf * sizeof(T);
        hipLaunchKernelGGL(k_factor_small<T>, dim3(L.small_count), dim3(threads), lds, st, P, K, arena,
                           L.small_begin, status, scale);
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
}

template <typename T>
void launch_fwd_level(const DevPlan& P, const LevelInfo& L, const T* arena, double* v_perm,
                      double* uvec, hipStream_t st) {
    if (L.all_count == 0) return;
    int threads = L.all_maxf > 64 ? 256 : 64;
    hipLaunchKernelGGL(k_fwd<T>, dim3(L.all_count), dim3(threads), (size_t)L.all_maxf * sizeof(double), st, P,
                       arena, L.all_begin, v_perm, uvec);
}

template <typename T>
void launch_bwd_level(const DevPlan& P, const LevelInfo& L, const T* arena, double* x_perm,
                      hipStream_t st) {
    if (L.all_count == 0) return;
    int threads = L.all_maxf > 64 ? 256 : 64;
    hipLaunchKernelGGL(k_bwd<T>, dim3(L.all_count), dim3(threads), (size_t)L.all_maxf * sizeof(double), st, P,
                       arena, L.all_begin, x_perm);
}

template void launch_factor_level<double>(const DevPlan&, const LevelInfo&, const double*, double*, int32_t*,
                                          const double*, hipStream_t);
template void launch_factor_level<float>(const DevPlan&, const LevelInfo&, const double*, float*, int32_t*,
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
