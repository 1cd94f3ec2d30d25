// Learned diagonal preconditioner: per-variable features, the 8-64-64-1
// tanh MLP (forward, backward, weight gradients, Adam) and the vector work
// of PCG around a stale factor with M^{-1} = D K_s^{-1} D, D = diag(exp(o)).
//
// Parameter layout (FP32): W1[64][8] row-major, b1[64], W2[64][64], b2[64],
// w3[64], b3.  All reductions are fixed-order (per-block partial sums, then
// one ordered pass), so training is bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "device.hpp"

namespace ckkt {

namespace {

constexpr int F = kMlpF, H = kMlpH;
constexpr int oW1 = 0, oB1 = H * F, oW2 = oB1 + H, oB2 = oW2 + H * H, oW3 = oB2 + H, oB3 = oW3 + H;
static_assert(oB3 + 1 == kMlpNParam, "parameter layout");

__device__ __forceinline__ double jv(const SysVals& v, int64_t nnzg, int32_t a) {
    return a < nnzg ? v.g_val[a] : v.h_val[a - nnzg];
}

__device__ __forceinline__ double lg10(double x) { return log10(fmax(x, 1e-30)); }

// diag(K) = diag(W) + sigma_x + sum_r d_r J_rj^2 from the unassembled data
__global__ void k_kdiag(DevPlan P, SysVals v, const double* __restrict__ d, double* __restrict__ kd) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    double acc = 0.0;
    for (int k = P.wf_ptr[i]; k < P.wf_ptr[i + 1]; ++k)
        if (P.wf_col[k] == i) acc += v.w_val[P.wf_vidx[k]];
    acc += v.sigma_x[i];
    for (int k = P.jt_ptr[i]; k < P.jt_ptr[i + 1]; ++k) {
        const double a = jv(v, P.nnzg, P.jt_vidx[k]);
        acc += d[P.jt_row[k]] * a * a;
    }
    kd[i] = acc;
}

// features f0..f7 of each variable (new system vs the stale one)
__global__ void k_features(DevPlan P, const double* __restrict__ sx_new, const double* __restrict__ d_new,
                           const double* __restrict__ kd_new, const double* __restrict__ sx_old,
                           const double* __restrict__ d_old, const double* __restrict__ kd_old,
                           float* __restrict__ feat) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    const double ls = lg10(sx_new[i]), lk = lg10(kd_new[i]);
    double f4 = 0.0, f5 = 0.0, f6 = 0.0;
    const int k0 = P.jt_ptr[i], k1 = P.jt_ptr[i + 1];
    if (k1 > k0) {
        f4 = -INFINITY; f5 = -INFINITY; f6 = INFINITY;
        for (int k = k0; k < k1; ++k) {
            const int r = P.jt_row[k];
            const double ln = lg10(d_new[r]);
            const double ch = ln - lg10(d_old[r]);
            f4 = fmax(f4, ln);
            f5 = fmax(f5, ch);
            f6 = fmin(f6, ch);
        }
    }
    float* o = feat + (int64_t)i * F;
    o[0] = (float)(ls / 8.0);
    o[1] = (float)((ls - lg10(sx_old[i])) / 8.0);
    o[2] = (float)(lk / 8.0);
    o[3] = (float)((lk - lg10(kd_old[i])) / 8.0);
    o[4] = (float)(f4 / 8.0);
    o[5] = (float)(f5 / 8.0);
    o[6] = (float)(f6 / 8.0);
    o[7] = 1.0f;
}

// Forward: one thread per variable, parameters staged in LDS.
__global__ void __launch_bounds__(256)
k_mlp_fwd(int64_t n, const float* __restrict__ feat, const float* __restrict__ prm, float* __restrict__ out,
          float* __restrict__ cache) {
    __shared__ float w[kMlpNParam];
    for (int t = threadIdx.x; t < kMlpNParam; t += blockDim.x) w[t] = prm[t];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float f[F];
#pragma unroll
    for (int c = 0; c < F; ++c) f[c] = feat[i * F + c];
    float h1[H];
#pragma unroll
    for (int h = 0; h < H; ++h) {
        float a = w[oB1 + h];
#pragma unroll
        for (int c = 0; c < F; ++c) a += w[oW1 + h * F + c] * f[c];
        h1[h] = tanhf(a);
    }
    float o = w[oB3];
    for (int h = 0; h < H; ++h) {
        float a = w[oB2 + h];
#pragma unroll
        for (int c = 0; c < H; ++c) a += w[oW2 + h * H + c] * h1[c];
        const float h2 = tanhf(a);
        o += w[oW3 + h] * h2;
        if (cache) cache[(int64_t)H * n + i * H + h] = h2;
    }
    if (cache) {
#pragma unroll
        for (int h = 0; h < H; ++h) cache[i * H + h] = h1[h];
    }
    out[i] = o;
}

// Backward through the activations, one thread per variable:
// ga2 = g_o w3 (1 - h2^2), ga1 = (W2^T ga2)(1 - h1^2)
__global__ void __launch_bounds__(256)
k_mlp_bwd_rows(int64_t n, const float* __restrict__ prm, const float* __restrict__ cache,
               const float* __restrict__ g_o, float* __restrict__ ga) {
    __shared__ float w[kMlpNParam];
    for (int t = threadIdx.x; t < kMlpNParam; t += blockDim.x) w[t] = prm[t];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float go = g_o[i];
    float a2[H];
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const float h2 = cache[(int64_t)H * n + i * H + h];
        a2[h] = go * w[oW3 + h] * (1.0f - h2 * h2);
        ga[(int64_t)H * n + i * H + h] = a2[h];
    }
    for (int c = 0; c < H; ++c) {
        float a = 0.0f;
#pragma unroll
        for (int h = 0; h < H; ++h) a += w[oW2 + h * H + c] * a2[h];
        const float h1 = cache[i * H + c];
        ga[i * H + c] = a * (1.0f - h1 * h1);
    }
}

constexpr int kRowsPerBlock = 256;

// Weight gradients: each block sums its rows' contributions to every
// parameter (rows in order), one partial vector per block.
__global__ void __launch_bounds__(256)
k_mlp_wgrad(int64_t n, const float* __restrict__ feat, const float* __restrict__ cache,
            const float* __restrict__ ga, const float* __restrict__ g_o, float* __restrict__ partial) {
    const int64_t r0 = (int64_t)blockIdx.x * kRowsPerBlock;
    const int64_t r1 = min((int64_t)n, r0 + kRowsPerBlock);
    for (int p = threadIdx.x; p < kMlpNParam; p += blockDim.x) {
        float acc = 0.0f;
        if (p < oB1) {                    // W1[h][c]
            const int h = p / F, c = p % F;
            for (int64_t i = r0; i < r1; ++i) acc += ga[i * H + h] * feat[i * F + c];
        } else if (p < oW2) {             // b1
            const int h = p - oB1;
            for (int64_t i = r0; i < r1; ++i) acc += ga[i * H + h];
        } else if (p < oB2) {             // W2[h][c]
            const int h = (p - oW2) / H, c = (p - oW2) % H;
            for (int64_t i = r0; i < r1; ++i) acc += ga[(int64_t)H * n + i * H + h] * cache[i * H + c];
        } else if (p < oW3) {             // b2
            const int h = p - oB2;
            for (int64_t i = r0; i < r1; ++i) acc += ga[(int64_t)H * n + i * H + h];
        } else if (p < oB3) {             // w3
            const int h = p - oW3;
            for (int64_t i = r0; i < r1; ++i) acc += g_o[i] * cache[(int64_t)H * n + i * H + h];
        } else {                          // b3
            for (int64_t i = r0; i < r1; ++i) acc += g_o[i];
        }
        partial[(int64_t)blockIdx.x * kMlpNParam + p] = acc;
    }
}

__global__ void k_mlp_reduce(int nblocks, const float* __restrict__ partial, float* __restrict__ grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kMlpNParam) return;
    double acc = 0.0;
    for (int b = 0; b < nblocks; ++b) acc += partial[(int64_t)b * kMlpNParam + p];
    grad[p] = (float)acc;
}

__global__ void k_adam(int np, float* __restrict__ prm, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int step, float lr, float b1, float b2, float eps) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const float gi = g[p];
    const float mi = b1 * m[p] + (1.0f - b1) * gi;
    const float vi = b2 * v[p] + (1.0f - b2) * gi * gi;
    m[p] = mi;
    v[p] = vi;
    const float mh = mi / (1.0f - powf(b1, (float)step));
    const float vh = vi / (1.0f - powf(b2, (float)step));
    prm[p] -= lr * mh / (sqrtf(vh) + eps);
}

// out = exp(clamp(o)) * x   (D applied to a vector)
__global__ void k_dscale(int n, const float* __restrict__ o, const double* __restrict__ x, double* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double oi = o ? (double)o[i] : 0.0;
    out[i] = exp(fmin(fmax(oi, -20.0), 20.0)) * x[i];
}

// e = D y - x ; returns e in place of z
__global__ void k_train_err(int n, const float* __restrict__ o, const double* __restrict__ y,
                            const double* __restrict__ x, double* __restrict__ e) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    e[i] = exp(fmin(fmax((double)o[i], -20.0), 20.0)) * y[i] - x[i];
}

// g_o = (g_z y + b w) D [|o| < 20], g_z = 2 e / ||x||^2 with sc[0] = e.e, sc[1] = x.x
__global__ void k_train_go(int n, const float* __restrict__ o, const double* __restrict__ e,
                           const double* __restrict__ y, const double* __restrict__ b, const double* __restrict__ w,
                           const double* __restrict__ sc, float* __restrict__ g_o) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double oi = (double)o[i];
    const double D = exp(fmin(fmax(oi, -20.0), 20.0));
    const double gz = 2.0 * e[i] / sc[1];
    const double gD = gz * y[i] + b[i] * w[i];
    g_o[i] = (fabs(oi) < 20.0) ? (float)(gD * D) : 0.0f;
}

// g_z D, the right-hand side of the second stale solve
__global__ void k_train_gzD(int n, const float* __restrict__ o, const double* __restrict__ e,
                            const double* __restrict__ sc, double* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = 2.0 * e[i] / sc[1] * exp(fmin(fmax((double)o[i], -20.0), 20.0));
}

inline int nb(int64_t n) { return (int)((n + 255) / 256); }

}  // namespace

void launch_kdiag(const DevPlan& P, const SysVals& v, const double* d, double* kd, hipStream_t st) {
    if (P.n > 0) hipLaunchKernelGGL(k_kdiag, dim3(nb(P.n)), dim3(256), 0, st, P, v, d, kd);
}
void launch_features(const DevPlan& P, const double* sx_new, const double* d_new, const double* kd_new,
                     const double* sx_old, const double* d_old, const double* kd_old, float* feat, hipStream_t st) {
    if (P.n > 0)
        hipLaunchKernelGGL(k_features, dim3(nb(P.n)), dim3(256), 0, st, P, sx_new, d_new, kd_new, sx_old, d_old,
                           kd_old, feat);
}
void launch_mlp_forward(int64_t n, const float* feat, const float* prm, float* out, float* cache, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_mlp_fwd, dim3(nb(n)), dim3(256), 0, st, n, feat, prm, out, cache);
}
constexpr int64_t mlp_workspace_floats(int64_t n) {
    return 2 * H * n + (n + kRowsPerBlock - 1) / kRowsPerBlock * (int64_t)kMlpNParam + 64;
}
size_t mlp_workspace_bytes(int64_t n) { return (size_t)mlp_workspace_floats(n) * sizeof(float); }

namespace {
// Scratch of ckkt_mlp_backward_noalloc: the backward's workspace for up to
// kMlpNoAllocRows rows (activation gradients, one partial gradient per
// 256-row block) in a file-scope device array, so that the call allocates
// nothing.  Every kernel writes the scratch it later reads, so nothing has
// to be cleared between calls.  Each device holds its own copy of the
// array; host code uses only the address returned for the current device.
static __device__ __align__(256) float scratch[mlp_workspace_floats(kMlpNoAllocRows)];
constexpr int kMaxDevices = 64;
}  // namespace

void* mlp_noalloc_scratch(hipError_t* err) {
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        *err = e != hipSuccess ? e : hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
            return nullptr;
        }
        addr[dev] = p;
    }
    *err = hipSuccess;
    return addr[dev];
}
void launch_mlp_backward(int64_t n, const float* feat, const float* prm, const float* cache, const float* g_o,
                         float* grad, void* ws, hipStream_t st) {
    float* ga = static_cast<float*>(ws);
    const int64_t nblocks = (n + kRowsPerBlock - 1) / kRowsPerBlock;
    float* partial = ga + 2 * H * n;
    if (n > 0) {
        hipLaunchKernelGGL(k_mlp_bwd_rows, dim3(nb(n)), dim3(256), 0, st, n, prm, cache, g_o, ga);
        hipLaunchKernelGGL(k_mlp_wgrad, dim3((int)nblocks), dim3(256), 0, st, n, feat, cache, ga, g_o, partial);
    }
    hipLaunchKernelGGL(k_mlp_reduce, dim3(nb(kMlpNParam)), dim3(256), 0, st, (int)nblocks, partial, grad);
}
void launch_adam(int np, float* prm, const float* g, float* m, float* v, int step, float lr, hipStream_t st) {
    if (np > 0)
        hipLaunchKernelGGL(k_adam, dim3(nb(np)), dim3(256), 0, st, np, prm, g, m, v, step, lr, 0.9f, 0.999f, 1e-8f);
}
void launch_dscale(int n, const float* o, const double* x, double* out, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_dscale, dim3(nb(n)), dim3(256), 0, st, n, o, x, out);
}
void launch_train_err(int n, const float* o, const double* y, const double* x, double* e, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_train_err, dim3(nb(n)), dim3(256), 0, st, n, o, y, x, e);
}
void launch_train_gzD(int n, const float* o, const double* e, const double* sc, double* out, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_train_gzD, dim3(nb(n)), dim3(256), 0, st, n, o, e, sc, out);
}
void launch_train_go(int n, const float* o, const double* e, const double* y, const double* b, const double* w,
                     const double* sc, float* g_o, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_train_go, dim3(nb(n)), dim3(256), 0, st, n, o, e, y, b, w, sc, g_o);
}

}  // namespace ckkt
