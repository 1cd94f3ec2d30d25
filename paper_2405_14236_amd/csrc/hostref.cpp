// Sequential host execution of the numeric phases over the analysis plan:
// the same assembly recipe, multifrontal factor layout, extend-add maps,
// level schedule and sweep update vectors as the HIP kernels, one front at
// a time.  It lets the analysis be validated on machines without a GPU; it
// is not used by the device path.
#include <cmath>
#include <cstdint>
#include <vector>

#include "analysis.hpp"

namespace ckkt {

int host_factor_solve(const Plan& P, int hy, const double* w_val, const double* g_val, const double* h_val,
                      const double* sigma_x, const double* sigma_s, double gamma, const double* b, double* x) {
    const int n = P.n, m = P.m;
    std::vector<double> d(m);
    for (int r = 0; r < m; ++r) d[r] = hy ? (r < P.m_eq ? gamma : sigma_s[r - P.m_eq]) : sigma_s[r];
    auto jv = [&](int a) { return a < P.nnz_g ? g_val[a] : h_val[a - P.nnz_g]; };
    const int64_t nnzk = P.kcolptr[n];
    std::vector<double> K(nnzk);
    for (int64_t t = 0; t < nnzk; ++t) {
        double acc = 0.0;
        if (P.k_wsrc[t] >= 0) acc = w_val[P.k_wsrc[t]];
        if (P.k_diag[t] >= 0) acc += sigma_x[P.k_diag[t]];
        for (int q = P.prod_ptr[t]; q < P.prod_ptr[t + 1]; ++q)
            acc += d[P.prod_r[q]] * (jv(P.prod_a[q]) * jv(P.prod_b[q]));
        K[t] = acc;
    }
    std::vector<double> arena(P.arena, 0.0);
    int failed = -1;
    std::vector<double> F;
    for (int l = 0; l < P.nlev; ++l)
        for (int t = P.lvl_all_ptr[l]; t < P.lvl_all_ptr[l + 1]; ++t) {
            const int s = P.lvl_all[t];
            const int c0 = P.sn_start[s], w = P.sn_start[s + 1] - c0;
            const int ro = P.sn_rowptr[s], f = P.sn_rowptr[s + 1] - ro, r = f - w;
            F.assign((size_t)f * f, 0.0);
            for (int j = c0; j < c0 + w; ++j)
                for (int u = P.kcolptr[j]; u < P.kcolptr[j + 1]; ++u) F[P.kmap[u] + (size_t)(j - c0) * f] = K[u];
            for (int j = 0; j < f; ++j)
                for (int q = P.cb_ptr[ro + j]; q < P.cb_ptr[ro + j + 1]; ++q) {
                    const double* Ucol = arena.data() + P.cb_uoff[q];
                    const int* rel = P.relmap.data() + P.cb_src[q];
                    for (int a = 0; a < P.cb_len[q]; ++a) F[rel[a] + (size_t)j * f] += Ucol[a];
                }
            for (int k = 0; k < w; ++k) {
                double dk = F[k + (size_t)k * f];
                if (!(dk > 0.0)) { if (failed < 0) failed = P.perm[c0 + k]; dk = 1.0; }
                dk = std::sqrt(dk);
                F[k + (size_t)k * f] = dk;
                for (int i = k + 1; i < f; ++i) F[i + (size_t)k * f] /= dk;
                for (int j = k + 1; j < f; ++j)
                    for (int i = j; i < f; ++i) F[i + (size_t)j * f] -= F[i + (size_t)k * f] * F[j + (size_t)k * f];
            }
            double* L = arena.data() + P.l_off[s];
            for (int j = 0; j < w; ++j)
                for (int i = 0; i < f; ++i) L[i + (size_t)j * f] = F[i + (size_t)j * f];
            double* U = arena.data() + P.u_off[s];
            for (int bb = 0; bb < r; ++bb)
                for (int a = bb; a < r; ++a) U[a + (size_t)bb * P.u_ld[s]] = F[(w + a) + (size_t)(w + bb) * f];
        }
    // sweeps
    std::vector<double> v(n), uvec(P.sn_rows.size(), 0.0), tmp;
    for (int k = 0; k < n; ++k) v[k] = b[P.perm[k]];
    for (int l = 0; l < P.nlev; ++l)
        for (int t = P.lvl_all_ptr[l]; t < P.lvl_all_ptr[l + 1]; ++t) {
            const int s = P.lvl_all[t];
            const int c0 = P.sn_start[s], w = P.sn_start[s + 1] - c0;
            const int ro = P.sn_rowptr[s], f = P.sn_rowptr[s + 1] - ro;
            tmp.assign(f, 0.0);
            for (int i = 0; i < f; ++i) {
                double acc = i < w ? v[c0 + i] : 0.0;
                for (int q = P.cb_ptr[ro + i]; q < P.cb_ptr[ro + i + 1]; ++q) acc += uvec[P.cb_src[q]];
                tmp[i] = acc;
            }
            const double* L = arena.data() + P.l_off[s];
            for (int k = 0; k < w; ++k) {
                tmp[k] /= L[k + (size_t)k * f];
                for (int i = k + 1; i < f; ++i) tmp[i] -= L[i + (size_t)k * f] * tmp[k];
            }
            for (int i = 0; i < f; ++i) {
                if (i < w) v[c0 + i] = tmp[i];
                else uvec[ro + i] = tmp[i];
            }
        }
    for (int l = P.nlev - 1; l >= 0; --l)
        for (int t = P.lvl_all_ptr[l]; t < P.lvl_all_ptr[l + 1]; ++t) {
            const int s = P.lvl_all[t];
            const int c0 = P.sn_start[s], w = P.sn_start[s + 1] - c0;
            const int ro = P.sn_rowptr[s], f = P.sn_rowptr[s + 1] - ro;
            tmp.assign(f, 0.0);
            for (int i = 0; i < f; ++i) tmp[i] = v[P.sn_rows[ro + i]];
            const double* L = arena.data() + P.l_off[s];
            for (int k = w - 1; k >= 0; --k) {
                double sum = 0.0;
                for (int i = k + 1; i < f; ++i) sum += L[i + (size_t)k * f] * tmp[i];
                tmp[k] = (tmp[k] - sum) / L[k + (size_t)k * f];
            }
            for (int i = 0; i < w; ++i) v[c0 + i] = tmp[i];
        }
    for (int k = 0; k < n; ++k) x[P.perm[k]] = v[k];
    return failed;
}

}  // namespace ckkt
