// C-ABI of the condensed-KKT library: handle life cycle, workspace
// carving, and the drivers of the numeric phases (assembly + factorization,
// triangular sweeps, FP64 iterative refinement, HyKKT conjugate gradient).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "ckkt.h"
#include "analysis.hpp"
#include "device.hpp"

using namespace ckkt;

namespace ckkt {
int host_factor_solve(const Plan& P, int hy, const double* w_val, const double* g_val, const double* h_val,
                      const double* sigma_x, const double* sigma_s, double gamma, const double* b, double* x);
}

namespace {

struct Region {
    size_t off = 0, bytes = 0;
};

struct Layout {
    size_t total = 0;
    Region add(size_t bytes) {
        Region r;
        r.off = (total + 255) & ~(size_t)255;
        r.bytes = bytes;
        total = r.off + bytes;
        return r;
    }
};

template <typename V>
size_t vbytes(const std::vector<V>& v) { return v.size() * sizeof(V); }

}  // namespace

// Launch shapes that do not change the factor layout; chosen by the
// autotuner per pattern.
struct Tune {
    int compact64 = kCompactFront64;  // FP64 fronts up to this order form the compact class
    int compact32 = kCompactFront32;  // same for FP32
    int tiny_front = 48;              // compact classes whose fronts are at most this order use tiny_threads
    int tiny_threads = 64;            // workgroup size of such a compact class
    int compact_threads = 256;        // workgroup size of the compact class otherwise
    int sweep_cutoff = 64;            // sweeps use 256 threads when a level's largest front exceeds this
    int tiled_front = kSweepTiledFront;  // fronts with at least this many rows use the tiled sweeps
    int wide_front = kWideFront;         // FP64 levels with fronts this large use wide panels
};

struct ckkt_handle {
    Tune tune;
    Plan plan;
    ckkt_options opt{};
    int32_t formulation = CKKT_LIFTED;
    int32_t precision = CKKT_FP64;
    std::vector<LevelInfo> levels;

    // workspace layout
    Layout lay;
    struct PlanRegion { Region r; const void* host; };
    std::vector<PlanRegion> plan_regions;
    Region r_perm, r_iperm, r_kcolptr, r_kwsrc, r_kdiag, r_prodptr, r_prodr, r_proda, r_prodb, r_snstart, r_snrowptr,
        r_snrows, r_snparent, r_snlevel, r_childptr, r_childlist, r_relmap, r_kmap, r_loff, r_uoff, r_uld, r_lvlsmall, r_lvlbig, r_lvlall,
        r_tilesn, r_tilecol, r_wfptr, r_wfcol, r_wfvidx, r_jptr, r_jcol, r_jtptr, r_jtrow, r_jtvidx, r_jtgend,
        r_instvar, r_insteq, r_kcol, r_cbptr, r_cbsrc, r_cblen, r_cbuoff;
    Region r_K, r_d, r_scale, r_arena64, r_arena32, r_uvec, r_vperm, r_status, r_bits, r_dotpart, r_sc;
    Region r_sxreg, r_ssreg;  // diagonals shifted by delta_w (inertia correction)
    Region r_jd, r_z, r_cap, r_dpart, r_du;  // split dense rows: J_d, K_s^{-1} J_d^T, capacitance, dots
    Region r_drowdot, r_drowpart, r_cpart;   // (J x)_r, (|J||x|)_r of the split rows; chunk partials
    Region r_ctl, r_done;  // dependency-driven sweeps: control words, per-supernode flags
    Region r_tflag;        // block flags of the tiled fronts (one launch per level)
    int64_t n_tflags = 0;
    unsigned* tflag = nullptr;
    bool tiled_level = true;              // tiled fronts swept in one launch per level
    bool sched_hybrid = false;            // dependency-driven sweeps above the single-wave levels only
    unsigned long long wait_ticks = 0;    // wait limit of the flag waits in wall-clock ticks
    Region r_dscr;         // factored diagonal blocks of tiled fronts between launches
    std::vector<Region> r_vn, r_vm, r_veq;  // scratch vectors of length n, m, m_eq
    std::vector<Region> r_vk2;              // augmented-system refinement: 5 vectors of length m
    // learned preconditioner (opt.learned)
    Region r_feat, r_o, r_cache, r_go, r_mlpws, r_grad, r_sxold, r_dold, r_kdold, r_kdnew, r_dnew;
    std::vector<Region> r_lv;

    // bound state
    char* ws = nullptr;
    size_t ws_bytes = 0;
    DevPlan dp{};
    double *K = nullptr, *d = nullptr, *scale = nullptr, *uvec = nullptr, *vperm = nullptr;
    double *sxreg = nullptr, *ssreg = nullptr;
    double *jd = nullptr, *zd = nullptr, *cap = nullptr, *dpart = nullptr, *du = nullptr;
    int32_t* drows = nullptr;  // device copy of plan.dense_rows
    Region r_drows;
    double* arena64 = nullptr;
    float* arena32 = nullptr;
    int32_t* status = nullptr;  // [0] failing column, [1] FP32 pivot floors, [2] sweep wait failure
    unsigned* ctl = nullptr;
    double* dscr = nullptr;
    unsigned* done = nullptr;
    SweepSched sched;
    bool sched_ok = false;
    unsigned long long* bits = nullptr;  // [ninst omega][resmax][bmax]
    double *dotpart = nullptr, *sc = nullptr;
    std::vector<double*> vn, vm, veq, vk2;
    float *feat = nullptr, *mo = nullptr, *cache = nullptr, *go = nullptr, *grad = nullptr;
    void* mlpws = nullptr;
    double *sxold = nullptr, *dold = nullptr, *kdold = nullptr, *kdnew = nullptr, *dnew = nullptr;
    std::vector<double*> lv;
    bool stale_valid = false;

    bool factored = false;
    bool fp64_factored = false;  // FP64 factor valid (fallback path of FP32_IR)
    // FP32_IR handles: after a system that needed the FP64 refactorization,
    // the next fp32_skip factorizations are FP64 from the start (the FP32
    // attempt would fail the same way on the neighbouring systems of an
    // interior-point sequence); the skip doubles while failures repeat
    int32_t fp32_skip = 0, fp32_backoff = 0;
    bool fp64_by_history = false;  // the current factor is FP64 for that reason
    SysVals vals{};
    int32_t failed_column = -1;

    // pinned host staging
    void* host = nullptr;
    size_t host_bytes = 0;

    // captured launch sequences (replayed with hipGraphLaunch on the
    // caller's stream): [0] factor FP64, [1] factor FP32, [2] sweeps FP64,
    // [3] sweeps FP32.  They reference only workspace memory.
    hipStream_t capture_stream = nullptr;
    SideStream side;  // second stream of the factorization (tiled fronts)
    // captured launch sequences: factorization (FP64, FP32), factor
    // application (FP64, FP32), HyKKT CG iteration (FP64, FP32 factor),
    // whole factorize-and-solve calls (FP64, FP32)
    hipGraphExec_t graphs[8] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    const void* cg_key[2][3] = {};  // G values, dx and dy a CG-iteration graph was captured with
    const void* fs_key[2][8] = {};  // pointers and step count a factorize-and-solve graph was captured with
    bool use_graphs = true;
    bool debug_launch = false;  // CKKT_DEBUG_LAUNCH=1: report the first failing launch per factor level

    // timing
    int32_t timing = 0;  // bit p: phase p is timed
    double ms[4] = {0, 0, 0, 0};
    int64_t calls[4] = {0, 0, 0, 0};
    struct Pending { int phase; hipEvent_t a, b; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> event_pool;
};

namespace {

ckkt_status hip_ok(hipError_t e) { return e == hipSuccess ? CKKT_OK : CKKT_ERR_HIP; }

#define HIP_TRY(x)                                   \
    do {                                             \
        hipError_t _e = (x);                         \
        if (_e != hipSuccess) return CKKT_ERR_HIP;   \
    } while (0)

hipEvent_t take_event(ckkt_handle* h) {
    if (!h->event_pool.empty()) {
        hipEvent_t e = h->event_pool.back();
        h->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct PhaseTimer {
    ckkt_handle* h;
    int phase;
    hipStream_t st;
    hipEvent_t a = nullptr;
    PhaseTimer(ckkt_handle* h_, int ph, hipStream_t s) : h(h_), phase(ph), st(s) {
        if (h->timing & (1 << phase)) {
            a = take_event(h);
            if (a) (void)hipEventRecord(a, st);
        }
    }
    ~PhaseTimer() {
        if (a) {
            hipEvent_t b = take_event(h);
            if (b) {
                (void)hipEventRecord(b, st);
                h->pending.push_back({phase, a, b});
            }
        }
    }
};

void destroy_side(SideStream& sd) {
    if (sd.stream) (void)hipStreamDestroy(sd.stream);
    for (hipEvent_t e : {sd.fork, sd.join})
        if (e) (void)hipEventDestroy(e);
    sd = SideStream{};
}

void build_levels(ckkt_handle* h) {
    const Plan& P = h->plan;
    const Tune& T = h->tune;
    h->levels.assign(P.nlev, LevelInfo{});
    h->n_tflags = 0;
    auto front = [&](int s) { return P.sn_rowptr[s + 1] - P.sn_rowptr[s]; };
    auto width = [&](int s) { return P.sn_start[s + 1] - P.sn_start[s]; };
    for (int l = 0; l < P.nlev; ++l) {
        LevelInfo& L = h->levels[l];
        L.small_begin = P.lvl_small_ptr[l];
        L.small_count = P.lvl_small_ptr[l + 1] - L.small_begin;
        L.small_maxf = 0;
        L.small_split = L.small_split32 = 0;
        L.small_maxf_a = L.small_maxf_a32 = 0;
        for (int t = L.small_begin; t < L.small_begin + L.small_count; ++t) {
            const int f = front(P.lvl_small[t]);
            L.small_maxf = std::max(L.small_maxf, f);
            if (f <= T.compact64) { L.small_split++; L.small_maxf_a = std::max(L.small_maxf_a, f); }
            if (f <= T.compact32) { L.small_split32++; L.small_maxf_a32 = std::max(L.small_maxf_a32, f); }
        }
        const int fa = h->precision == CKKT_FP32_IR ? L.small_maxf_a32 : L.small_maxf_a;
        L.small_threads_a = fa <= T.tiny_front ? T.tiny_threads : T.compact_threads;
        L.big_begin = P.lvl_big_ptr[l];
        L.big_count = P.lvl_big_ptr[l + 1] - L.big_begin;
        L.big_maxw = L.big_maxf = 0;
        for (int t = L.big_begin; t < L.big_begin + L.big_count; ++t) {
            L.big_maxw = std::max(L.big_maxw, width(P.lvl_big[t]));
            L.big_maxf = std::max(L.big_maxf, front(P.lvl_big[t]));
        }
        L.big_one = BigOne{0, 0, 0, -1};
        if (L.big_count == 1) {
            const int sb = P.lvl_big[L.big_begin];
            L.big_one = BigOne{P.sn_start[sb], width(sb), front(sb), P.l_off[sb]};
        }
        L.all_begin = P.lvl_all_ptr[l];
        L.all_count = P.lvl_all_ptr[l + 1] - L.all_begin;
        L.all_maxf = L.all_maxw = 0;
        L.sweep_small_count = 0;
        for (int t = L.all_begin; t < L.all_begin + L.all_count; ++t) {
            L.all_maxf = std::max(L.all_maxf, front(P.lvl_all[t]));
            L.all_maxw = std::max(L.all_maxw, width(P.lvl_all[t]));
            L.sweep_small_count += front(P.lvl_all[t]) < T.tiled_front;
        }
        L.tile_begin = P.big_tiles_ptr[l];
        L.tile_count = P.big_tiles_ptr[l + 1] - L.tile_begin;
        L.sweep_threads = L.all_maxf > T.sweep_cutoff ? 256 : 64;
        L.sweep_tiled_f = T.tiled_front;
        L.wide_front = T.wide_front;
        L.tflag_off = h->n_tflags;
        if (L.big_count > 0 && L.big_maxf >= L.sweep_tiled_f)
            h->n_tflags += L.big_count * ((L.big_maxw + 63) / 64);
    }
}

// Every launch of the plan fits the LDS of one workgroup (checked once at
// analysis, so no launch is ever rejected by the device).
bool plan_fits_lds(const ckkt_handle* h) {
    for (const LevelInfo& L : h->levels) {
        if ((size_t)L.small_maxf * L.small_maxf * sizeof(double) + kFactorStaticLds > (size_t)kLdsBytes) return false;
    }
    return true;
}

void build_layout(ckkt_handle* h) {
    const Plan& P = h->plan;
    Layout& L = h->lay;
    auto plan_region = [&](Region& r, const auto& vec) {
        r = L.add(std::max<size_t>(vbytes(vec), 8));
        h->plan_regions.push_back({r, vec.data()});
        h->plan_regions.back().r.bytes = vbytes(vec);
    };
    plan_region(h->r_perm, P.perm);
    plan_region(h->r_iperm, P.iperm);
    plan_region(h->r_kcolptr, P.kcolptr);
    plan_region(h->r_kwsrc, P.k_wsrc);
    plan_region(h->r_kdiag, P.k_diag);
    plan_region(h->r_prodptr, P.prod_ptr);
    plan_region(h->r_prodr, P.prod_r);
    plan_region(h->r_proda, P.prod_a);
    plan_region(h->r_prodb, P.prod_b);
    plan_region(h->r_snstart, P.sn_start);
    plan_region(h->r_snrowptr, P.sn_rowptr);
    plan_region(h->r_snrows, P.sn_rows);
    plan_region(h->r_snparent, P.sn_parent);
    plan_region(h->r_snlevel, P.sn_level);
    plan_region(h->r_childptr, P.child_ptr);
    plan_region(h->r_childlist, P.child_list);
    plan_region(h->r_relmap, P.relmap);
    plan_region(h->r_kmap, P.kmap);
    plan_region(h->r_loff, P.l_off);
    plan_region(h->r_uoff, P.u_off);
    plan_region(h->r_uld, P.u_ld);
    plan_region(h->r_lvlsmall, P.lvl_small);
    plan_region(h->r_lvlbig, P.lvl_big);
    plan_region(h->r_lvlall, P.lvl_all);
    plan_region(h->r_tilesn, P.big_tile_sn);
    plan_region(h->r_tilecol, P.big_tile_col);
    plan_region(h->r_wfptr, P.wf_ptr);
    plan_region(h->r_wfcol, P.wf_col);
    plan_region(h->r_wfvidx, P.wf_vidx);
    plan_region(h->r_jptr, P.j_ptr);
    plan_region(h->r_jcol, P.j_col);
    plan_region(h->r_jtptr, P.jt_ptr);
    plan_region(h->r_jtrow, P.jt_row);
    plan_region(h->r_jtvidx, P.jt_vidx);
    plan_region(h->r_jtgend, P.jt_gend);
    plan_region(h->r_instvar, P.inst_of_var);
    plan_region(h->r_insteq, P.inst_of_eqrow);
    plan_region(h->r_kcol, P.kcol);
    plan_region(h->r_cbptr, P.cb_ptr);
    plan_region(h->r_cbsrc, P.cb_src);
    plan_region(h->r_cblen, P.cb_len);
    plan_region(h->r_cbuoff, P.cb_uoff);
    plan_region(h->r_drows, P.dense_rows);

    const size_t n = std::max<int64_t>(P.n, 1), m = std::max<int64_t>(P.m, 1), me = std::max<int64_t>(P.m_eq, 1);
    h->r_K = L.add(std::max<size_t>(P.kcolptr.back(), 1) * sizeof(double));
    h->r_d = L.add(m * sizeof(double));
    h->r_scale = L.add(n * sizeof(double));
    // the FP64 arena is present in both precisions (FP32_IR falls back to it)
    h->r_arena64 = L.add(std::max<int64_t>(P.arena, 1) * sizeof(double));
    if (h->precision == CKKT_FP32_IR) h->r_arena32 = L.add(std::max<int64_t>(P.arena, 1) * sizeof(float));
    h->r_uvec = L.add(std::max<size_t>(P.sn_rows.size(), 1) * sizeof(double));
    h->r_vperm = L.add(n * sizeof(double));
    h->r_status = L.add(4 * sizeof(int32_t));
    h->r_ctl = L.add(kSweepCtlWords * sizeof(unsigned));
    h->r_tflag = L.add(std::max<size_t>((size_t)h->n_tflags * sizeof(unsigned), 8));
    h->r_done = L.add(std::max<size_t>(P.ns, 1) * sizeof(unsigned));
    {
        int maxbig = 1;
        for (int l = 0; l < P.nlev; ++l) maxbig = std::max(maxbig, P.lvl_big_ptr[l + 1] - P.lvl_big_ptr[l]);
        h->r_dscr = L.add((size_t)maxbig * kPanelNB * kPanelNB * sizeof(double));
    }
    h->r_bits = L.add((P.ninst + 2) * sizeof(unsigned long long));
    h->r_dotpart = L.add(kDotBlocks * sizeof(double));
    h->r_sc = L.add(16 * sizeof(double));
    h->r_sxreg = L.add(n * sizeof(double));
    h->r_ssreg = L.add(m * sizeof(double));
    {
        const size_t kd = std::max<size_t>(P.dense_rows.size(), 1);
        h->r_jd = L.add(kd * n * sizeof(double));
        h->r_z = L.add(kd * n * sizeof(double));
        h->r_cap = L.add(kd * kd * sizeof(double));
        h->r_dpart = L.add(kd * kDotBlocks * sizeof(double));
        h->r_du = L.add(kd * sizeof(double));
        h->r_drowdot = L.add(2 * kd * sizeof(double));
        h->r_drowpart = L.add(2 * kd * kDenseChunkBuf * sizeof(double));
        h->r_cpart = L.add(kd * (kd + 1) / 2 * kDenseChunkBuf * sizeof(double));
    }
    h->r_vn.clear();
    h->r_vm.clear();
    h->r_veq.clear();
    for (int i = 0; i < 8; ++i) h->r_vn.push_back(L.add(n * sizeof(double)));
    for (int i = 0; i < 2; ++i) h->r_vm.push_back(L.add(m * sizeof(double)));
    for (int i = 0; i < 6; ++i) h->r_veq.push_back(L.add(me * sizeof(double)));
    h->r_vk2.clear();
    for (int i = 0; i < 5; ++i) h->r_vk2.push_back(L.add(m * sizeof(double)));
    h->r_lv.clear();
    if (h->opt.learned) {
        h->r_feat = L.add(n * kMlpF * sizeof(float));
        h->r_o = L.add(n * sizeof(float));
        h->r_cache = L.add(2 * kMlpH * n * sizeof(float));
        h->r_go = L.add(n * sizeof(float));
        h->r_mlpws = L.add(mlp_workspace_bytes((int64_t)n));
        h->r_grad = L.add(kMlpNParam * sizeof(float));
        h->r_sxold = L.add(n * sizeof(double));
        h->r_dold = L.add(m * sizeof(double));
        h->r_kdold = L.add(n * sizeof(double));
        h->r_kdnew = L.add(n * sizeof(double));
        h->r_dnew = L.add(m * sizeof(double));
        for (int i = 0; i < 4; ++i) h->r_lv.push_back(L.add(n * sizeof(double)));
    }
}

template <typename T>
T* at(ckkt_handle* h, const Region& r) { return reinterpret_cast<T*>(h->ws + r.off); }

void fill_devplan(ckkt_handle* h) {
    const Plan& P = h->plan;
    DevPlan& D = h->dp;
    D.n = P.n; D.m_eq = P.m_eq; D.m_ineq = P.m_ineq; D.m = P.m; D.ns = P.ns; D.ninst = P.ninst;
    D.hy = h->formulation == CKKT_HYKKT ? 1 : 0;
    D.nnzk = P.kcolptr.back();
    D.nnzg = P.nnz_g;
    D.perm = at<int32_t>(h, h->r_perm); D.iperm = at<int32_t>(h, h->r_iperm);
    D.kcolptr = at<int32_t>(h, h->r_kcolptr); D.k_wsrc = at<int32_t>(h, h->r_kwsrc);
    D.k_diag = at<int32_t>(h, h->r_kdiag); D.prod_ptr = at<int32_t>(h, h->r_prodptr);
    D.prod_r = at<int32_t>(h, h->r_prodr); D.prod_a = at<int32_t>(h, h->r_proda); D.prod_b = at<int32_t>(h, h->r_prodb);
    D.sn_start = at<int32_t>(h, h->r_snstart); D.sn_rowptr = at<int32_t>(h, h->r_snrowptr);
    D.sn_rows = at<int32_t>(h, h->r_snrows);
    D.sn_parent = at<int32_t>(h, h->r_snparent); D.sn_level = at<int32_t>(h, h->r_snlevel);
    D.child_ptr = at<int32_t>(h, h->r_childptr);
    D.child_list = at<int32_t>(h, h->r_childlist); D.relmap = at<int32_t>(h, h->r_relmap);
    D.kmap = at<int32_t>(h, h->r_kmap); D.l_off = at<int64_t>(h, h->r_loff); D.u_off = at<int64_t>(h, h->r_uoff);
    D.u_ld = at<int32_t>(h, h->r_uld); D.lvl_small = at<int32_t>(h, h->r_lvlsmall);
    D.lvl_big = at<int32_t>(h, h->r_lvlbig); D.lvl_all = at<int32_t>(h, h->r_lvlall);
    D.big_tile_sn = at<int32_t>(h, h->r_tilesn); D.big_tile_col = at<int32_t>(h, h->r_tilecol);
    D.wf_ptr = at<int32_t>(h, h->r_wfptr); D.wf_col = at<int32_t>(h, h->r_wfcol); D.wf_vidx = at<int32_t>(h, h->r_wfvidx);
    D.j_ptr = at<int32_t>(h, h->r_jptr); D.j_col = at<int32_t>(h, h->r_jcol);
    D.jt_ptr = at<int32_t>(h, h->r_jtptr); D.jt_row = at<int32_t>(h, h->r_jtrow);
    D.jt_vidx = at<int32_t>(h, h->r_jtvidx); D.jt_gend = at<int32_t>(h, h->r_jtgend);
    D.inst_of_var = at<int32_t>(h, h->r_instvar); D.inst_of_eqrow = at<int32_t>(h, h->r_insteq);
    D.kcol = at<int32_t>(h, h->r_kcol);
    D.cb_ptr = at<int32_t>(h, h->r_cbptr); D.cb_src = at<int32_t>(h, h->r_cbsrc);
    D.cb_len = at<int32_t>(h, h->r_cblen); D.cb_uoff = at<int64_t>(h, h->r_cbuoff);
    D.drows = at<int32_t>(h, h->r_drows);
    D.ndense = (int32_t)P.dense_rows.size();
    D.dense_min = D.ndense > 0 ? h->opt.dense_row_min : 0;
    D.drowdot = at<double>(h, h->r_drowdot);
    D.drowpart = at<double>(h, h->r_drowpart);

    h->K = at<double>(h, h->r_K);
    h->d = at<double>(h, h->r_d);
    h->scale = at<double>(h, h->r_scale);
    h->arena64 = at<double>(h, h->r_arena64);
    h->arena32 = h->precision == CKKT_FP32_IR ? at<float>(h, h->r_arena32) : nullptr;
    h->uvec = at<double>(h, h->r_uvec);
    h->vperm = at<double>(h, h->r_vperm);
    h->status = at<int32_t>(h, h->r_status);
    h->ctl = at<unsigned>(h, h->r_ctl);
    h->tflag = at<unsigned>(h, h->r_tflag);
    h->done = at<unsigned>(h, h->r_done);
    h->dscr = at<double>(h, h->r_dscr);
    h->bits = at<unsigned long long>(h, h->r_bits);
    h->dotpart = at<double>(h, h->r_dotpart);
    h->sc = at<double>(h, h->r_sc);
    h->sxreg = at<double>(h, h->r_sxreg);
    h->ssreg = at<double>(h, h->r_ssreg);
    h->jd = at<double>(h, h->r_jd);
    h->zd = at<double>(h, h->r_z);
    h->cap = at<double>(h, h->r_cap);
    h->dpart = at<double>(h, h->r_dpart);
    h->du = at<double>(h, h->r_du);
    h->drows = at<int32_t>(h, h->r_drows);
    h->vn.clear(); h->vm.clear(); h->veq.clear();
    for (auto& r : h->r_vn) h->vn.push_back(at<double>(h, r));
    for (auto& r : h->r_vm) h->vm.push_back(at<double>(h, r));
    for (auto& r : h->r_veq) h->veq.push_back(at<double>(h, r));
    h->vk2.clear();
    for (auto& r : h->r_vk2) h->vk2.push_back(at<double>(h, r));
    h->lv.clear();
    if (h->opt.learned) {
        h->feat = at<float>(h, h->r_feat);
        h->mo = at<float>(h, h->r_o);
        h->cache = at<float>(h, h->r_cache);
        h->go = at<float>(h, h->r_go);
        h->mlpws = at<char>(h, h->r_mlpws);
        h->grad = at<float>(h, h->r_grad);
        h->sxold = at<double>(h, h->r_sxold);
        h->dold = at<double>(h, h->r_dold);
        h->kdold = at<double>(h, h->r_kdold);
        h->kdnew = at<double>(h, h->r_kdnew);
        h->dnew = at<double>(h, h->r_dnew);
        for (auto& r : h->r_lv) h->lv.push_back(at<double>(h, r));
    }
}

// Everything after the symbolic analysis: launch geometry and workspace
// layout (also the path of a plan loaded by ckkt_plan_load).
// The handle is owned by the unique_ptr until it is handed to the caller
// (*out), so every error return and every exception frees it.
using HandlePtr = std::unique_ptr<ckkt_handle>;

ckkt_status finish_plan(HandlePtr h, const AnalyzeOptions& ao, ckkt_handle** out, size_t* workspace_bytes);

ckkt_status finish_analyze(HandlePtr h, const AnalyzeOptions& ao, const PatternIn& pin, ckkt_handle** out,
                           size_t* workspace_bytes) {
    std::string err = analyze(pin, ao, h->plan);
    if (!err.empty()) {
        if (err.rfind("device:", 0) == 0) return CKKT_ERR_HIP;  // a HIP call of the device analysis failed
        return err.rfind("internal", 0) == 0 ? CKKT_ERR_ARG : CKKT_ERR_PATTERN;
    }
    return finish_plan(std::move(h), ao, out, workspace_bytes);
}

ckkt_status finish_plan(HandlePtr h, const AnalyzeOptions& ao, ckkt_handle** out, size_t* workspace_bytes) {
    if ((int)h->plan.dense_rows.size() > kMaxDenseRows) return CKKT_ERR_ARG;
    // CKKT_TILED_SWEEP_FRONT moves the size from which fronts are swept by
    // the tiled kernels; it stays above the LDS front limit (so that every
    // such front is in its level's big list) and at most the largest front
    // one sweep workgroup can stage.
    if (const char* tf = std::getenv("CKKT_TILED_SWEEP_FRONT")) {
        const int v = std::atoi(tf);
        if (v > 0) h->tune.tiled_front = std::min(std::max(v, ao.big_front + 1), kSweepMaxFront);
    }
    // CKKT_WIDE_FRONT moves the front size from which FP64 levels use
    // wide panels (any value above the LDS front limit)
    if (const char* wf = std::getenv("CKKT_WIDE_FRONT")) {
        const int v = std::atoi(wf);
        if (v > 0) h->tune.wide_front = std::max(v, ao.big_front + 1);
    }
    // CKKT_TINY_FRONT moves the largest front order of the compact classes
    // factored by one-wave workgroups (at most the compact class's limit)
    if (const char* tf = std::getenv("CKKT_TINY_FRONT")) {
        const int v = std::atoi(tf);
        if (v > 0) h->tune.tiny_front = std::min(v, kCompactFront64);
    }
    build_levels(h.get());
    if (!plan_fits_lds(h.get())) return CKKT_ERR_ARG;  // a small front beyond the LDS of one workgroup
    build_layout(h.get());
    if (workspace_bytes) *workspace_bytes = h->lay.total;
    *out = h.release();
    return CKKT_OK;
}

// The row pointer arrays start at 0 and never decrease, so copy_pattern
// reads index arrays of known, non-negative length (checked before any
// index array is touched; validate() checks the indices of the copy).
bool pattern_ptrs_ok(const ckkt_pattern* p) {
    auto ok = [](const int32_t* ptr, int64_t rows) {
        if (rows == 0 && !ptr) return true;
        if (!ptr || ptr[0] != 0) return false;
        for (int64_t r = 0; r < rows; ++r)
            if (ptr[r + 1] < ptr[r]) return false;
        return true;
    };
    return ok(p->w_ptr, p->n) && ok(p->g_ptr, p->m_eq) && ok(p->h_ptr, p->m_ineq);
}

PatternIn copy_pattern(const ckkt_pattern* p) {
    PatternIn q;
    q.n = p->n; q.m_eq = p->m_eq; q.m_ineq = p->m_ineq;
    auto cp = [](std::vector<int32_t>& dst, const int32_t* src, int64_t len) {
        dst.assign(len, 0);
        if (len > 0 && src) std::memcpy(dst.data(), src, len * sizeof(int32_t));
    };
    cp(q.w_ptr, p->w_ptr, p->n + 1);
    if (p->w_ptr && p->n >= 0) cp(q.w_idx, p->w_idx, p->w_ptr[p->n]);
    cp(q.g_ptr, p->g_ptr, p->m_eq + 1);
    if (p->g_ptr && p->m_eq > 0) cp(q.g_idx, p->g_idx, p->g_ptr[p->m_eq]);
    cp(q.h_ptr, p->h_ptr, p->m_ineq + 1);
    if (p->h_ptr && p->m_ineq > 0) cp(q.h_idx, p->h_idx, p->h_ptr[p->m_ineq]);
    return q;
}

bool pattern_args_ok(const ckkt_pattern* p) {
    if (!p || p->n < 0 || p->m_eq < 0 || p->m_ineq < 0) return false;
    if (!p->w_ptr || (p->w_ptr[p->n] > 0 && !p->w_idx)) return false;
    if (p->m_eq > 0 && (!p->g_ptr || (p->g_ptr[p->m_eq] > 0 && !p->g_idx))) return false;
    if (p->m_ineq > 0 && (!p->h_ptr || (p->h_ptr[p->m_ineq] > 0 && !p->h_idx))) return false;
    if (p->formulation != CKKT_LIFTED && p->formulation != CKKT_HYKKT) return false;
    return true;
}

AnalyzeOptions analyze_options(const ckkt_options& o) {
    AnalyzeOptions ao;
    ao.ordering = o.ordering;
    ao.relax = o.relax;
    ao.dense_row_min = o.dense_row_min;
    ao.threads = std::max(1, std::min<int>(kAnalyzeThreads, (int)std::thread::hardware_concurrency()));
    // the whole front of a small supernode lives in LDS (f^2 elements <= 160 KiB)
    // the FP64 factor is also built for FP32_IR handles (refactorization
    // fallback), so the FP64 LDS capacity bounds both precisions
    const int cap = kLdsFront64;
    ao.big_front = (o.lds_front_max > 0) ? std::min(o.lds_front_max, cap) : cap;
    return ao;
}

// ------------------------------------------------------------ numeric steps

template <typename T>
T* arena_of(ckkt_handle* h);
template <>
double* arena_of<double>(ckkt_handle* h) { return h->arena64; }
template <>
float* arena_of<float>(ckkt_handle* h) { return h->arena32; }

template <typename T>
void factor_levels(ckkt_handle* h, const double* scale, hipStream_t st) {
    T* arena = arena_of<T>(h);
    for (size_t l = 0; l < h->levels.size(); ++l) {
        launch_factor_level<T>(h->dp, h->levels[l], h->K, arena, h->status, scale, st, &h->side, h->dscr);
        if (h->debug_launch) {
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess)
                std::fprintf(stderr, "ckkt: factor level %zu (%s): %s\n", l, sizeof(T) == 8 ? "fp64" : "fp32",
                             hipGetErrorString(e));
        }
    }
}


// Split of the supernodes between the single-wave and the workgroup
// workers of the dependency-driven sweeps, and their launch shapes.
bool build_sweep_sched(ckkt_handle* h) {
    const Plan& P = h->plan;
    SweepSched S;
    S.ns = P.ns;
    int lw = 0;
    while (lw < (int)h->levels.size() && h->levels[lw].all_maxf <= kSweepWaveFront) ++lw;
    S.wave_lvl = lw;
    S.wave_t1 = P.ns ? P.lvl_all_ptr[lw] : 0;
    int lp = lw;
    while (lp < (int)h->levels.size() && h->levels[lp].all_maxf <= 2 * kSweepWaveFront &&
           h->levels[lp].all_maxw <= kSweepWaveFront)
        ++lp;
    S.pair_lvl = lp;
    S.pair_t1 = P.ns ? P.lvl_all_ptr[lp] : 0;
    int maxf = 1, maxw = 1;
    for (int l = lw; l < (int)h->levels.size(); ++l) {
        maxf = std::max(maxf, h->levels[l].all_maxf);
        maxw = std::max(maxw, h->levels[l].all_maxw);
    }
    if (maxf > kSweepMaxFront) return false;  // a workgroup stages its whole front vector
    S.ldd = sweep_diag_ld(maxw);
    S.rows = maxf <= kGroupThreads;
    // levels from rows_lvl on (fronts above kRowsMinFront rows) go to the
    // row-held forward kernel, the levels below it to the LDS one
    int lr = lp;
    while (lr < (int)h->levels.size() && h->levels[lr].all_maxf <= kRowsMinFront) ++lr;
    S.rows_lvl = S.rows ? lr : (int)h->levels.size();
    S.rows_t0 = P.ns ? P.lvl_all_ptr[S.rows_lvl] : 0;
    S.group_lds = (size_t)(((maxf + 1) & ~1) + S.ldd * S.ldd) * sizeof(double);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || !sweep_sched_grids(S, dev)) {
        (void)hipGetLastError();
        return false;
    }
    h->sched = S;
    return true;
}

template <typename T>
void sweep_levels(ckkt_handle* h, hipStream_t st) {
    const T* arena = arena_of<T>(h);
    if (h->sched_ok) {
        // dependency-driven: every supernode (CKKT_DEP_SWEEPS=1), or only the
        // levels above those of fronts with at most 128 rows and 64 columns,
        // which are swept level by level by waves and wave pairs
        // (CKKT_DEP_SWEEPS=2)
        const bool waves = !h->sched_hybrid;
        const int lw = h->sched.pair_lvl;
        launch_sweep_prep(h->ctl, st);
        if (!waves)
            for (int l = 0; l < lw; ++l) launch_fwd_level<T>(h->dp, h->levels[l], arena, h->vperm, h->uvec, st, nullptr);
        launch_fwd_sched<T>(h->dp, h->sched, arena, h->vperm, h->uvec, h->ctl, h->done, h->status + 2, st, waves);
        launch_bwd_sched<T>(h->dp, h->sched, arena, h->vperm, h->ctl, h->done, h->status + 2, st, waves);
        if (!waves)
            for (int l = lw; l-- > 0;) launch_bwd_level<T>(h->dp, h->levels[l], arena, h->vperm, st, nullptr);
        return;
    }
    TiledSync ts;
    const TiledSync* tsp = nullptr;
    if (h->tiled_level && h->n_tflags > 0) {
        launch_sweep_prep(h->ctl, st);  // advances the epoch the flags are compared with
        ts.ctl = h->ctl;
        ts.flags = h->tflag;
        ts.err = h->status + 2;
        ts.ticks = h->wait_ticks;
        tsp = &ts;
    }
    for (size_t l = 0; l < h->levels.size(); ++l)
        launch_fwd_level<T>(h->dp, h->levels[l], arena, h->vperm, h->uvec, st, tsp);
    for (size_t l = h->levels.size(); l-- > 0;) launch_bwd_level<T>(h->dp, h->levels[l], arena, h->vperm, st, tsp);
}

// Capture a launch sequence once on the private stream; replay it on `st`.
// Falls back to direct launches if capture is unavailable.
template <typename F>
void run_captured(ckkt_handle* h, int slot, hipStream_t st, F&& launches) {
    if (h->use_graphs && !h->graphs[slot] && h->capture_stream) {
        hipGraph_t g = nullptr;
        if (hipStreamBeginCapture(h->capture_stream, hipStreamCaptureModeThreadLocal) == hipSuccess) {
            launches(h->capture_stream);
            if (hipStreamEndCapture(h->capture_stream, &g) == hipSuccess && g) {
                hipGraphExec_t ex = nullptr;
                if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess) h->graphs[slot] = ex;
                (void)hipGraphDestroy(g);
            }
        }
        (void)hipGetLastError();
        if (!h->graphs[slot]) h->use_graphs = false;
    }
    if (h->use_graphs && h->graphs[slot]) {
        if (hipGraphLaunch(h->graphs[slot], st) == hipSuccess) return;
        (void)hipGetLastError();
    }
    launches(st);
}

template <typename T>
void factor_all(ckkt_handle* h, const double* scale, hipStream_t st) {
    run_captured(h, std::is_same<T, double>::value ? 0 : 1, st,
                 [&](hipStream_t s) { factor_levels<T>(h, scale, s); });
}

// x = (L L^T)^{-1} b in the user numbering (with the Jacobi scaling of the
// FP32 factor folded into the permutations).
template <typename T>
void apply_inverse_t(ckkt_handle* h, const double* b, double* x, const double* scale, hipStream_t st) {
    PhaseTimer tm(h, 2, st);
    launch_gather_perm(h->dp, b, h->vperm, scale, st);
    run_captured(h, std::is_same<T, double>::value ? 2 : 3, st, [&](hipStream_t s) { sweep_levels<T>(h, s); });
    launch_scatter_perm(h->dp, h->vperm, x, scale, st);
}

// The same launches, for use inside another captured sequence (no timer,
// no graph of its own).
void apply_inverse_launches(ckkt_handle* h, const double* b, double* x, bool use64, hipStream_t st) {
    const bool d = use64 || h->precision == CKKT_FP64;
    const double* scale = d ? nullptr : h->scale;
    launch_gather_perm(h->dp, b, h->vperm, scale, st);
    if (d) sweep_levels<double>(h, st);
    else sweep_levels<float>(h, st);
    launch_scatter_perm(h->dp, h->vperm, x, scale, st);
    if (d) launch_dense_correct(h->plan.n, (int)h->plan.dense_rows.size(), h->jd, h->zd, h->cap, h->dpart, h->du,
                                x, st);
}

// Uses the FP64 factor when `use64`, else the handle's precision.  With
// split dense rows (FP64 handles only) the sweeps apply K_s^{-1} and the
// Woodbury step turns the result into K^{-1} b.
void apply_inverse(ckkt_handle* h, const double* b, double* x, bool use64, hipStream_t st) {
    if (use64 || h->precision == CKKT_FP64) {
        apply_inverse_t<double>(h, b, x, nullptr, st);
        if (!h->plan.dense_rows.empty()) {
            PhaseTimer tm(h, 2, st);
            launch_dense_correct(h->plan.n, (int)h->plan.dense_rows.size(), h->jd, h->zd, h->cap, h->dpart, h->du,
                                 x, st);
        }
    } else {
        apply_inverse_t<float>(h, b, x, h->scale, st);
    }
}

// After the FP64 factorization of K_s: J_d, Z = K_s^{-1} J_d^T (k sweep
// pairs) and the Cholesky factor of C = D_d^{-1} + J_d Z.
void dense_rows_setup(ckkt_handle* h, hipStream_t st) {
    const int k = (int)h->plan.dense_rows.size(), n = h->plan.n;
    if (k == 0) return;
    {
        PhaseTimer tm(h, 1, st);
        launch_dense_setup_gather(h->dp, h->vals, h->drows, k, h->jd, st);
    }
    for (int b = 0; b < k; ++b) apply_inverse_t<double>(h, h->jd + (int64_t)b * n, h->zd + (int64_t)b * n, nullptr, st);
    PhaseTimer tm(h, 1, st);
    launch_dense_setup_cap(n, k, h->drows, h->d, h->jd, h->zd, at<double>(h, h->r_cpart), h->cap, h->status, st);
}

struct ResidualOut {
    double omega = 0.0;      // max over instances
    double resmax = 0.0;
    double rhsmax = 0.0;     // max |rhs| left by launch_rhs_max
    std::vector<double> per_inst;
    int32_t status0 = INT_MAX, status1 = 0, status2 = 0, status3 = 0;
};

double bits_to_double(unsigned long long b) {
    double d;
    std::memcpy(&d, &b, sizeof(d));
    return d;
}

// Read back (sync) what the last residual left: omega per instance, max
// |res|, max |rhs| and the status words.
ckkt_status read_residual(ckkt_handle* h, ResidualOut& out, hipStream_t st) {
    const int ni = h->plan.ninst;
    char* host = static_cast<char*>(h->host);
    HIP_TRY(hipMemcpyAsync(host, h->bits, (ni + 2) * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(host + (ni + 2) * sizeof(unsigned long long), h->status, 4 * sizeof(int32_t),
                           hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const unsigned long long* hb = reinterpret_cast<const unsigned long long*>(host);
    out.per_inst.resize(ni);
    out.omega = 0.0;
    for (int i = 0; i < ni; ++i) {
        out.per_inst[i] = bits_to_double(hb[i]);
        out.omega = std::max(out.omega, out.per_inst[i]);
    }
    out.resmax = bits_to_double(hb[ni]);
    out.rhsmax = bits_to_double(hb[ni + 1]);
    const int32_t* hs = reinterpret_cast<const int32_t*>(host + (ni + 2) * sizeof(unsigned long long));
    out.status0 = hs[0];
    out.status1 = hs[1];
    out.status2 = hs[2];
    out.status3 = hs[3];
    return out.status2 ? CKKT_ERR_TIMEOUT : CKKT_OK;
}

// Enqueue the residual of the current iterate and read omega back (sync).
ckkt_status residual_sync(ckkt_handle* h, const double* x, const double* y, const double* rhs1,
                          const double* rhs2, double* res1, double* res2, ResidualOut& out, hipStream_t st) {
    const int ni = h->plan.ninst;
    {
        PhaseTimer tm(h, 3, st);
        launch_zero_u64(h->bits, ni + 1, st);
        launch_residual(h->dp, h->vals, h->d, x, y, rhs1, rhs2, res1, res2, h->vm[0], h->vm[1], h->bits,
                        h->bits + ni, st);
    }
    return read_residual(h, out, st);
}

// max |rhs| into the word after the residual maxima, read back (without
// a synchronization of its own) by the next residual_sync
void launch_rhs_max(ckkt_handle* h, const double* a, int na, const double* b, int nb_, hipStream_t st) {
    unsigned long long* slot = h->bits + h->plan.ninst + 1;
    launch_zero_u64(slot, 1, st);
    launch_maxabs(na, a, slot, st);
    if (b) launch_maxabs(nb_, b, slot, st);
}

ckkt_status read_rhs_max(ckkt_handle* h, const double* a, int na, const double* b, int nb_, double& out,
                         hipStream_t st) {
    const int ni = h->plan.ninst;
    unsigned long long* slot = h->bits + ni + 1;
    launch_zero_u64(slot, 1, st);
    launch_maxabs(na, a, slot, st);
    if (b) launch_maxabs(nb_, b, slot, st);
    HIP_TRY(hipMemcpyAsync(h->host, slot, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    out = bits_to_double(*reinterpret_cast<unsigned long long*>(h->host));
    return CKKT_OK;
}

ckkt_status read_scalars(ckkt_handle* h, double* dst, int count, hipStream_t st) {
    HIP_TRY(hipMemcpyAsync(h->host, h->sc, count * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    std::memcpy(dst, h->host, count * sizeof(double));
    return CKKT_OK;
}

// CKKT_ERR_NONFINITE when an assembled entry was not finite, CKKT_ERR_NOT_SPD
// when the FP64 factor met a non-positive pivot, else CKKT_OK.
ckkt_status check_factor(ckkt_handle* h, const ResidualOut& r) {
    if (r.status3) return CKKT_ERR_NONFINITE;
    if (h->precision == CKKT_FP64 || h->fp64_factored) {
        if (r.status0 != INT_MAX) {
            h->failed_column = (r.status0 >= 0 && r.status0 < h->plan.n) ? h->plan.perm[r.status0] : r.status0;
            return CKKT_ERR_NOT_SPD;
        }
    }
    return CKKT_OK;
}

// FP64 factorization of the already assembled K (fallback of FP32_IR).
void refactor_fp64(ckkt_handle* h, hipStream_t st) {
    PhaseTimer tm(h, 1, st);
    launch_init_status(h->status, true, st);
    factor_all<double>(h, nullptr, st);
    h->fp64_factored = true;
}

// ------------------------------------------------------------ LiftedKKT

constexpr int kPcgMaxit = 50;

// FP64 preconditioned CG on K x = b (K applied unassembled), preconditioned
// by the FP32 factor, starting from the current x with its residual `res`.
// The true residual is recomputed every iteration (it also yields omega).
// Returns true when omega <= tol.
bool pcg_fp32(ckkt_handle* h, const double* b, double* x, double* res, ResidualOut& r, ckkt_solve_info* info,
              hipStream_t st, ckkt_status& rc) {
    const int n = h->plan.n;
    double* z = h->vn[1];
    double* p = h->vn[2];
    double* q = h->vn[3];
    double* sc = h->sc + 8;  // [0] rz, [1] pq, [2] alpha, [3] rz_new, [4] beta
    apply_inverse(h, res, z, false, st);
    {
        PhaseTimer tm(h, 3, st);
        launch_copy(n, z, p, st);
        launch_dot(n, res, z, h->dotpart, sc + 0, st);
    }
    double omega_start = r.omega;
    for (int k = 0; k < kPcgMaxit; ++k) {
        {
            PhaseTimer tm(h, 3, st);
            // q = -K p through the residual kernels with a zero right-hand side
            launch_zero_u64(h->bits, h->plan.ninst + 1, st);
            launch_residual(h->dp, h->vals, h->d, p, nullptr, nullptr, nullptr, q, nullptr, h->vm[0], h->vm[1],
                            h->bits, h->bits + h->plan.ninst, st);
            launch_dot(n, p, q, h->dotpart, sc + 1, st);  // = -p^T K p
            launch_cg_alpha(sc, st);                     // alpha = rz / (-pKp)
            launch_axpy_dev(n, sc, 2, -1.0, p, x, st);   // x += (rz / pKp) p
        }
        info->pcg_iters++;
        rc = residual_sync(h, x, nullptr, b, nullptr, res, nullptr, r, st);
        if (rc) return false;
        if (r.omega <= h->opt.tol) return true;
        if (!std::isfinite(r.omega)) return false;
        // give up early when the preconditioned iteration is not contracting
        if (k == 0) omega_start = r.omega;
        if (k == 7 && !(r.omega < 1e-2 * omega_start)) return false;
        apply_inverse(h, res, z, false, st);
        {
            PhaseTimer tm(h, 3, st);
            launch_dot(n, res, z, h->dotpart, sc + 3, st);
            launch_cg_beta(sc, st);
            launch_cg_direction(n, sc, z, p, st);
        }
    }
    return false;
}

// FP64 PCG on the current system (h->vals, unassembled) from x = 0,
// preconditioned by D K_s^{-1} D with the current (stale) factor; o = NULL
// means D = I.  Returns true when omega <= tol.
bool pcg_stale(ckkt_handle* h, const double* b, double* x, const float* o, int maxit, double tol, ResidualOut& r,
               ckkt_solve_info* info, hipStream_t st, ckkt_status& rc) {
    const int n = h->plan.n;
    double* res = h->vn[0];
    double* z = h->vn[1];
    double* p = h->vn[2];
    double* q = h->vn[3];
    double* t = h->vn[4];
    double* sc = h->sc + 8;
    const bool use64 = h->fp64_factored;
    auto precond = [&](const double* in, double* out) {  // out = D K_s^{-1} (D in)
        launch_dscale(n, o, in, t, st);
        apply_inverse(h, t, out, use64, st);
        launch_dscale(n, o, out, out, st);
    };
    {
        PhaseTimer tm(h, 3, st);
        launch_fill(n, 0.0, x, st);
        launch_copy(n, b, res, st);
    }
    precond(res, z);
    {
        PhaseTimer tm(h, 3, st);
        launch_copy(n, z, p, st);
        launch_dot(n, res, z, h->dotpart, sc + 0, st);
    }
    for (int k = 0; k < maxit; ++k) {
        {
            PhaseTimer tm(h, 3, st);
            launch_zero_u64(h->bits, h->plan.ninst + 1, st);
            launch_residual(h->dp, h->vals, h->d, p, nullptr, nullptr, nullptr, q, nullptr, h->vm[0], h->vm[1],
                            h->bits, h->bits + h->plan.ninst, st);  // q = -K p
            launch_dot(n, p, q, h->dotpart, sc + 1, st);
            launch_cg_alpha(sc, st);
            launch_axpy_dev(n, sc, 2, -1.0, p, x, st);
        }
        info->pcg_iters++;
        rc = residual_sync(h, x, nullptr, b, nullptr, res, nullptr, r, st);
        if (rc) return false;
        if (r.omega <= tol) return true;
        if (!std::isfinite(r.omega)) return false;
        precond(res, z);
        {
            PhaseTimer tm(h, 3, st);
            launch_dot(n, res, z, h->dotpart, sc + 3, st);
            launch_cg_beta(sc, st);
            launch_cg_direction(n, sc, z, p, st);
        }
    }
    return false;
}

// After a solve of an FP32_IR handle: a system that needed the FP64
// refactorization makes the next fp32_skip factorizations FP64 from the
// start (4, doubling while failures repeat, at most kFp32MaxSkip); a system
// the FP32 factor solved resets the count.
constexpr int kFp32FirstSkip = 4, kFp32MaxSkip = 64;
void note_fp32_outcome(ckkt_handle* h, const ckkt_solve_info* info) {
    if (h->precision != CKKT_FP32_IR || h->fp64_by_history) return;
    if (info->fallback == 2) {
        h->fp32_backoff = h->fp32_backoff ? std::min(2 * h->fp32_backoff, kFp32MaxSkip) : kFp32FirstSkip;
        h->fp32_skip = h->fp32_backoff;
    } else {
        h->fp32_backoff = 0;
        h->fp32_skip = 0;
    }
}

// The FP32 factor is given up at once (no Richardson or PCG steps) when
// static pivoting floored a pivot (the factor is then that of another
// matrix) or when the first FP32 solve has a backward error above this:
// the FP32 error in the small space grows with the largest diagonal
// weights (Sec. 4, eq:cond:inversecondensederror).
constexpr double kFp32Hopeless = 0.1;

// start_steps > 0: x already holds the iterate after that many refinement
// steps of the current factor (the device steps of
// ckkt_batch_factorize_solve), and the refinement continues from it.
ckkt_status solve_lifted(ckkt_handle* h, const double* b, double* x, ckkt_solve_info* info, hipStream_t st,
                         int start_steps = 0) {
    const int n = h->plan.n;
    double* res = h->vn[0];
    double* dx = h->vn[1];
    launch_rhs_max(h, b, n, nullptr, 0, st);
    ckkt_status rc = CKKT_OK;
    bool use64 = h->precision == CKKT_FP64 || h->fp64_factored;
    if (h->fp64_by_history) info->fallback = 8;
    if (start_steps == 0) apply_inverse(h, b, x, use64, st);
    ResidualOut r;
    int steps = start_steps;
    double prev = INFINITY;
    int stall = 0;
    auto refactor = [&]() {
        refactor_fp64(h, st);
        use64 = true;
        info->fallback = 2;
        apply_inverse(h, b, x, true, st);
        steps = 0;
        prev = INFINITY;
        stall = 0;
    };
    for (;;) {
        rc = residual_sync(h, x, nullptr, b, nullptr, res, nullptr, r, st);
        if (rc) return rc;
        if ((rc = check_factor(h, r)) != CKKT_OK) return info->status = rc;
        if (steps == 0 && !std::isfinite(r.rhsmax)) return info->status = CKKT_ERR_NONFINITE;
        info->omega = r.omega;
        info->rho = r.rhsmax > 0 ? r.resmax / r.rhsmax : r.resmax;
        if (r.omega <= h->opt.tol) break;
        if (!use64) {
            if (steps == start_steps && (r.status1 > 0 || !(r.omega <= kFp32Hopeless))) {
                refactor();
                continue;
            }
            // FP32 factor: Richardson while it contracts; when it stagnates,
            // FP64 PCG preconditioned by the same factor; if that fails too,
            // FP64 refactorization of the already assembled matrix.
            if (!(r.omega < 0.25 * prev) || !std::isfinite(r.omega)) stall++;
            if (stall >= 1 || steps >= h->opt.ir_maxit) {
                if (std::isfinite(r.omega) && info->fallback == 0) {
                    info->fallback = 1;
                    if (pcg_fp32(h, b, x, res, r, info, st, rc)) {
                        info->omega = r.omega;
                        info->rho = r.rhsmax > 0 ? r.resmax / r.rhsmax : r.resmax;
                        break;
                    }
                    if (rc) return rc;
                }
                refactor();
                continue;
            }
        } else if (steps >= h->opt.ir_maxit) {
            info->refine_steps = steps;
            return CKKT_ERR_NO_CONVERGENCE;
        }
        prev = r.omega;
        apply_inverse(h, res, dx, use64, st);
        {
            PhaseTimer tm(h, 3, st);
            launch_axpy(n, 1.0, dx, x, st);
        }
        steps++;
    }
    info->refine_steps = steps;
    return CKKT_OK;
}

// ------------------------------------------------------------ HyKKT

// One solve of K1 = [[K, G^T], [G, -delta_c I]] (dx, dy) = (R1, R2) for
// delta_c > 0 by the primal Schur complement of Remark 1 (eqn:primal), whose
// matrix K + G^T G / delta_c is the factor's K_gamma with gamma = 1/delta_c:
// dx = K_gamma^{-1}(R1 + gamma G^T R2), dy = gamma (G dx - R2).  No CG.
void primal_schur_inner(ckkt_handle* h, const double* R1, const double* R2, double* dx, double* dy, bool use64,
                        hipStream_t st) {
    const DevPlan& P = h->dp;
    double* s = h->vn[2];
    {
        PhaseTimer tm(h, 3, st);
        launch_gt(P, h->vals, R1, h->vals.gamma, R2, s, st);
    }
    apply_inverse(h, s, dx, use64, st);
    {
        PhaseTimer tm(h, 3, st);
        launch_g(P, h->vals, dx, R2, dy, st);
        launch_scale(P.m_eq, h->vals.gamma, dy, st);
    }
}

// One HyKKT solve of K1 (dx, dy) = (R1, R2) through K_gamma (Sec. 3.1):
// s = R1 + gamma G^T R2, w = K_gamma^{-1} s, CG on S_gamma dy = G w - R2
// (eq:kkt:schurcomplhykkt) from dy = 0, then dx = w - sum_k alpha_k u_k with
// u_k = K_gamma^{-1} G^T p_k, which equals K_gamma^{-1}(s - G^T dy).
ckkt_status hykkt_inner(ckkt_handle* h, const double* R1, const double* R2, double* dx, double* dy, bool use64,
                        int& cg_iters, bool& cg_ok, hipStream_t st) {
    const DevPlan& P = h->dp;
    const int n = P.n, me = P.m_eq;
    double* s = h->vn[2];
    double* t = h->vn[3];
    double* u = h->vn[4];
    double* r = h->veq[0];
    double* p = h->veq[1];
    double* q = h->veq[2];
    {
        PhaseTimer tm(h, 3, st);
        launch_gt(P, h->vals, R1, h->vals.gamma, R2, s, st);
    }
    apply_inverse(h, s, dx, use64, st);  // dx holds w and accumulates
    {
        PhaseTimer tm(h, 3, st);
        launch_g(P, h->vals, dx, R2, r, st);
        launch_fill(me, 0.0, dy, st);
        // p = 0 and beta = 0: the iteration's first step p = r + beta p
        // then gives p = r
        launch_fill(me, 0.0, p, st);
        launch_fill(1, 0.0, h->sc + 4, st);
        launch_dot(me, r, r, h->dotpart, h->sc + 0, st);
    }
    double hs[5];
    ckkt_status rc = read_scalars(h, hs, 1, st);
    if (rc) return rc;
    const double rr0 = hs[0];
    cg_ok = true;
    if (!(rr0 > 0.0)) return rr0 == 0.0 ? CKKT_OK : CKKT_ERR_BREAKDOWN;
    const double stop = h->opt.cg_tol * std::sqrt(rr0);
    int maxit = h->opt.cg_maxit > 0 ? h->opt.cg_maxit : std::max(1, std::min(me, 1000));
    // One CG iteration is one captured sequence (its pointers are the
    // handle's buffers, dx, dy and the G values of the current system; the
    // graph is captured again when any of the last three moves).  Phase time
    // counts as factor application.
    const int slot = (use64 || h->precision == CKKT_FP64) ? 4 : 5;
    const void* key[3] = {h->vals.g_val, dx, dy};
    const void** held = h->cg_key[slot - 4];
    if (h->graphs[slot] && (held[0] != key[0] || held[1] != key[1] || held[2] != key[2])) {
        (void)hipGraphExecDestroy(h->graphs[slot]);
        h->graphs[slot] = nullptr;
    }
    for (int i = 0; i < 3; ++i) held[i] = key[i];
    for (int k = 1; k <= maxit; ++k) {
        {
            PhaseTimer tm(h, 2, st);
            run_captured(h, slot, st, [&](hipStream_t s) {
                launch_cg_direction(me, h->sc, r, p, s);  // p = r + beta p
                launch_gt(P, h->vals, nullptr, 1.0, p, t, s);
                apply_inverse_launches(h, t, u, use64, s);
                launch_g(P, h->vals, u, nullptr, q, s);
                launch_dot(me, p, q, h->dotpart, h->sc + 1, s);
                launch_cg_alpha(h->sc, s);
                launch_cg_update(me, h->sc, p, q, dy, r, s);
                launch_axpy_dev(n, h->sc, 2, -1.0, u, dx, s);
                launch_dot(me, r, r, h->dotpart, h->sc + 3, s);
                launch_cg_beta(h->sc, s);  // beta = rr_new / rr, rr = rr_new
            });
        }
        rc = read_scalars(h, hs, 4, st);
        if (rc) return rc;
        cg_iters++;
        if (!(hs[1] > 0.0) || !std::isfinite(hs[1])) return CKKT_ERR_BREAKDOWN;
        if (std::sqrt(hs[3]) <= stop) return CKKT_OK;
    }
    cg_ok = false;
    return CKKT_OK;
}

ckkt_status solve_hykkt(ckkt_handle* h, const double* rhs, double* sol, ckkt_solve_info* info, hipStream_t st) {
    const int n = h->plan.n, me = h->plan.m_eq;
    const double* r1 = rhs;
    const double* r2 = rhs + n;
    double* x = sol;
    double* y = sol + n;
    double* res1 = h->vn[0];
    double* res2 = h->veq[3];
    double* ddx = h->vn[1];
    double* ddy = h->veq[4];
    launch_rhs_max(h, r1, n, r2, me, st);
    ckkt_status rc = CKKT_OK;
    {
        PhaseTimer tm(h, 3, st);
        launch_fill(n + me, 0.0, sol, st);
    }
    bool use64 = h->precision == CKKT_FP64 || h->fp64_factored;
    if (h->fp64_by_history) info->fallback = 8;
    ResidualOut r;
    // steps: outer steps taken (all factors); base: steps taken before the
    // current factor, so that the FP64 refactorization of the fallback gets
    // the full ir_maxit budget of its own, as in solve_lifted
    int steps = 0, base = 0, stall = 0;
    double prev = INFINITY;
    auto fall_back = [&]() {
        refactor_fp64(h, st);
        use64 = true;
        info->fallback = 2;
        stall = 0;
        prev = INFINITY;
        base = steps;
    };
    for (;;) {
        rc = residual_sync(h, x, y, r1, r2, res1, res2, r, st);
        if (rc) return rc;
        if ((rc = check_factor(h, r)) != CKKT_OK) return info->status = rc;
        if (steps == 0 && !std::isfinite(r.rhsmax)) return info->status = CKKT_ERR_NONFINITE;
        info->omega = r.omega;
        info->rho = r.rhsmax > 0 ? r.resmax / r.rhsmax : r.resmax;
        if (r.omega <= h->opt.tol && steps > 0) break;
        if (steps == 0 && !use64 && r.status1 > 0) fall_back();  // floored pivots: give up the FP32 factor at once
        if (steps > base && !use64) {
            if (!(r.omega < 0.5 * prev)) stall++;
            if (stall >= 2 || steps - base > h->opt.ir_maxit) fall_back();
        } else if (steps - base > h->opt.ir_maxit) {
            info->refine_steps = steps - 1;
            return CKKT_ERR_NO_CONVERGENCE;
        }
        prev = r.omega;
        int it = 0;
        bool ok = true;
        if (h->vals.delta_c > 0.0)
            primal_schur_inner(h, res1, res2, ddx, ddy, use64, st);
        else
            rc = hykkt_inner(h, res1, res2, ddx, ddy, use64, it, ok, st);
        info->cg_iters += it;
        if (rc == CKKT_ERR_BREAKDOWN && !use64) {
            // the FP32 factor of K_gamma is too inexact for CG on S_gamma:
            // refactorize in FP64 and redo this outer step
            fall_back();
            continue;
        }
        if (rc) return rc;
        {
            PhaseTimer tm(h, 3, st);
            launch_axpy(n, 1.0, ddx, x, st);
            launch_axpy(me, 1.0, ddy, y, st);
        }
        steps++;
    }
    info->refine_steps = steps - 1;
    return CKKT_OK;
}

// ------------------------------------------------ augmented system K2

// Newton step of K2 (Sec. 2.2, delta_c = 0) around the condensed factor:
// FP64 Richardson on K2 from d = 0, each correction K2 dd = R taken through
// the condensation (rbar1 = R1 + H^T (E R4 - R2), rbar2 = R3), the handle's
// condensed solve (LiftedKKT: one factor application; HyKKT: the CG step of
// hykkt_inner on K1) and the slack recovery (dz = R2 + E (H dx - R4),
// ds = (R2 - dz) / E).  Stops when the componentwise backward error of K2
// is <= opt.tol.
ckkt_status solve_augmented(ckkt_handle* h, const double* r1, const double* r2, const double* r3, const double* r4,
                            double* dx, double* ds, double* dy, double* dz, ckkt_solve_info* info, hipStream_t st) {
    const DevPlan& P = h->dp;
    const bool hy = h->formulation == CKKT_HYKKT;
    const int n = P.n, me = hy ? P.m_eq : 0, ms = P.m - me;
    // ddx, ddy: the buffers solve_hykkt gives hykkt_inner, so that the CG
    // iteration graph is shared by both solves
    double *R1 = h->vn[5], *rb1 = h->vn[6], *ddx = h->vn[1];
    double *R3 = h->veq[3], *ddy = h->veq[4];
    double *u = h->vk2[0], *R2 = h->vk2[1], *R4 = h->vk2[2], *dds = h->vk2[3], *ddz = h->vk2[4];
    unsigned long long* slot = h->bits + 2;
    {
        PhaseTimer tm(h, 3, st);
        launch_fill(n, 0.0, dx, st);
        launch_fill(ms, 0.0, ds, st);
        launch_fill(ms, 0.0, dz, st);
        launch_fill(me, 0.0, dy, st);
        launch_zero_u64(slot, 1, st);
        launch_maxabs(n, r1, slot, st);
        launch_maxabs(ms, r2, slot, st);
        launch_maxabs(me, r3, slot, st);
        launch_maxabs(ms, r4, slot, st);
    }
    bool use64 = h->precision == CKKT_FP64 || h->fp64_factored;
    // base: steps taken before the current factor (the FP64 refactorization
    // of the fallback gets the full ir_maxit budget of its own)
    int steps = 0, base = 0, stall = 0;
    double prev = INFINITY;
    auto fall_back = [&]() {
        refactor_fp64(h, st);
        use64 = true;
        info->fallback = 2;
        stall = 0;
        prev = INFINITY;
        base = steps;
    };
    char* host = static_cast<char*>(h->host);
    for (;;) {
        {
            PhaseTimer tm(h, 3, st);
            launch_zero_u64(h->bits, 2, st);
            launch_k2_residual(P, h->vals, h->d, r1, r2, r3, r4, dx, ds, dy, dz, R1, R2, R3, R4, h->bits,
                               h->bits + 1, st);
        }
        HIP_TRY(hipMemcpyAsync(host, h->bits, 3 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(host + 3 * sizeof(unsigned long long), h->status, 4 * sizeof(int32_t),
                               hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        const unsigned long long* hb = reinterpret_cast<const unsigned long long*>(host);
        const int32_t* hs = reinterpret_cast<const int32_t*>(host + 3 * sizeof(unsigned long long));
        if (hs[2]) return CKKT_ERR_TIMEOUT;
        ResidualOut r;
        r.status0 = hs[0];
        r.status3 = hs[3];
        if (ckkt_status fc = check_factor(h, r)) return fc;
        const double omega = bits_to_double(hb[0]), resmax = bits_to_double(hb[1]), rmax = bits_to_double(hb[2]);
        if (steps == 0 && !std::isfinite(rmax)) return CKKT_ERR_NONFINITE;
        info->omega = omega;
        info->rho = rmax > 0 ? resmax / rmax : resmax;
        if (omega <= h->opt.tol && steps > 0) break;
        if (steps > base && !use64) {
            if (!(omega < 0.5 * prev)) stall++;
            if (stall >= 2 || steps - base > h->opt.ir_maxit) fall_back();
        } else if (steps - base > h->opt.ir_maxit) {
            info->refine_steps = steps - 1;
            return CKKT_ERR_NO_CONVERGENCE;
        }
        prev = omega;
        {
            PhaseTimer tm(h, 3, st);
            launch_k2_condense(P, h->vals, h->d, R1, R2, R4, u, rb1, st);
        }
        if (hy) {
            int it = 0;
            bool ok = true;
            ckkt_status rc = hykkt_inner(h, rb1, R3, ddx, ddy, use64, it, ok, st);
            info->cg_iters += it;
            if (rc == CKKT_ERR_BREAKDOWN && !use64) {
                fall_back();
                continue;
            }
            if (rc) return rc;
        } else {
            apply_inverse(h, rb1, ddx, use64, st);
        }
        {
            PhaseTimer tm(h, 3, st);
            launch_k2_recover(P, h->vals, h->d, R2, R4, ddx, dds, ddz, st);
            launch_axpy(n, 1.0, ddx, dx, st);
            launch_axpy(ms, 1.0, dds, ds, st);
            launch_axpy(ms, 1.0, ddz, dz, st);
            launch_axpy(me, 1.0, ddy, dy, st);
        }
        steps++;
    }
    info->refine_steps = steps - 1;
    return CKKT_OK;
}

static bool inertia_params_ok(const ckkt_inertia* ic) {
    if (!ic) return false;
    auto pos = [](double v) { return std::isfinite(v) && v > 0.0; };
    return pos(ic->delta_w_min) && pos(ic->delta_w_0) && pos(ic->delta_w_max) && pos(ic->kappa_minus) &&
           ic->kappa_minus < 1.0 && pos(ic->kappa_plus) && ic->kappa_plus > 1.0 && pos(ic->kappa_plus_bar) &&
           ic->kappa_plus_bar > 1.0 && std::isfinite(ic->delta_w_last) && ic->delta_w_last >= 0.0;
}

// Inertia-controlling rule of Waechter & Biegler (2006, Sec. 3.1) without
// its zero-eigenvalue branch: `attempt(delta_w)` factorizes the system
// regularized by delta_w and returns CKKT_OK (positive definite, hence the
// inertia of K2 is correct by eq:ipm:inertia), CKKT_ERR_NOT_SPD, or another
// error that ends the search.  Every trial is larger than the one before by
// a factor > 1 and all are bounded by delta_w_max, so the loop ends.
template <class Attempt>
static ckkt_status inertia_search(ckkt_inertia* ic, Attempt attempt) {
    const bool history = ic->delta_w_last > 0.0;
    double delta = 0.0;
    ic->attempts = 0;
    for (;;) {
        ++ic->attempts;
        ic->delta_w = delta;
        const ckkt_status rc = attempt(delta);
        if (rc == CKKT_OK) {
            if (delta > 0.0) ic->delta_w_last = delta;
            return CKKT_OK;
        }
        if (rc != CKKT_ERR_NOT_SPD) return rc;
        if (delta == 0.0)
            delta = history ? std::max(ic->delta_w_min, ic->kappa_minus * ic->delta_w_last) : ic->delta_w_0;
        else
            delta *= history ? ic->kappa_plus : ic->kappa_plus_bar;
        if (!(delta <= ic->delta_w_max)) return CKKT_ERR_NOT_SPD;
    }
}

// ---------------------------------------------------- plan serialization

// Every field of the plan, in one order for writing and reading.
template <class A>
void plan_fields(Plan& P, A& a) {
    a.pod(P.n); a.pod(P.m_eq); a.pod(P.m_ineq); a.pod(P.m);
    a.pod(P.nnz_w); a.pod(P.nnz_g); a.pod(P.nnz_h);
    a.vec(P.perm); a.vec(P.iperm);
    a.vec(P.kcolptr); a.vec(P.krow); a.vec(P.k_wsrc); a.vec(P.k_diag);
    a.vec(P.prod_ptr); a.vec(P.prod_r); a.vec(P.prod_a); a.vec(P.prod_b); a.vec(P.dense_rows);
    a.pod(P.ns);
    a.vec(P.sn_start); a.vec(P.sn_rowptr); a.vec(P.sn_rows); a.vec(P.sn_parent);
    a.vec(P.child_ptr); a.vec(P.child_list); a.vec(P.relmap); a.vec(P.kmap); a.vec(P.kcol);
    a.vec(P.cb_ptr); a.vec(P.cb_src); a.vec(P.cb_len); a.vec(P.cb_uoff);
    a.vec(P.l_off); a.vec(P.u_off); a.vec(P.u_ld); a.vec(P.big);
    a.pod(P.arena); a.pod(P.nnz_l); a.pod(P.nnz_l_stored); a.pod(P.flops); a.pod(P.max_front); a.pod(P.n_big);
    a.pod(P.nlev);
    a.vec(P.sn_level); a.vec(P.lvl_ptr); a.vec(P.lvl_small); a.vec(P.lvl_small_ptr); a.vec(P.lvl_big);
    a.vec(P.lvl_big_ptr); a.vec(P.lvl_all); a.vec(P.lvl_all_ptr); a.vec(P.lvl_maxw_big);
    a.vec(P.big_tiles_ptr); a.vec(P.big_tile_sn); a.vec(P.big_tile_col);
    a.vec(P.wf_ptr); a.vec(P.wf_col); a.vec(P.wf_vidx);
    a.vec(P.j_ptr); a.vec(P.j_col);
    a.vec(P.jt_ptr); a.vec(P.jt_row); a.vec(P.jt_vidx); a.vec(P.jt_gend);
    a.pod(P.ninst); a.vec(P.inst_n); a.vec(P.inst_meq); a.vec(P.inst_of_var); a.vec(P.inst_of_eqrow);
    a.pod(P.analyze_seconds);
}

struct PlanWriter {
    std::vector<char> buf;
    template <class T>
    void pod(const T& v) {
        const char* p = reinterpret_cast<const char*>(&v);
        buf.insert(buf.end(), p, p + sizeof(T));
    }
    template <class T>
    void vec(const std::vector<T>& v) {
        pod((int64_t)v.size());
        const char* p = reinterpret_cast<const char*>(v.data());
        buf.insert(buf.end(), p, p + v.size() * sizeof(T));
    }
};

struct PlanReader {
    const char* p;
    const char* e;
    bool ok = true;
    template <class T>
    void pod(T& v) {
        if (!ok || (size_t)(e - p) < sizeof(T)) { ok = false; return; }
        std::memcpy(&v, p, sizeof(T));
        p += sizeof(T);
    }
    template <class T>
    void vec(std::vector<T>& v) {
        int64_t n = -1;
        pod(n);
        if (!ok || n < 0 || (uint64_t)n > (uint64_t)(e - p) / sizeof(T)) { ok = false; return; }
        v.resize((size_t)n);
        if (n > 0) std::memcpy(v.data(), p, (size_t)n * sizeof(T));
        p += (size_t)n * sizeof(T);
    }
};

// FNV-1a, 64 bit
uint64_t fnv1a(const char* p, size_t n) {
    uint64_t x = 1469598103934665603ull;
    for (size_t i = 0; i < n; ++i) {
        x ^= (unsigned char)p[i];
        x *= 1099511628211ull;
    }
    return x;
}

constexpr char kPlanMagic[8] = {'C', 'K', 'K', 'T', 'P', 'L', 'A', 'N'};
constexpr int32_t kPlanVersion = 1;

// header: magic, version, formulation, ordering, relax, lds front limit,
// dense_row_min (int32 each after the magic), payload length (int64);
// then the payload and its FNV-1a checksum
struct PlanHeader {
    char magic[8];
    int32_t version, formulation, ordering, relax, big_front, dense_row_min;
    int64_t payload;
};

std::vector<char> plan_blob(const ckkt_handle* h) {
    PlanWriter w;
    plan_fields(const_cast<Plan&>(h->plan), w);
    PlanHeader hd{};
    std::memcpy(hd.magic, kPlanMagic, 8);
    const AnalyzeOptions ao = analyze_options(h->opt);
    hd.version = kPlanVersion;
    hd.formulation = h->formulation;
    hd.ordering = h->opt.ordering;
    hd.relax = h->opt.relax;
    hd.big_front = ao.big_front;
    hd.dense_row_min = h->opt.dense_row_min;
    hd.payload = (int64_t)w.buf.size();
    std::vector<char> out(sizeof hd + w.buf.size() + sizeof(uint64_t));
    std::memcpy(out.data(), &hd, sizeof hd);
    std::memcpy(out.data() + sizeof hd, w.buf.data(), w.buf.size());
    const uint64_t sum = fnv1a(w.buf.data(), w.buf.size());
    std::memcpy(out.data() + sizeof hd + w.buf.size(), &sum, sizeof sum);
    return out;
}

}  // namespace

// ================================================================= C-ABI

extern "C" {

void ckkt_default_options(ckkt_options* o) {
    if (!o) return;
    o->precision = CKKT_FP64;
    o->ordering = CKKT_ORDER_AMD;
    o->tol = 1e-10;
    o->ir_maxit = 10;
    o->cg_tol = 1e-10;
    o->cg_maxit = 0;
    o->relax = 1;
    o->lds_front_max = 0;
    o->learned = 0;
}

void ckkt_default_inertia(ckkt_inertia* ic) {
    if (!ic) return;
    std::memset(ic, 0, sizeof(*ic));
    ic->delta_w_min = 1e-20;
    ic->delta_w_0 = 1e-4;
    ic->delta_w_max = 1e40;
    ic->kappa_minus = 1.0 / 3.0;
    ic->kappa_plus = 8.0;
    ic->kappa_plus_bar = 100.0;
}

static ckkt_status ckkt_analyze_impl(const ckkt_pattern* pat, const ckkt_options* opt, ckkt_handle** out,
                         size_t* workspace_bytes, SymbolicDevice* device = nullptr) {

    if (!out || !pattern_args_ok(pat)) return CKKT_ERR_ARG;
    *out = nullptr;
    HandlePtr h(new ckkt_handle());
    if (opt) h->opt = *opt;
    else ckkt_default_options(&h->opt);
    if (h->opt.precision != CKKT_FP64 && h->opt.precision != CKKT_FP32_IR) return CKKT_ERR_ARG;
    if (h->opt.ordering != CKKT_ORDER_AMD && h->opt.ordering != CKKT_ORDER_NATURAL) return CKKT_ERR_ARG;
    if (h->opt.dense_row_min < 0 || (h->opt.dense_row_min > 0 && h->opt.precision != CKKT_FP64))
        return CKKT_ERR_ARG;
    h->formulation = pat->formulation;
    h->precision = h->opt.precision;
    if (!pattern_ptrs_ok(pat)) return CKKT_ERR_PATTERN;
    PatternIn pin = copy_pattern(pat);
    AnalyzeOptions ao = analyze_options(h->opt);
    ao.device = device;
    return finish_analyze(std::move(h), ao, pin, out, workspace_bytes);
}

ckkt_status ckkt_analyze(const ckkt_pattern* pat, const ckkt_options* opt, ckkt_handle** out,
                         size_t* workspace_bytes) {
    try {
        return ckkt_analyze_impl(pat, opt, out, workspace_bytes);
    } catch (...) {  // std::bad_alloc, or a host thread that could not be started
        return CKKT_ERR_HOST_MEMORY;
    }
}

ckkt_status ckkt_analyze_device(const ckkt_pattern* pat, const ckkt_options* opt, void* stream, ckkt_handle** out,
                                size_t* workspace_bytes) {
    try {
        std::unique_ptr<SymbolicDevice> dev = make_symbolic_device(static_cast<hipStream_t>(stream));
        return ckkt_analyze_impl(pat, opt, out, workspace_bytes, dev.get());
    } catch (...) {
        return CKKT_ERR_HOST_MEMORY;
    }
}

static ckkt_status ckkt_plan_size_impl(const ckkt_handle* h, size_t* bytes) {

    if (!h || !bytes) return CKKT_ERR_ARG;
    *bytes = plan_blob(h).size();
    return CKKT_OK;
}

ckkt_status ckkt_plan_size(const ckkt_handle* h, size_t* bytes) {
    try {
        return ckkt_plan_size_impl(h, bytes);
    } catch (...) {  // std::bad_alloc, or a host thread that could not be started
        return CKKT_ERR_HOST_MEMORY;
    }
}

static ckkt_status ckkt_plan_save_impl(const ckkt_handle* h, void* buf, size_t bytes) {

    if (!h || !buf) return CKKT_ERR_ARG;
    const std::vector<char> blob = plan_blob(h);
    if (bytes < blob.size()) return CKKT_ERR_ARG;
    std::memcpy(buf, blob.data(), blob.size());
    return CKKT_OK;
}

ckkt_status ckkt_plan_save(const ckkt_handle* h, void* buf, size_t bytes) {
    try {
        return ckkt_plan_save_impl(h, buf, bytes);
    } catch (...) {  // std::bad_alloc, or a host thread that could not be started
        return CKKT_ERR_HOST_MEMORY;
    }
}

static ckkt_status ckkt_plan_load_impl(const void* buf, size_t bytes, const ckkt_options* opt, ckkt_handle** out,
                           size_t* workspace_bytes) {

    if (!out || !buf || bytes < sizeof(PlanHeader) + sizeof(uint64_t)) return CKKT_ERR_ARG;
    *out = nullptr;
    PlanHeader hd;
    std::memcpy(&hd, buf, sizeof hd);
    const char* base = static_cast<const char*>(buf);
    if (std::memcmp(hd.magic, kPlanMagic, 8) != 0 || hd.version != kPlanVersion || hd.payload < 0 ||
        (uint64_t)hd.payload != bytes - sizeof hd - sizeof(uint64_t))
        return CKKT_ERR_ARG;
    uint64_t sum;
    std::memcpy(&sum, base + sizeof hd + hd.payload, sizeof sum);
    if (sum != fnv1a(base + sizeof hd, (size_t)hd.payload)) return CKKT_ERR_ARG;
    if (hd.formulation != CKKT_LIFTED && hd.formulation != CKKT_HYKKT) return CKKT_ERR_ARG;
    HandlePtr h(new ckkt_handle());
    if (opt) h->opt = *opt;
    else ckkt_default_options(&h->opt);
    // the options that shaped the plan are the plan's
    h->opt.ordering = hd.ordering;
    h->opt.relax = hd.relax;
    h->opt.lds_front_max = hd.big_front;
    h->opt.dense_row_min = hd.dense_row_min;
    if ((h->opt.precision != CKKT_FP64 && h->opt.precision != CKKT_FP32_IR) ||
        (h->opt.dense_row_min > 0 && h->opt.precision != CKKT_FP64))
        return CKKT_ERR_ARG;
    h->formulation = hd.formulation;
    h->precision = h->opt.precision;
    PlanReader r{base + sizeof hd, base + sizeof hd + hd.payload};
    plan_fields(h->plan, r);
    if (!r.ok || r.p != r.e) return CKKT_ERR_ARG;
    if (h->plan.ninst > 1 && h->opt.dense_row_min != 0) return CKKT_ERR_ARG;
    const AnalyzeOptions ao = analyze_options(h->opt);
    return finish_plan(std::move(h), ao, out, workspace_bytes);
}

ckkt_status ckkt_plan_load(const void* buf, size_t bytes, const ckkt_options* opt, ckkt_handle** out,
                           size_t* workspace_bytes) {
    try {
        return ckkt_plan_load_impl(buf, bytes, opt, out, workspace_bytes);
    } catch (...) {  // std::bad_alloc, or a host thread that could not be started
        return CKKT_ERR_HOST_MEMORY;
    }
}

static ckkt_status ckkt_batch_analyze_impl(int32_t count, const ckkt_pattern* pats, const ckkt_options* opt,
                               ckkt_handle** out, size_t* workspace_bytes, SymbolicDevice* device = nullptr) {

    if (!out || count <= 0 || !pats) return CKKT_ERR_ARG;
    *out = nullptr;
    for (int i = 0; i < count; ++i) {
        if (!pattern_args_ok(&pats[i]) || pats[i].formulation != pats[0].formulation) return CKKT_ERR_ARG;
    }
    HandlePtr h(new ckkt_handle());
    if (opt) h->opt = *opt;
    else ckkt_default_options(&h->opt);
    if (h->opt.precision != CKKT_FP64 && h->opt.precision != CKKT_FP32_IR) return CKKT_ERR_ARG;
    if (h->opt.ordering != CKKT_ORDER_AMD && h->opt.ordering != CKKT_ORDER_NATURAL) return CKKT_ERR_ARG;
    if (h->opt.dense_row_min != 0) return CKKT_ERR_ARG;  // no dense-row split in a batch
    // every instance is a valid pattern on its own (indices below its own n)
    // before anything is built from it: the per-instance orderings and the
    // block-wise pair keys rely on that
    for (int i = 0; i < count; ++i) {
        if (!pattern_ptrs_ok(&pats[i])) return CKKT_ERR_PATTERN;
        if (!validate(copy_pattern(&pats[i])).empty()) return CKKT_ERR_PATTERN;
    }
    h->formulation = pats[0].formulation;
    h->precision = h->opt.precision;
    // block-diagonal union: variables and W blocks in instance order, then
    // all G rows (instance order), then all H rows (instance order)
    PatternIn u;
    int64_t n = 0, me = 0, mi = 0;
    for (int i = 0; i < count; ++i) { n += pats[i].n; me += pats[i].m_eq; mi += pats[i].m_ineq; }
    if (n > (int64_t)1 << 30) return CKKT_ERR_ARG;
    u.n = n; u.m_eq = me; u.m_ineq = mi;
    u.w_ptr.push_back(0); u.g_ptr.push_back(0); u.h_ptr.push_back(0);
    Plan& P = h->plan;
    P.ninst = count;
    P.inst_n.assign(count + 1, 0);
    P.inst_meq.assign(count + 1, 0);
    P.inst_of_var.assign(n, 0);
    P.inst_of_eqrow.assign(me, 0);
    int64_t off = 0, roff = 0;
    for (int i = 0; i < count; ++i) {
        const ckkt_pattern& p = pats[i];
        for (int64_t r = 0; r < p.n; ++r) {
            for (int32_t k = p.w_ptr[r]; k < p.w_ptr[r + 1]; ++k) u.w_idx.push_back((int32_t)(p.w_idx[k] + off));
            u.w_ptr.push_back((int32_t)u.w_idx.size());
            P.inst_of_var[off + r] = i;
        }
        for (int64_t r = 0; r < p.m_eq; ++r) {
            for (int32_t k = p.g_ptr[r]; k < p.g_ptr[r + 1]; ++k) u.g_idx.push_back((int32_t)(p.g_idx[k] + off));
            u.g_ptr.push_back((int32_t)u.g_idx.size());
            P.inst_of_eqrow[roff + r] = i;
        }
        for (int64_t r = 0; r < p.m_ineq; ++r) {
            for (int32_t k = p.h_ptr[r]; k < p.h_ptr[r + 1]; ++k) u.h_idx.push_back((int32_t)(p.h_idx[k] + off));
            u.h_ptr.push_back((int32_t)u.h_idx.size());
        }
        off += p.n;
        roff += p.m_eq;
        P.inst_n[i + 1] = (int32_t)off;
        P.inst_meq[i + 1] = (int32_t)roff;
    }
    AnalyzeOptions ao = analyze_options(h->opt);
    std::vector<int32_t> bn(P.inst_n), bg(P.inst_meq), bh(count + 1, 0);
    for (int i = 0; i < count; ++i) bh[i + 1] = bh[i] + (int32_t)pats[i].m_ineq;
    ao.block_n = &bn;
    ao.block_meq = &bg;
    ao.block_mineq = &bh;
    // The union graph is block diagonal: order every instance on its own,
    // instances spread over up to kAnalyzeThreads host threads, and hand the
    // concatenation to the analysis of the union.
    std::vector<int32_t> perm;
    if (h->opt.ordering == CKKT_ORDER_AMD) {
        std::vector<std::vector<int32_t>> orders(count);
        std::atomic<int> next{0};
        const int nthreads = std::max(1, std::min<int>({count, kAnalyzeThreads,
                                                        (int)std::max(1u, std::thread::hardware_concurrency())}));
        run_threads(nthreads, [&](int) {
            for (int i; (i = next.fetch_add(1)) < count;) orders[i] = order_pattern(copy_pattern(&pats[i]), 0);
        });
        perm.reserve(n);
        for (int i = 0; i < count; ++i)
            for (int32_t v : orders[i]) perm.push_back(v + P.inst_n[i]);
        ao.perm = &perm;
    }
    ao.device = device;
    return finish_analyze(std::move(h), ao, u, out, workspace_bytes);
}

ckkt_status ckkt_batch_analyze(int32_t count, const ckkt_pattern* pats, const ckkt_options* opt,
                               ckkt_handle** out, size_t* workspace_bytes) {
    try {
        return ckkt_batch_analyze_impl(count, pats, opt, out, workspace_bytes);
    } catch (...) {  // std::bad_alloc, or a host thread that could not be started
        return CKKT_ERR_HOST_MEMORY;
    }
}

ckkt_status ckkt_batch_analyze_device(int32_t count, const ckkt_pattern* pats, const ckkt_options* opt, void* stream,
                                      ckkt_handle** out, size_t* workspace_bytes) {
    try {
        std::unique_ptr<SymbolicDevice> dev = make_symbolic_device(static_cast<hipStream_t>(stream));
        return ckkt_batch_analyze_impl(count, pats, opt, out, workspace_bytes, dev.get());
    } catch (...) {
        return CKKT_ERR_HOST_MEMORY;
    }
}

ckkt_status ckkt_bind_workspace(ckkt_handle* h, void* dev_ptr, size_t bytes, void* stream) {
    if (!h) return CKKT_ERR_ARG;
    if (!dev_ptr || bytes < h->lay.total || (reinterpret_cast<uintptr_t>(dev_ptr) & 255)) return CKKT_ERR_WORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    (void)hipGetLastError();  // report only errors of this call's own launches
    if (!h->host) {
        h->host_bytes = (h->plan.ninst + 8) * sizeof(unsigned long long) + 64;
        if (hipHostMalloc(&h->host, h->host_bytes, hipHostMallocDefault) != hipSuccess) {
            h->host = nullptr;
            return CKKT_ERR_HIP;
        }
    }
    for (auto& g : h->graphs)
        if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
    if (!h->capture_stream) {
        if (hipStreamCreateWithFlags(&h->capture_stream, hipStreamNonBlocking) != hipSuccess) h->capture_stream = nullptr;
    }
    if (!h->side.stream) {
        SideStream& sd = h->side;
        if (hipStreamCreateWithFlags(&sd.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sd.fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&sd.join, hipEventDisableTiming) != hipSuccess) {
            destroy_side(sd);
            (void)hipGetLastError();
        }
    }
    const char* ng = std::getenv("CKKT_NO_GRAPH");
    h->use_graphs = !(ng && ng[0] == '1');
    const char* dl = std::getenv("CKKT_DEBUG_LAUNCH");
    h->debug_launch = dl && dl[0] == '1';
    h->ws = static_cast<char*>(dev_ptr);
    h->ws_bytes = bytes;
    for (auto& pr : h->plan_regions)
        if (pr.r.bytes > 0)
            HIP_TRY(hipMemcpyAsync(h->ws + pr.r.off, pr.host, pr.r.bytes, hipMemcpyHostToDevice, st));
    // sweep flags start below every epoch the sweeps will use
    HIP_TRY(hipMemsetAsync(h->ws + h->r_ctl.off, 0, h->r_ctl.bytes, st));
    HIP_TRY(hipMemsetAsync(h->ws + h->r_done.off, 0, h->r_done.bytes, st));
    HIP_TRY(hipMemsetAsync(h->ws + h->r_tflag.off, 0, h->r_tflag.bytes, st));
    {
        // tiled fronts swept in one launch per level (CKKT_TILED_LEVEL=0:
        // one launch per column block), with flag waits bounded in time
        int dev = 0, khz = 0;
        const char* tl = std::getenv("CKKT_TILED_LEVEL");
        h->tiled_level = !(tl && tl[0] == '0') && hipGetDevice(&dev) == hipSuccess &&
                         hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0;
        (void)hipGetLastError();
        h->wait_ticks = (unsigned long long)std::max(khz, 1) * 1000ull * kSweepWaitSeconds;
    }
    HIP_TRY(hipMemsetAsync(h->ws + h->r_status.off, 0, h->r_status.bytes, st));
    HIP_TRY(hipStreamSynchronize(st));
    fill_devplan(h);
    // Sweep schedule.  Default: the levels of single-wave fronts (order <=
    // 64, thousands of supernodes) level by level, the levels above
    // dependency-driven (workgroups taking supernodes in level order and
    // waiting on their children's or parent's flags): on this chip a
    // device-scope release per supernode (an L2 write-back on every
    // producer) costs more than a kernel boundary when a level holds
    // thousands of supernodes, less when it holds a few.  Plans with fronts
    // for the tiled sweeps stay level by level (a workgroup worker would
    // sweep such a front alone).  CKKT_DEP_SWEEPS=0: level by level
    // throughout; 1: dependency-driven throughout; 2: the default form.
    // The default takes the hybrid only while few supernodes lie above the
    // single-wave levels (kHybridMaxTasks): a batch of hundreds of
    // instances has thousands there and sweeps faster level by level.
    const char* ds = std::getenv("CKKT_DEP_SWEEPS");
    const char mode = ds ? ds[0] : (h->n_tflags == 0 ? '2' : '0');
    h->sched_ok = (mode == '1' || mode == '2') && build_sweep_sched(h);
    if (h->sched_ok && !ds && h->sched.ns - h->sched.wave_t1 > kHybridMaxTasks) h->sched_ok = false;
    h->sched_hybrid = h->sched_ok && mode == '2';
    h->factored = false;
    h->fp64_factored = false;
    return CKKT_OK;
}

ckkt_status ckkt_factorize(ckkt_handle* h, const double* w_val, const double* g_val, const double* h_val,
                           const double* sigma_x, const double* sigma_s, double gamma, void* stream) {
    if (!h) return CKKT_ERR_ARG;
    if (!h->ws) return CKKT_ERR_STATE;
    const Plan& P = h->plan;
    if ((P.nnz_w > 0 && !w_val) || (P.nnz_g > 0 && !g_val) || (P.nnz_h > 0 && !h_val) || (P.n > 0 && !sigma_x))
        return CKKT_ERR_ARG;
    int64_t ns_len = h->formulation == CKKT_HYKKT ? P.m_ineq : P.m;
    if (ns_len > 0 && !sigma_s) return CKKT_ERR_ARG;
    if (h->formulation == CKKT_HYKKT && P.m_eq > 0 && !(gamma > 0.0 && std::isfinite(gamma))) return CKKT_ERR_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    (void)hipGetLastError();  // report only errors of this call's own launches
    h->vals = SysVals{w_val, g_val, h_val, sigma_x, sigma_s, gamma};
    h->failed_column = -1;
    h->fp64_factored = false;
    // FP32_IR: FP64 from the start while an earlier FP32 failure is recent
    h->fp64_by_history = h->precision == CKKT_FP32_IR && h->fp32_skip > 0;
    if (h->fp64_by_history) h->fp32_skip--;
    const bool use32 = h->precision == CKKT_FP32_IR && !h->fp64_by_history;
    {
        PhaseTimer tm(h, 0, st);
        launch_init_status(h->status, false, st);
        launch_row_weights(h->dp, h->vals, h->d, st);
        launch_assemble(h->dp, h->vals, h->d, h->K, h->status + 3, st);
        if (use32) launch_diag_scale(h->dp, h->K, h->scale, st);
        if (h->opt.learned) {
            // the factorized system becomes the stale reference of the learned PCG
            launch_copy(h->plan.n, sigma_x, h->sxold, st);
            launch_copy(h->plan.m, h->d, h->dold, st);
            launch_kdiag(h->dp, h->vals, h->d, h->kdold, st);
            h->stale_valid = true;
        }
    }
    {
        PhaseTimer tm(h, 1, st);
        if (!use32) {
            factor_all<double>(h, nullptr, st);
            h->fp64_factored = true;
        } else {
            factor_all<float>(h, h->scale, st);
        }
    }
    if (!use32) dense_rows_setup(h, st);
    if (hipGetLastError() != hipSuccess) return CKKT_ERR_HIP;
    h->factored = true;
    return CKKT_OK;
}

ckkt_status ckkt_factorize_dual_reg(ckkt_handle* h, const double* w_val, const double* g_val, const double* h_val,
                                    const double* sigma_x, const double* sigma_s, double delta_c, void* stream) {
    if (!h) return CKKT_ERR_ARG;
    const double gamma = 1.0 / delta_c;
    if (h->formulation != CKKT_HYKKT || !(delta_c > 0.0) || !std::isfinite(delta_c) || !std::isfinite(gamma) ||
        !(gamma > 0.0))
        return CKKT_ERR_ARG;
    ckkt_status rc = ckkt_factorize(h, w_val, g_val, h_val, sigma_x, sigma_s, gamma, stream);
    if (rc != CKKT_OK) return rc;
    h->vals.delta_c = delta_c;  // ckkt_factorize leaves it 0; ckkt_solve now takes the direct path
    return CKKT_OK;
}

ckkt_status ckkt_factor_status(ckkt_handle* h, void* stream) {
    if (!h) return CKKT_ERR_ARG;
    if (!h->factored) return CKKT_ERR_STATE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    (void)hipGetLastError();  // report only errors of this call's own launches
    HIP_TRY(hipMemcpyAsync(h->host, h->status, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    int32_t s0 = static_cast<int32_t*>(h->host)[0];
    if (static_cast<int32_t*>(h->host)[2] != 0) return CKKT_ERR_TIMEOUT;
    if (static_cast<int32_t*>(h->host)[3] != 0) return CKKT_ERR_NONFINITE;
    if (h->fp64_factored && s0 != INT_MAX) {
        h->failed_column = (s0 >= 0 && s0 < h->plan.n) ? h->plan.perm[s0] : s0;
        return CKKT_ERR_NOT_SPD;
    }
    return CKKT_OK;
}

ckkt_status ckkt_factorize_inertia(ckkt_handle* h, const double* w_val, const double* g_val, const double* h_val,
                                   const double* sigma_x, const double* sigma_s, double gamma, ckkt_inertia* ic,
                                   void* stream) {
    if (!h || !inertia_params_ok(ic)) return CKKT_ERR_ARG;
    if (h->precision != CKKT_FP64 || h->plan.ninst > 1 || !h->plan.dense_rows.empty()) return CKKT_ERR_ARG;
    if (!h->ws) return CKKT_ERR_STATE;
    const Plan& P = h->plan;
    const int64_t ns_len = h->formulation == CKKT_HYKKT ? P.m_ineq : P.m;
    if ((P.n > 0 && !sigma_x) || (ns_len > 0 && !sigma_s)) return CKKT_ERR_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    return inertia_search(ic, [&](double delta) -> ckkt_status {
        (void)hipGetLastError();  // report only errors of this trial's own launches
        launch_shift_copy((int)P.n, sigma_x, delta, h->sxreg, st);
        launch_shift_copy((int)ns_len, sigma_s, delta, h->ssreg, st);
        if (hipGetLastError() != hipSuccess) return CKKT_ERR_HIP;
        ckkt_status rc = ckkt_factorize(h, w_val, g_val, h_val, h->sxreg, h->ssreg, gamma, stream);
        return rc != CKKT_OK ? rc : ckkt_factor_status(h, stream);
    });
}

ckkt_status ckkt_solve(ckkt_handle* h, const double* rhs, double* sol, ckkt_solve_info* info, void* stream) {
    ckkt_solve_info local{};
    if (!info) info = &local;
    std::memset(info, 0, sizeof(*info));
    if (!h) return info->status = CKKT_ERR_ARG;
    if (!h->ws || !h->factored) return info->status = CKKT_ERR_STATE;
    if ((h->plan.n > 0 || h->plan.m_eq > 0) && (!rhs || !sol)) return info->status = CKKT_ERR_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    (void)hipGetLastError();  // report only errors of this call's own launches
    ckkt_status rc = h->formulation == CKKT_HYKKT ? solve_hykkt(h, rhs, sol, info, st)
                                                   : solve_lifted(h, rhs, sol, info, st);
    if (rc == CKKT_OK && hipGetLastError() != hipSuccess) rc = CKKT_ERR_HIP;
    if (rc == CKKT_OK) note_fp32_outcome(h, info);
    info->status = rc;
    return rc;
}

// The launches of ckkt_batch_factorize_solve: assembly, factorization,
// x = K^{-1} b, `refine` refinement steps whose update is applied only to
// the instances still above the tolerance, and the residual of the result.
void factorize_solve_launches(ckkt_handle* h, bool d, int refine, const double* b, double* x, hipStream_t s) {
    const int ni = h->plan.ninst;
    double* res = h->vn[0];
    double* dx = h->vn[1];
    launch_init_status(h->status, false, s);
    launch_row_weights(h->dp, h->vals, h->d, s);
    launch_assemble(h->dp, h->vals, h->d, h->K, h->status + 3, s);
    if (d) {
        factor_levels<double>(h, nullptr, s);
    } else {
        launch_diag_scale(h->dp, h->K, h->scale, s);
        factor_levels<float>(h, h->scale, s);
    }
    launch_rhs_max(h, b, h->plan.n, nullptr, 0, s);
    apply_inverse_launches(h, b, x, d, s);
    for (int k = 0; k <= refine; ++k) {
        launch_zero_u64(h->bits, ni + 1, s);
        launch_residual(h->dp, h->vals, h->d, x, nullptr, b, nullptr, res, nullptr, h->vm[0], h->vm[1], h->bits,
                        h->bits + ni, s);
        if (k == refine) break;
        apply_inverse_launches(h, res, dx, d, s);
        launch_masked_axpy(h->dp, h->bits, h->opt.tol, dx, x, s);
    }
}

ckkt_status ckkt_batch_factorize_solve(ckkt_handle* h, const double* w_val, const double* g_val,
                                       const double* h_val, const double* sigma_x, const double* sigma_s,
                                       const double* rhs, double* sol, int32_t refine, double* inst_omega,
                                       ckkt_solve_info* info, void* stream) {
    ckkt_solve_info local{};
    if (!info) info = &local;
    std::memset(info, 0, sizeof(*info));
    if (!h) return info->status = CKKT_ERR_ARG;
    if (!h->ws) return info->status = CKKT_ERR_STATE;
    const Plan& P = h->plan;
    if (h->formulation != CKKT_LIFTED || !P.dense_rows.empty() || refine < 0 || refine > CKKT_MAX_DEVICE_REFINE)
        return info->status = CKKT_ERR_ARG;
    if ((P.nnz_w > 0 && !w_val) || (P.nnz_g > 0 && !g_val) || (P.nnz_h > 0 && !h_val) ||
        (P.n > 0 && (!sigma_x || !rhs || !sol)) || (P.m > 0 && !sigma_s))
        return info->status = CKKT_ERR_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    (void)hipGetLastError();  // report only errors of this call's own launches
    h->vals = SysVals{w_val, g_val, h_val, sigma_x, sigma_s, 0.0};
    h->failed_column = -1;
    h->factored = false;
    // FP32_IR: FP64 from the start while an earlier FP32 failure is recent
    // (the policy of ckkt_factorize)
    h->fp64_by_history = h->precision == CKKT_FP32_IR && h->fp32_skip > 0;
    if (h->fp64_by_history) h->fp32_skip--;
    const bool d = h->precision == CKKT_FP64 || h->fp64_by_history;
    h->fp64_factored = d;
    // an FP64 factor chosen by that policy takes at most one device step
    // (the tolerance of an FP32_IR handle is the metric's 1e-8); the host
    // refinement covers the rare rest
    if (h->fp64_by_history) refine = std::min(refine, 1);
    // the captured sequence holds the caller's pointers: captured again
    // when any of them (or the step count) differs from the last call's
    const int slot = d ? 6 : 7;
    const void* key[8] = {w_val, g_val, h_val, sigma_x, sigma_s, rhs, sol,
                          reinterpret_cast<const void*>(static_cast<intptr_t>(refine))};
    const void** held = h->fs_key[slot - 6];
    if (h->graphs[slot] && !std::equal(key, key + 8, held)) {
        (void)hipGraphExecDestroy(h->graphs[slot]);
        h->graphs[slot] = nullptr;
    }
    std::copy(key, key + 8, held);
    {
        PhaseTimer tm(h, 1, st);
        run_captured(h, slot, st, [&](hipStream_t s) { factorize_solve_launches(h, d, refine, rhs, sol, s); });
    }
    if (hipGetLastError() != hipSuccess) return info->status = CKKT_ERR_HIP;
    h->factored = true;
    ResidualOut r;
    ckkt_status rc = read_residual(h, r, st);  // the call's one host synchronization
    if (rc) return info->status = rc;
    if ((rc = check_factor(h, r)) != CKKT_OK) return info->status = rc;
    if (!std::isfinite(r.rhsmax)) return info->status = CKKT_ERR_NONFINITE;
    info->refine_steps = refine;
    if (!(r.omega <= h->opt.tol)) {
        // some instance is still above the tolerance: the refinement of
        // ckkt_solve (with its fallbacks for an FP32 factor) continues from
        // the iterate of the device steps
        ckkt_solve_info more{};
        rc = solve_lifted(h, rhs, sol, &more, st, refine);
        info->refine_steps = more.refine_steps;
        info->pcg_iters = more.pcg_iters;
        info->fallback = more.fallback | 4;
        if (rc) return info->status = rc;
        note_fp32_outcome(h, &more);
        if ((rc = read_residual(h, r, st)) != CKKT_OK) return info->status = rc;
    } else {
        note_fp32_outcome(h, info);  // the FP32 factor met the tolerance
    }
    if (h->fp64_by_history) info->fallback |= 8;
    info->omega = r.omega;
    info->rho = r.rhsmax > 0 ? r.resmax / r.rhsmax : r.resmax;
    if (inst_omega) std::copy(r.per_inst.begin(), r.per_inst.end(), inst_omega);
    if (hipGetLastError() != hipSuccess) rc = CKKT_ERR_HIP;
    return info->status = rc;
}

ckkt_status ckkt_solve_augmented(ckkt_handle* h, const double* r1, const double* r2, const double* r3,
                                 const double* r4, double* dx, double* ds, double* dy, double* dz,
                                 ckkt_solve_info* info, void* stream) {
    ckkt_solve_info local{};
    if (!info) info = &local;
    std::memset(info, 0, sizeof(*info));
    if (!h || h->plan.ninst > 1) return info->status = CKKT_ERR_ARG;
    if (!h->ws || !h->factored) return info->status = CKKT_ERR_STATE;
    if (h->vals.delta_c != 0.0) return info->status = CKKT_ERR_STATE;
    const Plan& P = h->plan;
    const bool hy = h->formulation == CKKT_HYKKT;
    const int64_t me = hy ? P.m_eq : 0, ms = P.m - me;
    if ((P.n > 0 && (!r1 || !dx)) || (ms > 0 && (!r2 || !r4 || !ds || !dz)) || (me > 0 && (!r3 || !dy)))
        return info->status = CKKT_ERR_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    (void)hipGetLastError();  // report only errors of this call's own launches
    ckkt_status rc = solve_augmented(h, r1, r2, r3, r4, dx, ds, dy, dz, info, st);
    if (rc == CKKT_OK && hipGetLastError() != hipSuccess) rc = CKKT_ERR_HIP;
    return info->status = rc;
}

ckkt_status ckkt_recover_bound_dual(int64_t count, const double* s, const double* v, double mu, const double* ds,
                                   double* dv, void* stream) {
    if (count < 0 || (count > 0 && (!s || !v || !ds || !dv)) || !std::isfinite(mu)) return CKKT_ERR_ARG;
    if (count == 0) return CKKT_OK;
    (void)hipGetLastError();  // report only errors of this call's own launches
    launch_bound_dual(count, s, v, mu, ds, dv, static_cast<hipStream_t>(stream));
    return hipGetLastError() == hipSuccess ? CKKT_OK : CKKT_ERR_HIP;
}

ckkt_status ckkt_apply_inverse(ckkt_handle* h, const double* rhs, double* sol, void* stream) {
    if (!h) return CKKT_ERR_ARG;
    if (!h->ws || !h->factored) return CKKT_ERR_STATE;
    if (h->plan.n > 0 && (!rhs || !sol)) return CKKT_ERR_ARG;
    (void)hipGetLastError();  // report only errors of this call's own launches
    apply_inverse(h, rhs, sol, h->fp64_factored, static_cast<hipStream_t>(stream));
    return hipGetLastError() == hipSuccess ? CKKT_OK : CKKT_ERR_HIP;
}

ckkt_status ckkt_export_k(ckkt_handle* h, int32_t* rows, int32_t* cols, double* values, void* stream) {
    if (!h) return CKKT_ERR_ARG;
    const Plan& P = h->plan;
    if (rows || cols) {
        for (int32_t j = 0; j < P.n; ++j)
            for (int32_t t = P.kcolptr[j]; t < P.kcolptr[j + 1]; ++t) {
                int32_t a = P.perm[P.krow[t]], b = P.perm[j];
                if (rows) rows[t] = std::max(a, b);
                if (cols) cols[t] = std::min(a, b);
            }
    }
    if (values) {
        if (!h->ws || !h->factored) return CKKT_ERR_STATE;
        hipStream_t st = static_cast<hipStream_t>(stream);
        (void)hipGetLastError();  // report only errors of this call's own launches
        HIP_TRY(hipMemcpyAsync(values, h->K, P.kcolptr.back() * sizeof(double), hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    return CKKT_OK;
}

static ckkt_status ckkt_host_factor_solve_impl(const ckkt_handle* h, const double* w_val, const double* g_val,
                                  const double* h_val, const double* sigma_x, const double* sigma_s,
                                  double gamma, const double* rhs, double* sol, int32_t* failed_column) {

    if (!h || !rhs || !sol) return CKKT_ERR_ARG;
    const Plan& P = h->plan;
    const bool hy = h->formulation == CKKT_HYKKT;
    int fc = host_factor_solve(P, hy, w_val, g_val, h_val, sigma_x, sigma_s, gamma, rhs, sol);
    if (failed_column) *failed_column = fc;
    if (fc >= 0) return CKKT_ERR_NOT_SPD;
    const int k = (int)P.dense_rows.size(), n = P.n;
    if (k == 0) return CKKT_OK;
    // Woodbury around K_s: sol -= Z C^{-1} (J_d sol), Z = K_s^{-1} J_d^T,
    // C = D_d^{-1} + J_d Z (each column of Z by a host run of its own)
    auto jv = [&](int32_t a) { return a < P.nnz_g ? g_val[a] : h_val[a - P.nnz_g]; };
    auto weight = [&](int32_t r) { return hy ? (r < P.m_eq ? gamma : sigma_s[r - P.m_eq]) : sigma_s[r]; };
    std::vector<double> jd((size_t)k * n, 0.0), z((size_t)k * n), c((size_t)k * k), t(k);
    for (int b = 0; b < k; ++b) {
        const int32_t r = P.dense_rows[b];
        for (int32_t a = P.j_ptr[r]; a < P.j_ptr[r + 1]; ++a) jd[(size_t)b * n + P.j_col[a]] = jv(a);
        if (host_factor_solve(P, hy, w_val, g_val, h_val, sigma_x, sigma_s, gamma, &jd[(size_t)b * n],
                              &z[(size_t)b * n]) >= 0)
            return CKKT_ERR_NOT_SPD;
    }
    for (int a = 0; a < k; ++a)
        for (int e = 0; e <= a; ++e) {
            double acc = 0.0;
            for (int i = 0; i < n; ++i) acc += jd[(size_t)a * n + i] * z[(size_t)e * n + i];
            c[a * k + e] = acc + (a == e ? 1.0 / weight(P.dense_rows[a]) : 0.0);
        }
    for (int j = 0; j < k; ++j) {  // Cholesky, lower
        double dj = c[j * k + j];
        for (int l = 0; l < j; ++l) dj -= c[j * k + l] * c[j * k + l];
        if (!(dj > 0.0)) {
            if (failed_column) *failed_column = n;
            return CKKT_ERR_NOT_SPD;
        }
        c[j * k + j] = std::sqrt(dj);
        for (int i = j + 1; i < k; ++i) {
            double v = c[i * k + j];
            for (int l = 0; l < j; ++l) v -= c[i * k + l] * c[j * k + l];
            c[i * k + j] = v / c[j * k + j];
        }
    }
    for (int b = 0; b < k; ++b) {
        double acc = 0.0;
        for (int i = 0; i < n; ++i) acc += jd[(size_t)b * n + i] * sol[i];
        for (int l = 0; l < b; ++l) acc -= c[b * k + l] * t[l];
        t[b] = acc / c[b * k + b];
    }
    for (int b = k - 1; b >= 0; --b) {
        double v = t[b];
        for (int l = b + 1; l < k; ++l) v -= c[l * k + b] * t[l];
        t[b] = v / c[b * k + b];
    }
    for (int i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int b = 0; b < k; ++b) acc += z[(size_t)b * n + i] * t[b];
        sol[i] -= acc;
    }
    return CKKT_OK;
}

ckkt_status ckkt_host_factor_solve(const ckkt_handle* h, const double* w_val, const double* g_val,
                                  const double* h_val, const double* sigma_x, const double* sigma_s,
                                  double gamma, const double* rhs, double* sol, int32_t* failed_column) {
    try {
        return ckkt_host_factor_solve_impl(h, w_val, g_val, h_val, sigma_x, sigma_s, gamma, rhs, sol, failed_column);
    } catch (...) {  // std::bad_alloc, or a host thread that could not be started
        return CKKT_ERR_HOST_MEMORY;
    }
}

static ckkt_status ckkt_host_factor_solve_inertia_impl(const ckkt_handle* h, const double* w_val, const double* g_val,
                                           const double* h_val, const double* sigma_x, const double* sigma_s,
                                           double gamma, ckkt_inertia* ic, const double* rhs, double* sol) {

    if (!h || !rhs || !sol || !inertia_params_ok(ic) || h->plan.ninst > 1 || !h->plan.dense_rows.empty())
        return CKKT_ERR_ARG;
    const Plan& P = h->plan;
    const bool hy = h->formulation == CKKT_HYKKT;
    const int64_t ns_len = hy ? P.m_ineq : P.m;
    if ((P.n > 0 && !sigma_x) || (ns_len > 0 && !sigma_s)) return CKKT_ERR_ARG;
    std::vector<double> sx(P.n), ss(ns_len);
    return inertia_search(ic, [&](double delta) -> ckkt_status {
        for (int64_t i = 0; i < P.n; ++i) sx[i] = sigma_x[i] + delta;
        for (int64_t r = 0; r < ns_len; ++r) ss[r] = sigma_s[r] + delta;
        int fc = host_factor_solve(P, hy, w_val, g_val, h_val, sx.data(), ss.data(), gamma, rhs, sol);
        return fc >= 0 ? CKKT_ERR_NOT_SPD : CKKT_OK;
    });
}

ckkt_status ckkt_host_factor_solve_inertia(const ckkt_handle* h, const double* w_val, const double* g_val,
                                           const double* h_val, const double* sigma_x, const double* sigma_s,
                                           double gamma, ckkt_inertia* ic, const double* rhs, double* sol) {
    try {
        return ckkt_host_factor_solve_inertia_impl(h, w_val, g_val, h_val, sigma_x, sigma_s, gamma, ic, rhs, sol);
    } catch (...) {  // std::bad_alloc, or a host thread that could not be started
        return CKKT_ERR_HOST_MEMORY;
    }
}

static ckkt_status set_new_values(ckkt_handle* h, const double* w_val, const double* g_val, const double* h_val,
                                  const double* sigma_x, const double* sigma_s, double gamma, hipStream_t st) {
    const Plan& P = h->plan;
    if ((P.nnz_w > 0 && !w_val) || (P.nnz_g > 0 && !g_val) || (P.nnz_h > 0 && !h_val) || (P.n > 0 && !sigma_x))
        return CKKT_ERR_ARG;
    int64_t ns_len = h->formulation == CKKT_HYKKT ? P.m_ineq : P.m;
    if (ns_len > 0 && !sigma_s) return CKKT_ERR_ARG;
    h->vals = SysVals{w_val, g_val, h_val, sigma_x, sigma_s, gamma};
    launch_row_weights(h->dp, h->vals, h->d, st);
    return CKKT_OK;
}

static ckkt_status learned_ready(ckkt_handle* h) {
    if (!h) return CKKT_ERR_ARG;
    if (!h->opt.learned) return CKKT_ERR_ARG;
    if (!h->ws || !h->factored || !h->stale_valid) return CKKT_ERR_STATE;
    return CKKT_OK;
}

// features of the current values (h->vals, h->d) against the stale system
static void compute_features(ckkt_handle* h, float* out, hipStream_t st) {
    launch_copy(h->plan.m, h->d, h->dnew, st);
    launch_kdiag(h->dp, h->vals, h->dnew, h->kdnew, st);
    launch_features(h->dp, h->vals.sigma_x, h->dnew, h->kdnew, h->sxold, h->dold, h->kdold, out, st);
}

ckkt_status ckkt_features(ckkt_handle* h, const double* w_val, const double* g_val, const double* h_val,
                          const double* sigma_x, const double* sigma_s, double gamma, float* features,
                          void* stream) {
    ckkt_status rc = learned_ready(h);
    if (rc) return rc;
    if (!features && h->plan.n > 0) return CKKT_ERR_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    (void)hipGetLastError();  // report only errors of this call's own launches
    rc = set_new_values(h, w_val, g_val, h_val, sigma_x, sigma_s, gamma, st);
    if (rc) return rc;
    compute_features(h, features, st);
    return hipGetLastError() == hipSuccess ? CKKT_OK : CKKT_ERR_HIP;
}

ckkt_status ckkt_mlp_forward(int64_t n, const float* features, const float* params, float* out, float* cache,
                             void* stream) {
    if (n < 0 || (n > 0 && (!features || !params || !out))) return CKKT_ERR_ARG;
    launch_mlp_forward(n, features, params, out, cache, static_cast<hipStream_t>(stream));
    return hipGetLastError() == hipSuccess ? CKKT_OK : CKKT_ERR_HIP;
}

size_t ckkt_mlp_workspace(int64_t n) { return n < 0 ? 0 : mlp_workspace_bytes(n); }

ckkt_status ckkt_mlp_backward(int64_t n, const float* features, const float* params, const float* cache,
                              const float* g_out, float* grad, void* ws, void* stream) {
    if (n < 0 || !params || !grad || !ws || (n > 0 && (!features || !cache || !g_out))) return CKKT_ERR_ARG;
    launch_mlp_backward(n, features, params, cache, g_out, grad, ws, static_cast<hipStream_t>(stream));
    return hipGetLastError() == hipSuccess ? CKKT_OK : CKKT_ERR_HIP;
}

ckkt_status ckkt_mlp_backward_noalloc(int64_t n, const float* features, const float* params, const float* cache,
                                      const float* g_out, float* grad, void* stream) {
    static_assert(CKKT_MLP_NOALLOC_MAX_ROWS == kMlpNoAllocRows, "row limit of the static scratch");
    if (n < 0 || n > CKKT_MLP_NOALLOC_MAX_ROWS) return CKKT_ERR_ARG;
    if (!params || !grad || (n > 0 && (!features || !cache || !g_out))) return CKKT_ERR_ARG;
    (void)hipGetLastError();  // report only errors of this call's own launches
    hipError_t e = hipSuccess;
    void* ws = mlp_noalloc_scratch(&e);
    if (!ws) return CKKT_ERR_HIP;
    launch_mlp_backward(n, features, params, cache, g_out, grad, ws, static_cast<hipStream_t>(stream));
    return hipGetLastError() == hipSuccess ? CKKT_OK : CKKT_ERR_HIP;
}

ckkt_status ckkt_adam(int32_t nparam, float* params, const float* grad, float* m, float* v, int32_t step,
                      float lr, void* stream) {
    if (nparam < 0 || step < 1 || (nparam > 0 && (!params || !grad || !m || !v))) return CKKT_ERR_ARG;
    launch_adam(nparam, params, grad, m, v, step, lr, static_cast<hipStream_t>(stream));
    return hipGetLastError() == hipSuccess ? CKKT_OK : CKKT_ERR_HIP;
}

ckkt_status ckkt_mlp_train_step(ckkt_handle* h, const double* w_val, const double* g_val, const double* h_val,
                                const double* sigma_x, const double* sigma_s, double gamma, const double* rhs,
                                const double* target, float* params, float* m, float* v, int32_t step, float lr,
                                double* loss, void* stream) {
    ckkt_status rc = learned_ready(h);
    if (rc) return rc;
    if (h->formulation != CKKT_LIFTED) return CKKT_ERR_ARG;
    const int n = h->plan.n;
    if (n > 0 && (!rhs || !target)) return CKKT_ERR_ARG;
    if (!params || !m || !v || step < 1) return CKKT_ERR_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    (void)hipGetLastError();  // report only errors of this call's own launches
    rc = set_new_values(h, w_val, g_val, h_val, sigma_x, sigma_s, gamma, st);
    if (rc) return rc;
    const bool use64 = h->fp64_factored;
    double *y = h->lv[0], *e = h->lv[1], *w = h->lv[2], *t = h->lv[3];
    double* sc = h->sc + 13;  // [0] e.e, [1] x.x
    compute_features(h, h->feat, st);
    launch_mlp_forward(n, h->feat, params, h->mo, h->cache, st);
    launch_dscale(n, h->mo, rhs, t, st);            // D b
    apply_inverse(h, t, y, use64, st);               // y = K_s^{-1} D b
    launch_train_err(n, h->mo, y, target, e, st);    // e = D y - x
    launch_dot(n, e, e, h->dotpart, sc + 0, st);
    launch_dot(n, target, target, h->dotpart, sc + 1, st);
    launch_train_gzD(n, h->mo, e, sc, t, st);        // D g_z
    apply_inverse(h, t, w, use64, st);               // w = K_s^{-1} D g_z
    launch_train_go(n, h->mo, e, y, rhs, w, sc, h->go, st);
    launch_mlp_backward(n, h->feat, params, h->cache, h->go, h->grad, h->mlpws, st);
    launch_adam(kMlpNParam, params, h->grad, m, v, step, lr, st);
    double hs[2];
    HIP_TRY(hipMemcpyAsync(h->host, sc, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    std::memcpy(hs, h->host, sizeof(hs));
    if (loss) *loss = hs[1] > 0 ? hs[0] / hs[1] : 0.0;
    return hipGetLastError() == hipSuccess ? CKKT_OK : CKKT_ERR_HIP;
}

ckkt_status ckkt_pcg_solve(ckkt_handle* h, const double* w_val, const double* g_val, const double* h_val,
                           const double* sigma_x, const double* sigma_s, double gamma, const float* params,
                           const double* rhs, double* sol, int32_t maxit, double tol, int32_t allow_refactor,
                           ckkt_solve_info* info, void* stream) {
    ckkt_solve_info local{};
    if (!info) info = &local;
    std::memset(info, 0, sizeof(*info));
    ckkt_status rc = learned_ready(h);
    if (rc) return info->status = rc;
    if (h->formulation != CKKT_LIFTED) return info->status = CKKT_ERR_ARG;
    const int n = h->plan.n;
    if (n > 0 && (!rhs || !sol)) return info->status = CKKT_ERR_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    (void)hipGetLastError();  // report only errors of this call's own launches
    rc = set_new_values(h, w_val, g_val, h_val, sigma_x, sigma_s, gamma, st);
    if (rc) return info->status = rc;
    const float* o = nullptr;
    if (params) {
        compute_features(h, h->feat, st);
        launch_mlp_forward(n, h->feat, params, h->mo, nullptr, st);
        o = h->mo;
    }
    ResidualOut r;
    double bmax = 0.0;
    rc = read_rhs_max(h, rhs, n, nullptr, 0, bmax, st);
    if (rc) return info->status = rc;
    if (!std::isfinite(bmax)) return info->status = CKKT_ERR_NONFINITE;
    bool ok = pcg_stale(h, rhs, sol, o, maxit, tol, r, info, st, rc);
    if (rc) return info->status = rc;
    info->omega = r.omega;
    info->rho = bmax > 0 ? r.resmax / bmax : r.resmax;
    if (ok) return info->status = CKKT_OK;
    if (!allow_refactor) return info->status = CKKT_ERR_NO_CONVERGENCE;
    // fallback (and judge): factorize the new system, which becomes the
    // stale reference of the following solves, and solve it directly
    int pcg_iters = info->pcg_iters;
    rc = ckkt_factorize(h, w_val, g_val, h_val, sigma_x, sigma_s, gamma, stream);
    if (rc) return info->status = rc;
    rc = ckkt_solve(h, rhs, sol, info, stream);
    info->pcg_iters += pcg_iters;
    info->fallback = 2;
    return info->status = rc;
}

// Per-pattern cache of autotuned launch shapes (signature of the plan).
static std::vector<std::pair<uint64_t, Tune>>& tune_cache() {
    static std::vector<std::pair<uint64_t, Tune>> c;
    return c;
}

static uint64_t plan_signature(const ckkt_handle* h) {
    const Plan& P = h->plan;
    uint64_t x = 1469598103934665603ull;
    auto mix = [&](uint64_t v) { x = (x ^ v) * 1099511628211ull; };
    mix(P.n); mix(P.m_eq); mix(P.m_ineq); mix(P.ns); mix(P.nlev); mix((uint64_t)P.nnz_l); mix(P.max_front);
    mix(h->precision); mix(h->formulation);
    for (int32_t v : P.sn_rowptr) mix((uint64_t)v);
    return x;
}

static void apply_tune(ckkt_handle* h, const Tune& t) {
    h->tune = t;
    build_levels(h);
    for (auto& g : h->graphs)
        if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
}

ckkt_status ckkt_autotune(ckkt_handle* h, const double* w_val, const double* g_val, const double* h_val,
                          const double* sigma_x, const double* sigma_s, double gamma, int32_t reps,
                          int32_t* chosen, double* best_ms, void* stream) {
    if (!h) return CKKT_ERR_ARG;
    if (!h->ws) return CKKT_ERR_STATE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    (void)hipGetLastError();  // report only errors of this call's own launches
    const uint64_t sig = plan_signature(h);
    for (auto& e : tune_cache())
        if (e.first == sig) {
            apply_tune(h, e.second);
            if (chosen) { chosen[0] = e.second.compact64; chosen[1] = e.second.compact_threads;
                          chosen[2] = e.second.tiny_threads; chosen[3] = e.second.sweep_cutoff; }
            if (best_ms) *best_ms = -1.0;
            return CKKT_OK;
        }
    if (reps < 1) reps = 3;
    std::vector<Tune> cands;
    for (int compact : {32, 48, 64})
        for (int cth : {128, 256})
            for (int tth : {64, 128})
                for (int cut : {32, 64, 128}) {
                    Tune t;
                    t.compact64 = compact;
                    t.compact32 = compact == 64 ? kCompactFront32 : compact;
                    t.compact_threads = cth;
                    t.tiny_threads = tth;
                    t.sweep_cutoff = cut;
                    cands.push_back(t);
                }
    double* b = h->vn[6];
    double* x = h->vn[7];
    launch_fill(h->plan.n, 1.0, b, st);
    hipEvent_t e0 = take_event(h), e1 = take_event(h);
    if (!e0 || !e1) return CKKT_ERR_HIP;
    double best = INFINITY;
    Tune bt = h->tune;
    for (const Tune& t : cands) {
        apply_tune(h, t);
        // warm (captures the graphs of this shape), then time
        ckkt_status rc = ckkt_factorize(h, w_val, g_val, h_val, sigma_x, sigma_s, gamma, stream);
        if (rc) return rc;
        apply_inverse(h, b, x, h->fp64_factored, st);
        HIP_TRY(hipEventRecord(e0, st));
        for (int r = 0; r < reps; ++r) {
            rc = ckkt_factorize(h, w_val, g_val, h_val, sigma_x, sigma_s, gamma, stream);
            if (rc) return rc;
            apply_inverse(h, b, x, h->fp64_factored, st);
        }
        HIP_TRY(hipEventRecord(e1, st));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        if (ms / reps < best) { best = ms / reps; bt = t; }
    }
    h->event_pool.push_back(e0);
    h->event_pool.push_back(e1);
    apply_tune(h, bt);
    tune_cache().push_back({sig, bt});
    if (chosen) { chosen[0] = bt.compact64; chosen[1] = bt.compact_threads; chosen[2] = bt.tiny_threads;
                  chosen[3] = bt.sweep_cutoff; }
    if (best_ms) *best_ms = best;
    // the timing runs left a valid factor of the given values
    return hipGetLastError() == hipSuccess ? CKKT_OK : CKKT_ERR_HIP;
}

ckkt_status ckkt_get_info(const ckkt_handle* h, ckkt_info* info) {
    if (!h || !info) return CKKT_ERR_ARG;
    const Plan& P = h->plan;
    std::memset(info, 0, sizeof(*info));
    info->n = P.n;
    info->m_eq = P.m_eq;
    info->m_ineq = P.m_ineq;
    info->nnz_k = P.kcolptr.empty() ? 0 : P.kcolptr.back();
    info->nnz_l = P.nnz_l;
    info->nnz_l_stored = P.nnz_l_stored;
    info->factor_flops = P.flops;
    info->assembly_products = (double)P.prod_r.size();
    info->n_supernodes = P.ns;
    info->n_levels = P.nlev;
    info->max_front = P.max_front;
    info->n_big_fronts = P.n_big;
    info->workspace_bytes = (int64_t)h->lay.total;
    info->analyze_seconds = P.analyze_seconds;
    info->order_seconds = P.order_seconds;
    info->symbolic_seconds = P.symbolic_seconds;
    info->n_instances = P.ninst;
    info->failed_column = h->failed_column;
    info->n_dense_rows = (int32_t)h->plan.dense_rows.size();
    return CKKT_OK;
}

const char* ckkt_status_string(ckkt_status s) {
    switch (s) {
        case CKKT_OK: return "ok";
        case CKKT_ERR_ARG: return "invalid argument";
        case CKKT_ERR_PATTERN: return "malformed sparsity pattern";
        case CKKT_ERR_NOT_SPD: return "matrix not positive definite (non-positive pivot)";
        case CKKT_ERR_NO_CONVERGENCE: return "refinement or CG did not converge";
        case CKKT_ERR_BREAKDOWN: return "CG breakdown";
        case CKKT_ERR_STATE: return "call out of order";
        case CKKT_ERR_HIP: return "HIP runtime error";
        case CKKT_ERR_WORKSPACE: return "workspace missing, too small or misaligned";
        case CKKT_ERR_NONFINITE: return "non-finite input";
        case CKKT_ERR_TIMEOUT: return "dependency wait in a triangular sweep timed out";
        case CKKT_ERR_HOST_MEMORY: return "host memory or a host thread could not be obtained";
        default: return "unknown status";
    }
}

void ckkt_destroy(ckkt_handle* h) {
    if (!h) return;
    for (auto& p : h->pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : h->event_pool) (void)hipEventDestroy(e);
    for (auto& g : h->graphs)
        if (g) (void)hipGraphExecDestroy(g);
    if (h->capture_stream) (void)hipStreamDestroy(h->capture_stream);
    destroy_side(h->side);
    if (h->host) (void)hipHostFree(h->host);
    delete h;
}

ckkt_status ckkt_set_timing(ckkt_handle* h, int32_t enable) {
    if (!h) return CKKT_ERR_ARG;
    h->timing = enable & 0xF;
    return CKKT_OK;
}

ckkt_status ckkt_get_timing(ckkt_handle* h, double ms[4], int64_t calls[4]) {
    if (!h || !ms || !calls) return CKKT_ERR_ARG;
    for (auto& p : h->pending) {
        HIP_TRY(hipEventSynchronize(p.b));
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, p.a, p.b));
        h->ms[p.phase] += t;
        h->calls[p.phase] += 1;
        h->event_pool.push_back(p.a);
        h->event_pool.push_back(p.b);
    }
    h->pending.clear();
    for (int i = 0; i < 4; ++i) {
        ms[i] = h->ms[i];
        calls[i] = h->calls[i];
        h->ms[i] = 0;
        h->calls[i] = 0;
    }
    return CKKT_OK;
}

}  // extern "C"
