"""Benchmark: condensed-KKT solves/s at a 1e-8 residual on one MI355X.

Headline (``value``): LiftedKKT FP64 on the large network-flow problem
(80,000 nodes, 104,000 edges: n = 528,000 variables, 160,000 equality and
416,000 inequality rows), the stand-in for the paper's 674k-variable OPF
instance (Sec. 6.1, tab:linsol:time, fig:timebreakdown).  One step = one new
system (diagonals drawn log-uniform in [1e-8, 1e8] afresh for every step)
through assembly, factorization and solve with FP64 refinement until the
componentwise relative backward error is <= 1e-10 (below the metric's 1e-8).

The other arms of the metric are timed in the same run and reported under
``forms``:

* ``netflow80k``: HyKKT FP64 (gamma = 1e7, CG tol 1e-10) on the same systems;
* ``seq80k``: the 60-system IPM-like sequence on the same pattern (diagonals
  moving from 1 to 1e+-8), FP64 versus FP32 factor + FP64 refinement, per
  system, with the systems on which FP32 + refinement wins;
* ``batch512``: 512 independent network-flow instances of uneven size
  (500..2000 nodes), FP64 and FP32 + FP64 refinement;
* ``pde48``: the 48^3 PDE-control problem's 80-system sequence, FP64
  refactorization of every system versus PCG around a stale factor with
  D = I and with the learned preconditioner (trained on systems 0..19);
* ``netflow10k``: the 66,000-variable network flow with the forms built
  around the path (inertia correction, dual regularization, the K2 Newton
  step, split dense rows).

Prints one JSON line.  Inputs are resident in HBM before a timed region
starts; ``--parts`` restricts the run to some of the parts (the headline is
always measured).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
METRIC = "condensed-KKT solves/s at 1e-8 rel. residual: FP64 vs FP32+IR/batched/PCG"
HEADLINE_NODES = 80_000
PARTS = ("netflow80k", "seq80k", "batch512", "pde48", "netflow10k", "analysis", "pde48factor")
DEFAULT_PARTS = PARTS[:6]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--parts", default=",".join(DEFAULT_PARTS),
                    help="comma list of " + ", ".join(PARTS) + " (the headline always runs); 'none' for none; "
                         "pde48factor (not in the default) only factorizes and solves the first --systems systems "
                         "of the PDE sequence in FP64 (a short run for counter collection)")
    ap.add_argument("--forms10k",
                    default="lifted_fp64,hykkt_fp64,lifted_fp64_inertia,hykkt_fp64_dualreg,lifted_fp64_k2,"
                            "hykkt_fp64_k2,lifted_fp64_dense4,lifted_fp32ir,hykkt_fp32ir",
                    help="forms of the netflow10k part")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the oracle CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--systems", type=int, default=None, help="sequence lengths (seq80k: 60, pde48: 80)")
    ap.add_argument("--instances", type=int, default=512, help="batch size")
    ap.add_argument("--side", type=int, default=48, help="grid side of the PDE workload")
    ap.add_argument("--pmc-calibration", action="store_true",
                    help="first run one plain device copy of 512 MiB (scale of the HBM byte counters)")
    return ap.parse_args()


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_factor_netflow80k.md")
KERNEL_SRC = os.path.join(ROOT, "paper_2405_14236_amd", "csrc", "kernels.hip")


def measured_traffic():
    """HBM bytes per factorization from the committed counter summary, or
    None when the factor kernels changed since the counters were taken."""
    import hashlib
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for ln in open(TRAFFIC_FILE):
        if ":" in ln and ln.strip().startswith(("source_sha256", "traffic_bytes_per_factorization")):
            k, v = ln.strip().split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if "source_sha256" not in vals or "traffic_bytes_per_factorization" not in vals:
        return None
    sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    return float(vals["traffic_bytes_per_factorization"]) if sha == vals["source_sha256"] else None


def algorithmic_counts(p, info):
    """Algorithmic bytes / flops per unit of work, from the analysis."""
    nnz_w, nnz_g, nnz_h = len(p.w_idx), len(p.g_idx), len(p.h_idx)
    n, m = p.n, p.m_eq + p.m_ineq
    nnz_k, nnz_l = info["nnz_k"], info["nnz_l"]
    return dict(assemble_bytes=8 * (nnz_w + nnz_g + nnz_h + n + m) + 8 * nnz_k,
                factor_bytes=8 * nnz_k + 8 * nnz_l, factor_flops=info["factor_flops"],
                sweep_bytes=2 * 8 * nnz_l + 6 * 8 * n, sweep_flops=4 * nnz_l,
                resid_bytes=8 * (nnz_w + 2 * (nnz_g + nnz_h)) + 5 * 8 * n)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


INERTIA_SHIFT = 1.0
GAMMA = 1e7


def time_form(form, p, sig, steps, warmup, torch, Solver, device_values):
    """One form: <lifted|hykkt>_<fp64|fp32ir>[_inertia|_dualreg|_k2|_dense4],
    one new system per step (sig[k] = (sigma_x, sigma_s) of step k).  The
    _inertia forms lower W's diagonal by INERTIA_SHIFT (negative curvature
    wherever K_jj is below it) and factorize with inertia correction,
    carrying delta_w_last from one system to the next as an interior-point
    method does.  hykkt_*_dualreg solves K1 with dual regularization
    delta_c = 1/gamma directly through the same K_gamma factor (no CG).  The
    _k2 forms take the full Newton step of the augmented system K2
    (ckkt_solve_augmented) for seeded r1..r4 instead of the condensed solve.
    The _dense4 forms add four inequality rows over half of the variables,
    kept out of K (opt.dense_row_min) and applied by the Woodbury step."""
    formulation, precision, *variant = form.split("_")
    prec = {"fp64": "fp64", "fp32ir": "fp32_ir"}[precision]
    inertia = variant == ["inertia"]
    dualreg = variant == ["dualreg"]
    k2 = variant == ["k2"]
    opts = {} if prec == "fp64" else {"tol": 1e-8}
    if variant == ["dense4"]:
        import paper_2405_14236_amd.workloads as wl
        p = wl.with_dense_rows(p, count=4, frac=0.5, seed=1)
        rng = np.random.default_rng(11)
        sig = [(a, np.concatenate([b, wl.log_uniform(rng, 4)])) for a, b in sig]
        opts["dense_row_min"] = 1000
    dev = "cuda"
    s = Solver(p, formulation, prec, **opts).bind(dev)
    info = s.info()
    w, g, h, _, _ = device_values(p, dev, formulation)
    if inertia:
        rows = np.repeat(np.arange(p.n), np.diff(p.w_ptr))
        wv = p.w_val.copy()
        wv[rows == p.w_idx] -= INERTIA_SHIFT
        w = torch.as_tensor(wv, device=dev)
    last, attempts, deltas = [0.0], [], []
    sx = [torch.as_tensor(a, device=dev) for a, _ in sig]
    ss = [torch.as_tensor(b if formulation == "lifted" else b[p.m_eq:], device=dev) for _, b in sig]

    def factorize(k):
        if dualreg:
            s.factorize_dual_reg(w, g, h, sx[k], ss[k], 1.0 / GAMMA)
            return
        if not inertia:
            s.factorize(w, g, h, sx[k], ss[k], GAMMA)
            return
        st, r = s.factorize_inertia(w, g, h, sx[k], ss[k], GAMMA, delta_w_last=last[0])
        last[0] = r["delta_w_last"]
        attempts.append(r["attempts"])
        deltas.append(r["delta_w"])
    rhs = np.concatenate([p.r1bar, p.r2bar]) if formulation == "hykkt" else p.b
    rhs = torch.as_tensor(rhs, device=dev)
    out = torch.empty_like(rhs)
    if k2:
        rng = np.random.default_rng(5)
        ms = p.m if formulation == "lifted" else p.m_ineq
        me = 0 if formulation == "lifted" else p.m_eq
        rk2 = [torch.as_tensor(rng.standard_normal(c), device=dev) for c in (p.n, ms, me, ms)]
        if formulation == "lifted":
            rk2[2] = None

    def solve(raise_on_error=True):
        if k2:
            return s.solve_augmented(*rk2, raise_on_error=raise_on_error)[-1]
        return s.solve(rhs, out, raise_on_error=raise_on_error)[1]
    names = ["assemble", "factor", "sweeps", "vector"]
    # all phases are timed over the warm-up to find the dominant one; the
    # timed region records events for that phase only (fewer event records)
    s.set_timing(True)
    s.get_timing()  # reset
    for k in range(warmup):
        factorize(k)
        solve(raise_on_error=False)
    torch.cuda.synchronize()
    wms, wcalls = s.get_timing()
    dom = int(np.argmax(wms)) if warmup > 0 and max(wms) > 0 else None
    attempts.clear()
    deltas.clear()
    s.set_timing(True, phases=None if dom is None else (dom,))
    s.get_timing()  # reset
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for k in range(warmup, warmup + steps):
        factorize(k)
        infos.append(solve(raise_on_error=False))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms, calls = s.get_timing()
    s.set_timing(False)
    ok = all(si["status"] == 0 and si["omega"] <= 1e-8 for si in infos)
    extra = {"delta_c": 1.0 / GAMMA} if dualreg else {}
    if variant == ["dense4"]:
        extra = {"dense_rows": info["n_dense_rows"], "nnz_k": info["nnz_k"]}
    if inertia:
        extra = dict(w_diag_shift=-INERTIA_SHIFT, attempts_mean=float(np.mean(attempts)),
                     delta_w=[float(f"{d:.4g}") for d in deltas])
    res = dict(solves_per_s=steps / (t1 - t0), ms_per_solve=1e3 * (t1 - t0) / steps, gate_ok=ok, **extra,
               omega_max=max(si["omega"] for si in infos), rho_max=max(si["rho"] for si in infos),
               refine_steps=float(np.mean([si["refine_steps"] for si in infos])),
               cg_iters=float(np.mean([si["cg_iters"] for si in infos])),
               fallbacks=int(sum(si["fallback"] != 0 for si in infos)),
               phase_ms=dict(zip(names, ms)), phase_calls=dict(zip(names, calls)),
               phase_ms_warmup=dict(zip(names, wms)), phase_calls_warmup=dict(zip(names, wcalls)),
               dominant_phase=names[dom] if dom is not None else max(names, key=lambda q: ms[names.index(q)]))
    log(f"[{form}] n={p.n}: {res['solves_per_s']:.1f} solves/s, omega_max {res['omega_max']:.2e}, "
        f"gate {'ok' if ok else 'FAILED'}")
    return res, info


def host_description():
    model = None
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return dict(cpu_model=model, nproc=avail, cpu_count=os.cpu_count())


def cpu_baseline(p, sig, budget_s):
    """The oracle (SuperLU factor + FP64 refinement to omega <= 1e-10,
    unassembled residual) on one host core, on as many of the timed systems
    as fit in the budget (at least one)."""
    from threadpoolctl import threadpool_limits
    from oracle import sparse as osp
    P = osp.Problem(p)
    done, worst = 0, 0.0
    with threadpool_limits(1):
        t0 = time.perf_counter()
        while done < len(sig):
            sx, ss = sig[done]
            x, hist = osp.solve_lifted(P, sx, ss, p.b, tol=1e-10)
            worst = max(worst, hist[-1])
            done += 1
            if time.perf_counter() - t0 > budget_s:
                break
        dt = time.perf_counter() - t0
    return dict(value=done / dt, unit="solves/s", cores=1, kind="oracle",
                sample=f"the first {done} of the timed LiftedKKT FP64 systems of the headline workload "
                       f"(n={p.n}; SuperLU + FP64 refinement to omega<=1e-10, BLAS limited to one thread), "
                       f"worst omega {worst:.1e}",
                **host_description())


def part_netflow80k(a, p, sig, torch, Solver, device_values):
    """HyKKT FP64 on the headline systems."""
    out = {}
    res, _ = time_form("hykkt_fp64", p, sig, a.steps, a.warmup, torch, Solver, device_values)
    out["hykkt_fp64"] = res
    return out


def part_seq80k(a, p, torch, workloads, Solver, device_values):
    """IPM-like sequence on the headline pattern: every system factorized and
    solved in FP64, then with the FP32 factor + FP64 refinement; per system
    wall time and the library's own backward error (the independent check of
    these systems against the oracle is a test)."""
    num = a.systems or 60
    seq = workloads.ipm_sigma_sequence(p, num, seed=a.seed)
    w, g, h, _, _ = device_values(p, "cuda", "lifted")
    sx = [torch.as_tensor(x, device="cuda") for x, _ in seq]
    ss = [torch.as_tensor(y, device="cuda") for _, y in seq]
    b = torch.as_tensor(p.b, device="cuda")
    out = {}
    for prec in ("fp64", "fp32_ir"):
        s = Solver(p, "lifted", prec, tol=1e-10 if prec == "fp64" else 1e-8).bind("cuda")
        x = torch.empty_like(b)
        s.factorize(w, g, h, sx[0], ss[0]); s.solve(b, x, raise_on_error=False)
        torch.cuda.synchronize()
        per, infos = [], []
        for k in range(num):
            t0 = time.perf_counter()
            s.factorize(w, g, h, sx[k], ss[k])
            _, si = s.solve(b, x, raise_on_error=False)
            torch.cuda.synchronize()
            per.append(time.perf_counter() - t0)
            infos.append(si)
        out[prec] = dict(solves_per_s=len(per) / sum(per), ms_per_solve=1e3 * float(np.mean(per)),
                         ms_per_system=[round(1e3 * t, 3) for t in per],
                         fallback=[si["fallback"] for si in infos],
                         refine_steps=[si["refine_steps"] for si in infos],
                         pcg_iters=[si["pcg_iters"] for si in infos],
                         omega_max=max(si["omega"] for si in infos),
                         gate_ok=all(si["status"] == 0 and si["omega"] <= 1e-8 for si in infos))
        log(f"[seq80k {prec}] {out[prec]['solves_per_s']:.1f} solves/s, gate {out[prec]['gate_ok']}")
        del s
    f64, f32 = out["fp64"]["ms_per_system"], out["fp32_ir"]["ms_per_system"]
    wins = [k for k in range(num) if f32[k] < f64[k]]
    out["fp32_ir_faster_on_systems"] = wins
    out["workload"] = (f"network-flow NLP {HEADLINE_NODES} nodes (n={p.n}), {num}-system IPM-like sigma "
                       "sequence (1 -> 1e+-8), LiftedKKT")
    return out


def part_batch512(a, torch, workloads, Solver):
    """512 independent network-flow instances of uneven size analysed as one
    block-diagonal system, autotuned; FP64 and FP32 + FP64 refinement."""
    probs = workloads.batch_network_flow(a.instances, seed=a.seed)
    rng = np.random.default_rng(a.seed + 5)
    cat = lambda xs: torch.as_tensor(np.concatenate(xs), device="cuda")
    w = cat([q.w_val for q in probs]); g = cat([q.g_val for q in probs]); h = cat([q.h_val for q in probs])
    b = cat([q.b for q in probs])
    nsys = a.steps + a.warmup
    sig = []
    for _ in range(nsys):
        sxs = [workloads.log_uniform(rng, q.n) for q in probs]
        sss = [workloads.log_uniform(rng, q.m) for q in probs]
        sig.append((cat(sxs), cat([x[:q.m_eq] for x, q in zip(sss, probs)] + [x[q.m_eq:] for x, q in zip(sss, probs)])))
    out = {}
    blob = None
    for prec in ("fp64", "fp32_ir"):
        t0 = time.perf_counter()
        tol = 1e-8 if prec == "fp32_ir" else 1e-10
        if blob is None:
            s = Solver(None, "lifted", prec, batch=probs, tol=tol)
            blob = s.save_plan()
            t_an = time.perf_counter() - t0
        else:
            s = Solver.from_plan(blob, precision=prec, tol=tol)  # same analysis, reloaded
        s.bind("cuda")
        log(f"[batch {prec}] analysed in {t_an:.2f} s")
        chosen, best = s.autotune(w, g, h, sig[0][0], sig[0][1])
        x = torch.empty_like(b)
        # one call per batch (ckkt_batch_factorize_solve): the values of step
        # k are copied into fixed buffers first, so the captured sequence is
        # replayed (the copies are inside the timed region)
        refine = 1 if prec == "fp64" else 3
        sxb, ssb = torch.empty_like(sig[0][0]), torch.empty_like(sig[0][1])
        for k in range(a.warmup):
            sxb.copy_(sig[k][0]); ssb.copy_(sig[k][1])
            s.factorize_solve(w, g, h, sxb, ssb, b, x, refine=refine, raise_on_error=False)
        torch.cuda.synchronize()
        infos = []
        t0 = time.perf_counter()
        for k in range(a.warmup, nsys):
            sxb.copy_(sig[k][0]); ssb.copy_(sig[k][1])
            _, si, _ = s.factorize_solve(w, g, h, sxb, ssb, b, x, refine=refine, raise_on_error=False)
            infos.append(si)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        # the same systems through ckkt_factorize + ckkt_solve (host-driven refinement)
        infos2 = []
        t1 = time.perf_counter()
        for k in range(a.warmup, nsys):
            s.factorize(w, g, h, *sig[k])
            _, si = s.solve(b, x, raise_on_error=False)
            infos2.append(si)
        torch.cuda.synchronize()
        dt2 = time.perf_counter() - t1
        out[prec] = dict(solves_per_s=a.instances * a.steps / dt, ms_per_batch=1e3 * dt / a.steps,
                         device_refine_steps=refine, analyze_s=t_an, autotune=chosen, autotune_best_ms=best,
                         gate_ok=all(si["status"] == 0 and si["omega"] <= 1e-8 for si in infos),
                         omega_max=max(si["omega"] for si in infos),
                         host_handovers=int(sum((si["fallback"] & 4) != 0 for si in infos)),
                         fallbacks=int(sum((si["fallback"] & 3) != 0 for si in infos)),
                         two_calls=dict(solves_per_s=a.instances * a.steps / dt2, ms_per_batch=1e3 * dt2 / a.steps,
                                        gate_ok=all(si["status"] == 0 and si["omega"] <= 1e-8 for si in infos2),
                                        fallbacks=int(sum(si["fallback"] != 0 for si in infos2))))
        log(f"[batch {prec}] {out[prec]['solves_per_s']:.0f} solves/s one call "
            f"({out[prec]['two_calls']['solves_per_s']:.0f} with factorize + solve), gate {out[prec]['gate_ok']}")
        del s
    out["workload"] = (f"{a.instances} network-flow instances, nodes uniform in [500, 2000], LiftedKKT, one "
                       "block-diagonal analysis, autotuned launch shapes, one captured factorize-and-solve call "
                       "per batch (ckkt_batch_factorize_solve)")
    return out


def part_analysis(a, p, torch, workloads, Solver):
    """Analysis time with the symbolic factorization on the host
    (ckkt_analyze) and on the GPU (ckkt_analyze_device), both after the same
    host ordering: the 528,000-variable network flow, the 48^3 PDE-control
    pattern and the 512-instance batch.  The two plans are equal byte for
    byte (GPU tests); order_s is the host part up to the ordering, symbolic_s
    the part the GPU takes over."""
    Solver(workloads.tiny_grid(0), "lifted", analysis="device")  # first device use outside the timing
    cases = [("netflow80k", lambda mode: Solver(p, "lifted", analysis=mode))]
    pde = workloads.pde_control(a.side)
    cases.append((f"pde{a.side}", lambda mode: Solver(pde, "lifted", analysis=mode)))
    probs = workloads.batch_network_flow(a.instances, seed=a.seed)
    cases.append((f"batch{a.instances}", lambda mode: Solver(None, "lifted", batch=probs, analysis=mode)))
    out = {}
    for name, make in cases:
        row = {}
        for mode in ("host", "device"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s = make(mode)
            wall = time.perf_counter() - t0
            inf = s.info()
            row[mode] = {"wall_s": wall, "analyze_s": inf["analyze_seconds"], "order_s": inf["order_seconds"],
                         "symbolic_s": inf["symbolic_seconds"]}
            del s
        row["symbolic_speedup"] = row["host"]["symbolic_s"] / max(row["device"]["symbolic_s"], 1e-9)
        row["analysis_speedup"] = row["host"]["analyze_s"] / max(row["device"]["analyze_s"], 1e-9)
        out[name] = row
        print(f"[analysis] {name}: {row}", file=sys.stderr, flush=True)
    return out


def part_pde48factor(a, torch, workloads, Solver, device_values):
    """FP64 factorization and solve of the first systems of the PDE
    sequence only (matrix-core counters of the 48^3 factorization)."""
    p = workloads.pde_control(a.side, seed=a.seed)
    num = a.systems or 3
    seq = workloads.ipm_sigma_sequence(p, 80, seed=a.seed)
    rhs = torch.as_tensor(np.random.default_rng(a.seed + 11).standard_normal(p.n), device="cuda")
    w, g, h, _, _ = device_values(p, "cuda", "lifted")
    s = Solver(p, "lifted", "fp64").bind("cuda")
    x = torch.empty_like(rhs)
    per = []
    for k in range(num):
        sx, ss = (torch.as_tensor(v, device="cuda") for v in seq[k])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.factorize(w, g, h, sx, ss)
        _, si = s.solve(rhs, x)
        torch.cuda.synchronize()
        per.append(time.perf_counter() - t0)
    inf = s.info()
    out = dict(ms_per_system=[round(1e3 * t, 2) for t in per], factor_flops=inf["factor_flops"], nnz_l=inf["nnz_l"])
    log(f"[pde{a.side} factor only] {num} systems, {np.mean(per) * 1e3:.1f} ms each")
    return out


def part_pde48(a, torch, workloads, Solver, device_values):
    """PDE-constrained problem, IPM-like sequence: FP64 refactorization of
    every system versus PCG around a stale factor, with D = I and with the
    learned preconditioner (trained on systems 0..19 with the stale factor
    of system 10, then used around the factor of system 19, refreshed on
    fallback)."""
    from paper_2405_14236_amd.solver import init_mlp_params
    p = workloads.pde_control(a.side, seed=a.seed)
    num = a.systems or 80
    seq = workloads.ipm_sigma_sequence(p, num, seed=a.seed)
    rng = np.random.default_rng(a.seed + 11)
    rhs = [torch.as_tensor(rng.standard_normal(p.n), device="cuda") for _ in range(num)]
    w, g, h, _, _ = device_values(p, "cuda", "lifted")
    T = lambda v: torch.as_tensor(v, device="cuda")
    sx = [T(x) for x, _ in seq]; ss = [T(y) for _, y in seq]
    out = {}
    s64 = Solver(p, "lifted", "fp64").bind("cuda")
    x = torch.empty_like(rhs[0])
    s64.factorize(w, g, h, sx[0], ss[0]); s64.solve(rhs[0], x); torch.cuda.synchronize()
    per64 = []
    targets = []
    for k in range(num):
        t0 = time.perf_counter()
        s64.factorize(w, g, h, sx[k], ss[k])
        _, si = s64.solve(rhs[k], x)
        torch.cuda.synchronize()
        per64.append(time.perf_counter() - t0)
        if k < 20:
            targets.append(x.clone())
    out["fp64_refactor"] = dict(solves_per_s=num / sum(per64), ms_per_system=[round(1e3 * t, 2) for t in per64])
    log(f"[pde{a.side} fp64 refactor] {out['fp64_refactor']['solves_per_s']:.2f} solves/s")
    del s64
    # FP32 factor (matrix cores) + FP64 refinement of every system, with its
    # fallbacks (PCG around the FP32 factor, FP64 refactorization)
    s32 = Solver(p, "lifted", "fp32_ir", tol=1e-8).bind("cuda")
    s32.factorize(w, g, h, sx[0], ss[0]); s32.solve(rhs[0], x, raise_on_error=False); torch.cuda.synchronize()
    per32, inf32 = [], []
    for k in range(num):
        t0 = time.perf_counter()
        s32.factorize(w, g, h, sx[k], ss[k])
        _, si = s32.solve(rhs[k], x, raise_on_error=False)
        torch.cuda.synchronize()
        per32.append(time.perf_counter() - t0)
        inf32.append(si)
    out["fp32_ir_refactor"] = dict(solves_per_s=num / sum(per32), ms_per_system=[round(1e3 * t, 2) for t in per32],
                                   fallback=[si["fallback"] for si in inf32],
                                   refine_steps=[si["refine_steps"] for si in inf32],
                                   omega_max=max(si["omega"] for si in inf32),
                                   gate_ok=all(si["status"] == 0 and si["omega"] <= 1e-8 for si in inf32),
                                   faster_than_fp64_on_systems=[k for k in range(num) if per32[k] < per64[k]])
    log(f"[pde{a.side} fp32+IR refactor] {out['fp32_ir_refactor']['solves_per_s']:.2f} solves/s, faster than FP64 "
        f"on {len(out['fp32_ir_refactor']['faster_than_fp64_on_systems'])} of {num} systems")
    del s32
    s = Solver(p, "lifted", "fp32_ir", learned=1).bind("cuda")
    s.factorize(w, g, h, sx[10], ss[10])
    prm = init_mlp_params(a.seed, device="cuda")
    m = torch.zeros_like(prm); v = torch.zeros_like(prm)
    t0 = time.perf_counter()
    step, losses = 0, []
    for epoch in range(20):
        for k in range(20):
            if k == 10:
                continue
            step += 1
            losses.append(s.mlp_train_step((w, g, h, sx[k], ss[k]), 0.0, rhs[k], targets[k], prm, m, v, step, 3e-3))
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    for name, params in (("pcg_learned", prm), ("pcg_identity", None)):
        s.factorize(w, g, h, sx[19], ss[19])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        iters, fb, oms = [], 0, []
        for k in range(20, num):
            _, si = s.pcg_solve((w, g, h, sx[k], ss[k]), 0.0, params, rhs[k], maxit=50, tol=1e-8,
                                allow_refactor=True, raise_on_error=False)
            iters.append(si["pcg_iters"]); fb += si["fallback"] != 0; oms.append(si["omega"])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[name] = dict(solves_per_s=(num - 20) / dt, pcg_iters=iters, refactorizations=fb,
                         omega_max=max(oms), gate_ok=max(oms) <= 1e-8)
        log(f"[pde{a.side} {name}] {out[name]['solves_per_s']:.2f} solves/s, {np.mean(iters):.1f} PCG iterations")
    out["training"] = dict(seconds=train_s, steps=step, loss_first=losses[0], loss_last=losses[-1])
    inf = s.info()
    out["workload"] = (f"3-D Poisson control {a.side}^3 states + stride-2 controls (n={p.n}, nnz(L)={inf['nnz_l']}, "
                       f"{inf['factor_flops']:.3g} flops per factor), {num}-system IPM-like sigma sequence, "
                       "LiftedKKT; PCG around a stale FP32 factor")
    return out


def part_netflow10k(a, torch, workloads, Solver, device_values):
    p = workloads.network_flow(10_000, seed=a.seed)
    rng = np.random.default_rng(a.seed + 1)
    nsys = a.steps + a.warmup
    sig = [(workloads.log_uniform(rng, p.n), workloads.log_uniform(rng, p.m)) for _ in range(nsys)]
    out = {}
    for f in a.forms10k.split(","):
        out[f], _ = time_form(f, p, sig, a.steps, a.warmup, torch, Solver, device_values)
    out["workload"] = (f"network-flow NLP 10000 nodes ({p.n} vars, {p.m_eq} eq, {p.m_ineq} ineq), new "
                       "log-uniform sigma in [1e-8,1e8] per solve")
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only (one process, one device); "
                                   "--gpus must be 1", "n_gpus": a.gpus}))
        sys.exit(2)
    import torch
    from paper_2405_14236_amd import workloads
    from paper_2405_14236_amd.solver import Solver, device_values
    parts = [] if a.parts == "none" else [q for q in a.parts.split(",") if q]
    for q in parts:
        if q not in PARTS:
            raise SystemExit(f"unknown part {q}")

    if a.pmc_calibration:
        src = torch.ones(64 << 20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"pmc calibration: one device copy of {src.numel() * 8} bytes read and written")
        del src, dst

    p = workloads.network_flow(HEADLINE_NODES, seed=a.seed)
    rng = np.random.default_rng(a.seed + 1)
    nsys = a.steps + a.warmup
    sig = [(workloads.log_uniform(rng, p.n), workloads.log_uniform(rng, p.m)) for _ in range(nsys)]
    head, info = time_form("lifted_fp64", p, sig, a.steps, a.warmup, torch, Solver, device_values)
    cnt = algorithmic_counts(p, info)

    # roofline of the dominant phase of the headline (HIP events recorded by
    # the library on its stream over the timed region)
    ph_ms, ph_calls = head["phase_ms"], head["phase_calls"]
    per_call = {k: ph_ms[k] / max(ph_calls[k], 1) for k in ph_ms}
    dom = head["dominant_phase"]
    unit_bytes, flops = {"factor": (cnt["factor_bytes"], cnt["factor_flops"]),
                         "sweeps": (cnt["sweep_bytes"], cnt["sweep_flops"]),
                         "assemble": (cnt["assemble_bytes"], None),
                         "vector": (cnt["resid_bytes"], None)}[dom]
    achieved = unit_bytes / (per_call[dom] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS,
                "traffic": measured_traffic() if dom == "factor" else None,
                "kernel": dom, "unit_bytes": unit_bytes, "avg_ms": per_call[dom]}
    if flops:
        roofline["fp64_tflops"] = flops / (per_call[dom] * 1e-3) / 1e12
        roofline["fp64_frac"] = roofline["fp64_tflops"] / FP64_PEAK_TFLOPS

    forms = {"netflow80k": {"lifted_fp64": head}}
    if "netflow80k" in parts:
        forms["netflow80k"].update(part_netflow80k(a, p, sig, torch, Solver, device_values))
    if "seq80k" in parts:
        forms["seq80k"] = part_seq80k(a, p, torch, workloads, Solver, device_values)
    if "batch512" in parts:
        forms["batch512"] = part_batch512(a, torch, workloads, Solver)
    if "pde48factor" in parts:
        forms["pde48factor"] = part_pde48factor(a, torch, workloads, Solver, device_values)
    if "pde48" in parts:
        forms["pde48"] = part_pde48(a, torch, workloads, Solver, device_values)
    if "netflow10k" in parts:
        forms["netflow10k"] = part_netflow10k(a, torch, workloads, Solver, device_values)
    if "analysis" in parts:
        forms["analysis"] = part_analysis(a, p, torch, workloads, Solver)

    cpu = None if a.no_cpu_baseline else cpu_baseline(p, sig[a.warmup:], a.cpu_seconds)
    line = {
        "metric": METRIC,
        "value": head["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": head["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"network-flow NLP, {HEADLINE_NODES} nodes / {p.n} vars / {p.m_eq} eq / "
                               f"{p.m_ineq} ineq, LiftedKKT FP64, new log-uniform sigma in [1e-8,1e8] per solve",
                   "n": p.n, "nnz_k": info["nnz_k"], "nnz_l": info["nnz_l"], "supernodes": info["n_supernodes"],
                   "levels": info["n_levels"], "max_front": info["max_front"],
                   "analyze_s": info["analyze_seconds"], "gate_omega": 1e-10},
        "gate_ok": head["gate_ok"],
        "roofline": roofline,
        "cpu_baseline": cpu,
        "forms": forms,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
