"""Python binding of the condensed-KKT library: argument marshalling only.

Every step of the path (assembly, factorization, sweeps, refinement, CG)
runs in the HIP library; this module passes pointers of torch tensors and
the caller's current HIP stream through the C-ABI declared in
include/ckkt.h.  Torch provides device memory (the workspace and the
value/right-hand-side/solution tensors) and streams.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np

from . import _lib as L


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(L.P_i32)


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(L.P_f64)


def _pattern(prob, formulation):
    keep = []
    fields = {}
    for key in ("w_ptr", "w_idx", "g_ptr", "g_idx", "h_ptr", "h_idx"):
        arr, ptr = _i32(getattr(prob, key))
        keep.append(arr)
        fields[key] = ptr
    pat = L.Pattern(n=prob.n, m_eq=prob.m_eq, m_ineq=prob.m_ineq, formulation=formulation, **fields)
    return pat, keep


def options(precision="fp64", ordering="amd", tol=1e-10, ir_maxit=10, cg_tol=1e-10, cg_maxit=0, relax=1,
            lds_front_max=0, learned=0, dense_row_min=0):
    lib = L.load()
    o = L.Options()
    lib.ckkt_default_options(ctypes.byref(o))
    o.precision = {"fp64": L.FP64, "fp32_ir": L.FP32_IR}[precision]
    o.ordering = {"amd": L.ORDER_AMD, "natural": L.ORDER_NATURAL}[ordering]
    o.tol, o.ir_maxit, o.cg_tol, o.cg_maxit, o.relax = tol, ir_maxit, cg_tol, cg_maxit, relax
    o.lds_front_max = lds_front_max
    o.learned = int(learned)
    o.dense_row_min = int(dense_row_min)
    return o


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Solver:
    """One analysed pattern (single system, or a block-diagonal batch).

    ``formulation``: "lifted" (K_tau d_x = b) or "hykkt" (K1 through K_gamma + CG).
    ``precision``: "fp64" or "fp32_ir" (FP32 factor, FP64 refinement).
    ``analysis``: "host" (ckkt_analyze) or "device" (ckkt_analyze_device: the
    symbolic factorization runs on the current torch stream).
    """

    def __init__(self, prob, formulation="lifted", precision="fp64", *, batch: Optional[Sequence] = None,
                 analysis="host", **opts):
        self.lib = L.load()
        if analysis not in ("host", "device"):
            raise ValueError("analysis must be 'host' or 'device'")
        self.formulation = {"lifted": L.LIFTED, "hykkt": L.HYKKT}[formulation]
        self.opts = options(precision=precision, **opts)
        h = ctypes.c_void_p()
        ws = ctypes.c_size_t()
        if batch is None:
            pat, self._keep = _pattern(prob, self.formulation)
            if analysis == "device":
                L.check(self.lib.ckkt_analyze_device(ctypes.byref(pat), ctypes.byref(self.opts), _stream(),
                                                     ctypes.byref(h), ctypes.byref(ws)), "ckkt_analyze_device")
            else:
                L.check(self.lib.ckkt_analyze(ctypes.byref(pat), ctypes.byref(self.opts), ctypes.byref(h),
                                              ctypes.byref(ws)), "ckkt_analyze")
            self.n, self.m_eq, self.m_ineq = prob.n, prob.m_eq, prob.m_ineq
        else:
            pats, keep = [], []
            for p in batch:
                pat, k = _pattern(p, self.formulation)
                pats.append(pat)
                keep += k
            arr = (L.Pattern * len(pats))(*pats)
            if analysis == "device":
                L.check(self.lib.ckkt_batch_analyze_device(len(pats), arr, ctypes.byref(self.opts), _stream(),
                                                           ctypes.byref(h), ctypes.byref(ws)),
                        "ckkt_batch_analyze_device")
            else:
                L.check(self.lib.ckkt_batch_analyze(len(pats), arr, ctypes.byref(self.opts), ctypes.byref(h),
                                                    ctypes.byref(ws)), "ckkt_batch_analyze")
            self._keep = keep
            self.n = sum(p.n for p in batch)
            self.m_eq = sum(p.m_eq for p in batch)
            self.m_ineq = sum(p.m_ineq for p in batch)
        self.h = h
        self.workspace_bytes = ws.value
        self.workspace = None
        self._vals = None

    # ------------------------------------------------------ plan checkpoint
    def save_plan(self) -> bytes:
        """The serialized analysis plan (ckkt_plan_save)."""
        size = ctypes.c_size_t()
        L.check(self.lib.ckkt_plan_size(self.h, ctypes.byref(size)), "ckkt_plan_size")
        buf = ctypes.create_string_buffer(size.value)
        L.check(self.lib.ckkt_plan_save(self.h, buf, size.value), "ckkt_plan_save")
        return buf.raw

    @classmethod
    def from_plan(cls, blob: bytes, precision="fp64", **opts):
        """A solver built from a saved plan, without analysing the pattern
        again (ckkt_plan_load); the formulation and the options that shaped
        the plan come from it."""
        import struct
        self = cls.__new__(cls)
        self.lib = L.load()
        self.opts = options(precision=precision, **opts)
        # header: 8-byte magic, int32 version, int32 formulation, ...
        self.formulation = struct.unpack_from("<i", blob, 12)[0] if len(blob) >= 16 else -1
        h = ctypes.c_void_p()
        ws = ctypes.c_size_t()
        buf = ctypes.create_string_buffer(bytes(blob), len(blob))
        L.check(self.lib.ckkt_plan_load(buf, len(blob), ctypes.byref(self.opts), ctypes.byref(h), ctypes.byref(ws)),
                "ckkt_plan_load")
        self.h = h
        self.workspace_bytes = ws.value
        self.workspace = None
        self._vals = None
        self._keep = []
        inf = self.info()
        self.n, self.m_eq, self.m_ineq = inf["n"], inf["m_eq"], inf["m_ineq"]
        return self

    # ---------------------------------------------------------------- info
    def info(self):
        inf = L.Info()
        L.check(self.lib.ckkt_get_info(self.h, ctypes.byref(inf)), "ckkt_get_info")
        return inf.as_dict()

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.lib.ckkt_destroy(h)
            self.h = None

    # ------------------------------------------------------------- device
    def bind(self, device="cuda"):
        import torch
        self.workspace = torch.empty(max(self.workspace_bytes, 256), dtype=torch.uint8, device=device)
        L.check(self.lib.ckkt_bind_workspace(self.h, _ptr(self.workspace), self.workspace.numel(), _stream()),
                "ckkt_bind_workspace")
        return self

    def factorize(self, w_val, g_val, h_val, sigma_x, sigma_s, gamma=0.0):
        """Device float64 tensors; kept referenced until the next factorize."""
        if self.workspace is None:
            self.bind()
        self._vals = (w_val, g_val, h_val, sigma_x, sigma_s)
        L.check(self.lib.ckkt_factorize(self.h, _ptr(w_val), _ptr(g_val), _ptr(h_val), _ptr(sigma_x),
                                        _ptr(sigma_s), float(gamma), _stream()), "ckkt_factorize")

    def factor_status(self):
        return self.lib.ckkt_factor_status(self.h, _stream())

    def factorize_dual_reg(self, w_val, g_val, h_val, sigma_x, sigma_s, delta_c):
        """HyKKT with dual regularization delta_c > 0 (ckkt_factorize_dual_reg):
        the following solves are direct, without CG."""
        if self.workspace is None:
            self.bind()
        self._vals = (w_val, g_val, h_val, sigma_x, sigma_s)
        L.check(self.lib.ckkt_factorize_dual_reg(self.h, _ptr(w_val), _ptr(g_val), _ptr(h_val), _ptr(sigma_x),
                                                 _ptr(sigma_s), float(delta_c), _stream()),
                "ckkt_factorize_dual_reg")

    def factorize_inertia(self, w_val, g_val, h_val, sigma_x, sigma_s, gamma=0.0, delta_w_last=0.0,
                          raise_on_error=True, **params):
        """Factorization with inertia correction (ckkt_factorize_inertia).

        sigma_x / sigma_s are the unregularized diagonals; ``params`` override
        the rule's constants (delta_w_min, delta_w_0, delta_w_max, kappa_minus,
        kappa_plus, kappa_plus_bar).  Returns (status, dict with delta_w,
        attempts and delta_w_last)."""
        if self.workspace is None:
            self.bind()
        self._vals = (w_val, g_val, h_val, sigma_x, sigma_s)
        ic = inertia_params(delta_w_last, **params)
        st = self.lib.ckkt_factorize_inertia(self.h, _ptr(w_val), _ptr(g_val), _ptr(h_val), _ptr(sigma_x),
                                             _ptr(sigma_s), float(gamma), ctypes.byref(ic), _stream())
        if raise_on_error:
            L.check(st, "ckkt_factorize_inertia")
        return st, inertia_result(ic)

    def solve(self, rhs, out=None, raise_on_error=True):
        import torch
        if out is None:
            out = torch.empty_like(rhs)
        si = L.SolveInfo()
        st = self.lib.ckkt_solve(self.h, _ptr(rhs), _ptr(out), ctypes.byref(si), _stream())
        if raise_on_error:
            L.check(st, "ckkt_solve")
        return out, si.as_dict()

    def factorize_solve(self, w, g, h, sigma_x, sigma_s, rhs, out=None, refine=1, raise_on_error=True):
        """ckkt_batch_factorize_solve: factorization and solve (LiftedKKT) in one
        captured call with one host synchronization; returns (sol, info,
        per-instance omega as a numpy array)."""
        import torch
        if out is None:
            out = torch.empty_like(rhs)
        ninst = self._ninst()
        om = np.zeros(max(ninst, 1))
        si = L.SolveInfo()
        st = self.lib.ckkt_batch_factorize_solve(self.h, _ptr(w), _ptr(g), _ptr(h), _ptr(sigma_x), _ptr(sigma_s),
                                                 _ptr(rhs), _ptr(out), int(refine), om.ctypes.data_as(L.P_f64),
                                                 ctypes.byref(si), _stream())
        if raise_on_error:
            L.check(st, "ckkt_batch_factorize_solve")
        return out, si.as_dict(), om[:ninst]

    def _ninst(self):
        return self.info()["n_instances"]

    def solve_augmented(self, r1, r2, r3, r4, raise_on_error=True):
        """Newton step of K2 (ckkt_solve_augmented): returns (dx, ds, dy, dz, info).
        r3 / dy are used by HyKKT only (pass None for LiftedKKT)."""
        import torch
        dx, ds, dz = torch.empty_like(r1), torch.empty_like(r2), torch.empty_like(r4)
        dy = torch.empty_like(r3) if r3 is not None else None
        si = L.SolveInfo()
        st = self.lib.ckkt_solve_augmented(self.h, _ptr(r1), _ptr(r2), _ptr(r3), _ptr(r4), _ptr(dx), _ptr(ds),
                                           _ptr(dy), _ptr(dz), ctypes.byref(si), _stream())
        if raise_on_error:
            L.check(st, "ckkt_solve_augmented")
        return dx, ds, dy, dz, si.as_dict()

    def apply_inverse(self, rhs, out=None):
        import torch
        if out is None:
            out = torch.empty_like(rhs)
        L.check(self.lib.ckkt_apply_inverse(self.h, _ptr(rhs), _ptr(out), _stream()), "ckkt_apply_inverse")
        return out

    def export_k(self):
        import torch
        nnz = self.info()["nnz_k"]
        rows = np.empty(nnz, np.int32)
        cols = np.empty(nnz, np.int32)
        vals = torch.empty(nnz, dtype=torch.float64, device=self.workspace.device)
        L.check(self.lib.ckkt_export_k(self.h, rows.ctypes.data_as(L.P_i32), cols.ctypes.data_as(L.P_i32),
                                       _ptr(vals), _stream()), "ckkt_export_k")
        return rows, cols, vals

    def set_timing(self, on=True, phases=None):
        """Per-phase HIP-event timing: all phases, or only the given phase
        numbers (0 assemble, 1 factor, 2 sweeps, 3 vector work)."""
        mask = 0 if not on else (-1 if phases is None else sum(1 << int(q) for q in phases))
        L.check(self.lib.ckkt_set_timing(self.h, mask))

    def get_timing(self):
        ms = (ctypes.c_double * 4)()
        calls = (ctypes.c_int64 * 4)()
        L.check(self.lib.ckkt_get_timing(self.h, ms, calls))
        return list(ms), list(calls)

    def autotune(self, w_val, g_val, h_val, sigma_x, sigma_s, gamma=0.0, reps=3):
        """Times candidate launch shapes on this pattern and keeps the fastest."""
        if self.workspace is None:
            self.bind()
        chosen = (ctypes.c_int32 * 4)()
        best = ctypes.c_double()
        L.check(self.lib.ckkt_autotune(self.h, _ptr(w_val), _ptr(g_val), _ptr(h_val), _ptr(sigma_x), _ptr(sigma_s),
                                       float(gamma), int(reps), chosen, ctypes.byref(best), _stream()),
                "ckkt_autotune")
        keys = ("compact_front", "compact_threads", "tiny_threads", "sweep_cutoff")
        return dict(zip(keys, list(chosen))), best.value

    # ------------------------------------------------------- learned PCG
    def features(self, w_val, g_val, h_val, sigma_x, sigma_s, gamma=0.0):
        import torch
        out = torch.empty((self.n, L.MLP_F), dtype=torch.float32, device=self.workspace.device)
        L.check(self.lib.ckkt_features(self.h, _ptr(w_val), _ptr(g_val), _ptr(h_val), _ptr(sigma_x),
                                       _ptr(sigma_s), float(gamma), _ptr(out), _stream()), "ckkt_features")
        return out

    def mlp_train_step(self, vals, gamma, rhs, target, params, m, v, step, lr):
        loss = ctypes.c_double()
        w, g, hv, sx, ss = vals
        L.check(self.lib.ckkt_mlp_train_step(self.h, _ptr(w), _ptr(g), _ptr(hv), _ptr(sx), _ptr(ss), float(gamma),
                                             _ptr(rhs), _ptr(target), _ptr(params), _ptr(m), _ptr(v), int(step),
                                             float(lr), ctypes.byref(loss), _stream()), "ckkt_mlp_train_step")
        return loss.value

    def pcg_solve(self, vals, gamma, params, rhs, maxit=50, tol=1e-8, allow_refactor=True, out=None,
                  raise_on_error=True):
        import torch
        if out is None:
            out = torch.empty_like(rhs)
        w, g, hv, sx, ss = vals
        si = L.SolveInfo()
        st = self.lib.ckkt_pcg_solve(self.h, _ptr(w), _ptr(g), _ptr(hv), _ptr(sx), _ptr(ss), float(gamma),
                                     _ptr(params), _ptr(rhs), _ptr(out), int(maxit), float(tol), int(allow_refactor),
                                     ctypes.byref(si), _stream())
        if raise_on_error:
            L.check(st, "ckkt_pcg_solve")
        return out, si.as_dict()

    # ---------------------------------------------------------------- host
    def host_factor_solve(self, w_val, g_val, h_val, sigma_x, sigma_s, gamma, rhs):
        """Sequential host run of the numeric phase over the same plan (no GPU)."""
        keep = [_f64(a) for a in (w_val, g_val, h_val, sigma_x, sigma_s, rhs)]
        out = np.empty(len(rhs), np.float64)
        fc = ctypes.c_int32(-1)
        st = self.lib.ckkt_host_factor_solve(self.h, keep[0][1], keep[1][1], keep[2][1], keep[3][1], keep[4][1],
                                             float(gamma), keep[5][1], out.ctypes.data_as(L.P_f64),
                                             ctypes.byref(fc))
        return out, st, fc.value

    def host_factor_solve_inertia(self, w_val, g_val, h_val, sigma_x, sigma_s, gamma, rhs, delta_w_last=0.0,
                                  **params):
        """Host run of the inertia-corrected factorization, then one solve."""
        keep = [_f64(a) for a in (w_val, g_val, h_val, sigma_x, sigma_s, rhs)]
        out = np.empty(len(rhs), np.float64)
        ic = inertia_params(delta_w_last, **params)
        st = self.lib.ckkt_host_factor_solve_inertia(self.h, keep[0][1], keep[1][1], keep[2][1], keep[3][1],
                                                     keep[4][1], float(gamma), ctypes.byref(ic), keep[5][1],
                                                     out.ctypes.data_as(L.P_f64))
        return out, st, inertia_result(ic)


def recover_bound_dual(s, v, mu, ds):
    """d_v = -S^-1 (V d_s - mu e) - v on the device (ckkt_recover_bound_dual)."""
    import torch
    dv = torch.empty_like(ds)
    L.check(L.load().ckkt_recover_bound_dual(ds.numel(), _ptr(s), _ptr(v), float(mu), _ptr(ds), _ptr(dv),
                                             _stream()), "ckkt_recover_bound_dual")
    return dv


def inertia_params(delta_w_last=0.0, **params):
    ic = L.Inertia()
    L.load().ckkt_default_inertia(ctypes.byref(ic))
    ic.delta_w_last = float(delta_w_last)
    for k, v in params.items():
        if k not in ("delta_w_min", "delta_w_0", "delta_w_max", "kappa_minus", "kappa_plus", "kappa_plus_bar"):
            raise TypeError(f"unknown inertia parameter {k}")
        setattr(ic, k, float(v))
    return ic


def inertia_result(ic):
    return {"delta_w": ic.delta_w, "attempts": ic.attempts, "delta_w_last": ic.delta_w_last}


def device_values(prob, device="cuda", formulation="lifted"):
    """Uploads a problem's values as float64 device tensors (w, g, h, sigma_x, sigma_s)."""
    import torch

    def t(a):
        return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=device)

    ss = prob.sigma_s if formulation == "lifted" else prob.sigma_s_ineq
    return t(prob.w_val), t(prob.g_val), t(prob.h_val), t(prob.sigma_x), t(ss)


def mlp_forward(feat, params, cache=None):
    import torch
    n = feat.shape[0]
    out = torch.empty(n, dtype=torch.float32, device=feat.device)
    lib = L.load()
    L.check(lib.ckkt_mlp_forward(n, _ptr(feat), _ptr(params), _ptr(out), _ptr(cache), _stream()), "ckkt_mlp_forward")
    return out


def mlp_backward(feat, params, cache, g_out):
    import torch
    n = feat.shape[0]
    lib = L.load()
    ws = torch.empty(max(lib.ckkt_mlp_workspace(n), 16), dtype=torch.uint8, device=feat.device)
    grad = torch.empty(L.MLP_NPARAM, dtype=torch.float32, device=feat.device)
    L.check(lib.ckkt_mlp_backward(n, _ptr(feat), _ptr(params), _ptr(cache), _ptr(g_out), _ptr(grad), _ptr(ws),
                                  _stream()), "ckkt_mlp_backward")
    return grad


def mlp_backward_noalloc(feat, params, cache, g_out, grad=None):
    """ckkt_mlp_backward_noalloc: the same gradient with the library's static
    scratch (no workspace); ``grad`` may be a preallocated output."""
    import torch
    n = feat.shape[0]
    lib = L.load()
    if grad is None:
        grad = torch.empty(L.MLP_NPARAM, dtype=torch.float32, device=feat.device)
    L.check(lib.ckkt_mlp_backward_noalloc(n, _ptr(feat), _ptr(params), _ptr(cache), _ptr(g_out), _ptr(grad),
                                          _stream()), "ckkt_mlp_backward_noalloc")
    return grad


def adam(params, grad, m, v, step, lr):
    lib = L.load()
    L.check(lib.ckkt_adam(params.numel(), _ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(step), float(lr),
                          _stream()), "ckkt_adam")


def init_mlp_params(seed=0, device="cuda"):
    """Starting parameters of the learned preconditioner's MLP (layout of
    CKKT_MLP_NPARAM in include/ckkt.h), as a float32 device tensor: hidden
    weights drawn N(0, 1/fan_in) (LeCun scaling for the tanh layers), zero
    biases, and an output layer of small weights so that the network starts
    near o = 0 (D = I, the plain stale-factor preconditioner)."""
    import torch
    rng = np.random.default_rng(seed + 0x5EED)
    F, H = L.MLP_F, L.MLP_H
    parts = [rng.normal(0.0, 1.0 / np.sqrt(F), H * F), np.zeros(H),
             rng.normal(0.0, 1.0 / np.sqrt(H), H * H), np.zeros(H),
             rng.normal(0.0, 1e-2, H), np.zeros(1)]
    theta = np.concatenate(parts).astype(np.float32)
    assert theta.size == L.MLP_NPARAM
    return torch.as_tensor(theta, device=device)
