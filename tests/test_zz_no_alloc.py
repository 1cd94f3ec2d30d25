"""The allocation-free MLP backward (ckkt_mlp_backward_noalloc) against the
workspace form (ckkt_mlp_backward) through the C-ABI: bitwise equal
gradients on two calls in a row, the first at the row limit and the second
smaller (the static scratch still holds the first call's values), plus the
oracle's gradient within the FP32 tolerance of the other MLP tests, and the
row limit rejected before any device work."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import mlp as om
from paper_2405_14236_amd import _lib as L
from paper_2405_14236_amd.solver import mlp_backward, mlp_backward_noalloc, mlp_forward

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _case(n, seed):
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((n, om.F)) * 0.5
    f[:, 7] = 1.0
    theta = om.init_params(seed) + 0.05 * rng.standard_normal(om.NPARAM)
    g_o = rng.standard_normal(n)
    t32 = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=DEV)
    return f, theta, g_o, t32(f), t32(theta), t32(g_o)


@pytest.mark.parametrize("sizes", [(L.MLP_NOALLOC_MAX_ROWS, 1000), (5000, 1)])
def test_noalloc_backward_matches_workspace_form(sizes):
    for call, n in enumerate(sizes):
        print(f"\n[case] mlp_backward_noalloc call {call} n={n}", flush=True)
        f, theta, g_o, feat, prm, go = _case(n, 10 + call)
        cache = torch.empty(2 * om.H * n, dtype=torch.float32, device=DEV)
        mlp_forward(feat, prm, cache)
        g_ws = mlp_backward(feat, prm, cache, go)
        g_na = mlp_backward_noalloc(feat, prm, cache, go)
        torch.cuda.synchronize()
        assert torch.equal(g_ws, g_na), (call, n, (g_ws - g_na).abs().max().item())
        f32, th32 = f.astype(np.float32).astype(np.float64), theta.astype(np.float32).astype(np.float64)
        _, c_ref = om.forward(th32, f32)
        g_ref = om.backward(th32, f32, c_ref, g_o.astype(np.float32).astype(np.float64))
        g = g_na.cpu().numpy()
        assert np.abs(g - g_ref).max() <= 1e-3 * max(1.0, np.abs(g_ref).max()), np.abs(g - g_ref).max()


def test_noalloc_backward_rejects_rows_beyond_limit():
    lib = L.load()
    grad = torch.zeros(L.MLP_NPARAM, dtype=torch.float32, device=DEV)
    dummy = torch.zeros(8, dtype=torch.float32, device=DEV)
    p = lambda t: __import__("ctypes").c_void_p(t.data_ptr())
    rc = lib.ckkt_mlp_backward_noalloc(L.MLP_NOALLOC_MAX_ROWS + 1, p(dummy), p(dummy), p(dummy), p(dummy), p(grad),
                                       None)
    assert rc == -1  # CKKT_ERR_ARG, nothing launched
    assert torch.count_nonzero(grad).item() == 0
