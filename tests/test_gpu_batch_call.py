"""ckkt_batch_factorize_solve: factorization and solve of a whole batch in one
call (one captured launch sequence, one host synchronization).

* every instance meets the gate by the oracle's certificate, and agrees
  with the two-call path (ckkt_factorize + ckkt_solve) on the same batch;
* the device refinement is masked per instance: an instance that already met
  the tolerance after the first solve is bitwise the same whatever the
  number of device steps;
* the captured sequence is replayed for new values in the same buffers and
  captured again for new buffers;
* an FP32 factor whose device steps cannot reach the tolerance hands over
  to the refinement of ckkt_solve (fallback flag 4) and still meets the
  gate; arguments out of range are rejected.
"""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2405_14236_amd import _lib as L
from paper_2405_14236_amd import workloads
from paper_2405_14236_amd.solver import Solver
from tests._common import omega_of

pytestmark = pytest.mark.gpu
DEV = "cuda"


def print_case(name, **kw):
    print(f"\n[case] {name} {kw}", flush=True)


def _batch(nodes, seed, srange=(-8, 8)):
    return [workloads.network_flow(N, seed=seed + i, sigma_range=srange) for i, N in enumerate(nodes)]


def _vals(probs):
    cat = lambda xs: torch.as_tensor(np.concatenate(xs), device=DEV)
    w = cat([q.w_val for q in probs]); g = cat([q.g_val for q in probs]); h = cat([q.h_val for q in probs])
    sx = cat([q.sigma_x for q in probs])
    ss = cat([q.sigma_s[:q.m_eq] for q in probs] + [q.sigma_s[q.m_eq:] for q in probs])
    return [w, g, h, sx, ss], cat([q.b for q in probs])


def _split(probs, z):
    out, off = [], 0
    for q in probs:
        out.append(z[off:off + q.n]); off += q.n
    return out


@pytest.mark.parametrize("precision,gate", [("fp64", 1e-10), ("fp32_ir", 1e-8)])
def test_one_call_meets_gate_and_matches_two_calls(precision, gate):
    probs = _batch([600, 1100, 800, 1400, 500, 950], seed=200)
    print_case("batch_call", precision=precision, count=len(probs))
    s = Solver(None, "lifted", precision, batch=probs, tol=gate).bind(DEV)
    vals, b = _vals(probs)
    x, info, om = s.factorize_solve(*vals, b, refine=2)
    torch.cuda.synchronize()
    print(info, om)
    assert info["status"] == 0 and om.shape == (len(probs),) and om.max() <= gate
    parts = _split(probs, x.cpu().numpy())
    for q, xi in zip(probs, parts):
        assert omega_of(q, "lifted", xi) <= gate
    s2 = Solver(None, "lifted", precision, batch=probs, tol=gate).bind(DEV)
    s2.factorize(*vals)
    z, _ = s2.solve(b)
    for xi, zi in zip(parts, _split(probs, z.cpu().numpy())):
        assert np.abs(xi - zi).max() <= 1e-6 * np.abs(zi).max()


def test_masked_steps_leave_converged_instances_bitwise():
    probs = _batch([700, 1200, 900, 1300], seed=230)
    print_case("batch_call_masked", count=len(probs))
    s = Solver(None, "lifted", "fp64", batch=probs, tol=1e-10).bind(DEV)
    vals, b = _vals(probs)
    x0, info0, om0 = s.factorize_solve(*vals, b, refine=0, raise_on_error=False)
    x0 = x0.cpu().numpy()
    x3, info3, om3 = s.factorize_solve(*vals, b, refine=3)
    x3 = x3.cpu().numpy()
    print(info0, om0, info3, om3)
    assert om3.max() <= 1e-10
    done = om0 <= 1e-10
    for i, (a, c) in enumerate(zip(_split(probs, x0), _split(probs, x3))):
        if done[i]:
            assert np.array_equal(a, c), i


def test_replay_for_new_values_and_recapture_for_new_buffers():
    probs = _batch([800, 1000, 600], seed=260)
    print_case("batch_call_replay", count=len(probs))
    s = Solver(None, "lifted", "fp64", batch=probs, tol=1e-10).bind(DEV)
    vals, b = _vals(probs)
    x, info, _ = s.factorize_solve(*vals, b, refine=1)
    rng = np.random.default_rng(3)
    # new diagonals written into the same buffers: the captured sequence is replayed
    sx_new = np.concatenate([workloads.log_uniform(rng, q.n) for q in probs])
    vals[3].copy_(torch.as_tensor(sx_new, device=DEV))
    x, info, om = s.factorize_solve(*vals, b, refine=1)
    xs = _split(probs, x.cpu().numpy())
    off = 0
    for q, xi in zip(probs, xs):
        q2 = dataclasses.replace(q, sigma_x=sx_new[off:off + q.n]); off += q.n
        assert omega_of(q2, "lifted", xi) <= 1e-10
    # a new right-hand side buffer and a new solution buffer: captured again
    b2 = b.clone() * 2.0
    out2 = torch.empty_like(b2)
    x2, info2, _ = s.factorize_solve(*vals, b2, out=out2, refine=1)
    assert x2.data_ptr() == out2.data_ptr()
    assert torch.allclose(x2, 2.0 * x, rtol=1e-8, atol=0.0)


def test_fp32_device_steps_hand_over_to_host_refinement():
    probs = _batch([900, 700], seed=290)
    print_case("batch_call_handover", count=len(probs))
    s = Solver(None, "lifted", "fp32_ir", batch=probs, tol=1e-8).bind(DEV)
    vals, b = _vals(probs)
    x, info, om = s.factorize_solve(*vals, b, refine=0)
    print(info, om)
    assert info["status"] == 0 and info["fallback"] & 4 and om.max() <= 1e-8
    for q, xi in zip(probs, _split(probs, x.cpu().numpy())):
        assert omega_of(q, "lifted", xi) <= 1e-8


def test_arguments_out_of_range():
    probs = _batch([500, 600], seed=300)
    vals, b = _vals(probs)
    s = Solver(None, "lifted", "fp64", batch=probs).bind(DEV)
    out = torch.empty_like(b)
    rc = s.factorize_solve(*vals, b, out, refine=L.MAX_DEVICE_REFINE + 1, raise_on_error=False)[1]["status"]
    assert rc == -1
    hy = Solver(None, "hykkt", "fp64", batch=probs).bind(DEV)
    rc = hy.factorize_solve(*vals, b, out, raise_on_error=False)[1]["status"]
    assert rc == -1
