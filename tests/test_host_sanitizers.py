"""The host analysis (ordering, symbolic factorization, assembly recipe with
its worker threads) and the sequential host factor-solve built with g++
under AddressSanitizer + UndefinedBehaviorSanitizer and, separately,
ThreadSanitizer, and run on generated patterns (LiftedKKT, HyKKT, split
dense rows, a network-flow problem).  Any report aborts the run.  CPU only;
no GPU code is built with a sanitizer."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

from paper_2405_14236_amd import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2405_14236_amd", "csrc")
SOURCES = [os.path.join(ROOT, "tests", "sanitize", "driver.cpp")] + \
          [os.path.join(CSRC, f) for f in ("analysis.cpp", "ordering.cpp", "hostref.cpp")]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


def _write_cases(path):
    cases = [(workloads.tiny_grid(0), 0, 0),
             (workloads.tiny_grid(1), 1, 0),
             (workloads.with_dense_rows(workloads.tiny_grid(2, sigma_range=(-2, 2)), count=3, frac=0.6, seed=2), 0, 50),
             (workloads.network_flow(300, seed=3), 0, 0)]
    with open(path, "wb") as f:
        def put(a, dt):
            a = np.ascontiguousarray(a, dtype=dt)
            f.write(struct.pack("q", a.size))
            f.write(a.tobytes())
        for p, hy, dmin in cases:
            put([p.n, p.m_eq, p.m_ineq, hy, dmin], np.int32)
            for a in (p.w_ptr, p.w_idx, p.g_ptr, p.g_idx, p.h_ptr, p.h_idx):
                put(a, np.int32)
            ss = p.sigma_s_ineq if hy else p.sigma_s
            rhs = p.r1bar if hy else p.b
            for a in (p.w_val, p.g_val, p.h_val, p.sigma_x, ss, rhs):
                put(a, np.float64)
    return len(cases)


@pytest.mark.parametrize("sanitizer", ["address,undefined", "thread"])
def test_host_code_under_sanitizer(tmp_path, sanitizer):
    ncases = _write_cases(tmp_path / "cases.bin")
    exe = tmp_path / "drv"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-pthread", f"-fsanitize={sanitizer}",
           "-fno-sanitize-recover=all", "-I", CSRC, "-o", str(exe)] + SOURCES
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1",
               TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([str(exe), str(tmp_path / "cases.bin")], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("case ")]
    assert len(lines) == ncases and all(" failed -1 " in ln for ln in lines), r.stdout
    assert "dense 3" in lines[2]
