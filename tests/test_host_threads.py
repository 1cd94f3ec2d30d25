"""Host worker threads of the analysis: an exception in a worker (e.g. an
allocation failure) is carried to the calling thread and every thread is
joined (run_threads in analysis.hpp), built with g++ and also run under
ThreadSanitizer.  CPU only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2405_14236_amd", "csrc")
SRC = os.path.join(ROOT, "tests", "sanitize", "threads.cpp")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


@pytest.mark.parametrize("flags", [[], ["-fsanitize=thread"]])
def test_worker_exception_reaches_caller(tmp_path, flags):
    exe = tmp_path / "threads"
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-pthread", *flags, "-I", CSRC, "-o", str(exe), SRC],
                   check=True, capture_output=True, timeout=300)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120,
                       env=dict(os.environ, TSAN_OPTIONS="halt_on_error=1"))
    assert r.returncode == 0, (r.stdout, r.stderr[-3000:])
    assert "run_threads ok" in r.stdout
