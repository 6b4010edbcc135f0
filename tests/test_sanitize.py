"""Host Green tables (green_table.cpp) under AddressSanitizer and
UndefinedBehaviorSanitizer: the quadrature, its threads and the table writes run
without a report, and the tables still equal the oracle's."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import green, jm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1803_06237_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("asan") / "tables_asan")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + CSRC,
           "-I" + os.path.join(ROOT, "include"), os.path.join(CSRC, "green_table.cpp"),
           os.path.join(ROOT, "tests", "sanitize", "tables_main.cpp"), "-o", out, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return out


@pytest.mark.parametrize("n,kappa", [((4, 3, 5), 0.3), ((1, 2, 9), 0.05)], ids=["4x3x5", "1x2x9"])
def test_tables_clean_under_sanitizers(driver, tmp_path, n, kappa):
    path = str(tmp_path / "tables.bin")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([driver, *map(str, n), repr(kappa), "3", path], capture_output=True, text=True, env=env,
                       timeout=300)
    assert r.returncode == 0 and "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, \
        r.stderr[-3000:]
    N = int(np.prod(n))
    raw = np.fromfile(path, dtype=np.complex128)
    assert raw.size == 9 * N
    tn = raw[:6 * N].reshape((6,) + n)
    tk = raw[6 * N:].reshape((3,) + n)
    want_n = green.green_table(n, kappa)
    want_k = jm.curl_table(n, kappa)
    assert np.max(np.abs(tn - want_n)) <= 1e-13 * np.max(np.abs(want_n))
    assert np.max(np.abs(tk - want_k)) <= 1e-13 * np.max(np.abs(want_k))
