"""The bench's tuned CPU baseline computes the oracle's product."""
import numpy as np

import bench
from oracle import matvec as mv


def test_tuned_cpu_matvec_equals_the_oracle():
    rng = np.random.default_rng(4)
    n = (3, 5, 6)
    M = mv.circulant_size(n)
    spec = rng.standard_normal((6,) + M) + 1j * rng.standard_normal((6,) + M)
    chi = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x = rng.standard_normal((3,) + n) + 1j * rng.standard_normal((3,) + n)
    want = mv.matvec_fft(spec, chi, x)
    got = bench.cpu_tuned_matvec(spec, chi, x, workers=2)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_tuned_cpu_baseline_reports_its_cores():
    r = bench.cpu_tuned_baseline((4, 4, 8), seconds_budget=0.2)
    assert r["value"] > 0 and r["cores"] >= 1 and r["kind"] == "scipy.fft"
