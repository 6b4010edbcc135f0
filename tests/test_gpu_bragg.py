"""The Bragg-grating transmission read-out on the GPU path (Section II-B, Section V):
the slice field from solved currents against the oracle, and a solve of a short
grating judged by the oracle's own residual."""
import math

import numpy as np
import pytest

from oracle import green, matvec as mv, observables
from paper_1803_06237_amd import experiments, inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1803_06237_amd import vie
    vie.lib()
    return vie


def _small_grating(lam=1.55):
    """9 x 5 x 64 voxels of 20 nm: a 7-voxel strip whose sidewalls step by one voxel
    every 8 voxels over two periods, absorbers of 8 voxels on both ends."""
    n3 = 64
    lo = np.zeros(n3, dtype=np.int64)
    hi = np.zeros(n3, dtype=np.int64)
    for p in range(2):
        a = 12 + 16 * p
        lo[a:a + 8], hi[a:a + 8] = -1, 1
        lo[a + 8:a + 16], hi[a + 8:a + 16] = 1, -1
    k0 = 2 * math.pi / lam
    return inputs.Waveguide(n=(9, 5, n3), h=0.02, core_x=(1, 8), core_y=(0, 5), core_z=(0, n3), n_abs=8, d=2,
                            sigma_max=inputs.sigma_max_for(1e-10, 2, 0.16, k0=k0), k0=k0, rough_lo=lo,
                            rough_hi=hi, ends="both")


def test_slice_field_matches_oracle():
    """E on the transmission slice (background voxels included) from arbitrary currents:
    the GPU read-out (one product with a uniform contrast of 1/2) against the oracle's
    (h^{3/2} e_inc + N w) / (h^{3/2} eps_r) with N w by its own FFT product."""
    vie = _dev()
    wg = _small_grating()
    z = inputs.bragg_slice(wg)
    assert z == 46 and (~wg.core_mask()[:, :, z]).any()
    rng = np.random.default_rng(5)
    w = rng.standard_normal((3,) + wg.n) + 1j * rng.standard_normal((3,) + wg.n)
    e = inputs.bragg_source(wg)
    plan = vie.Plan(wg.n, wg.h, wg.k0, wg.eps_b, fp32=True)
    got = experiments.bragg_slice_field(plan, wg, torch.from_numpy(w).cuda(), e)
    plan.close()
    spec = mv.spectrum(green.green_table(wg.n, mv.kappa_of(wg.h, wg.k0, wg.eps_b)))
    want = observables.total_field(w, mv.apply_N_fft(spec, w), e, wg.eps(), wg.eps_b, wg.h)[..., z]
    err = np.abs(got - want).max() / np.abs(want).max()
    print(f"slice field rel err {err:.3e}")
    assert err < 1e-12
    T = observables.slice_transmission(got, wg.h)
    assert abs(T - observables.slice_transmission(want, wg.h)) < 1e-10 * T


@pytest.mark.parametrize("lam", [1.52, 1.55])
def test_short_grating_solve_and_transmission(lam):
    """Ten periods behind a two-period lead-in (27 x 11 x 432 voxels), at two
    wavelengths: the batched mixed solve reaches 1e-8, the FP64 residual recomputed
    with the plan's FP64 product (oracle-parity tested on its own) agrees, and a
    single FP64 GMRES solve and a block-circulant preconditioned one give the same
    transmitted power."""
    vie = _dev()
    res = experiments.bragg_transmission([lam * 1e3], periods=10, lead_periods=2, batch=1)
    assert res["status"] == [0] and res["rel_res"][0] <= 1e-8
    T = res["T"][0]
    assert np.isfinite(T) and T > 0
    wg = inputs.bragg_grating(lam, periods=10, lead_periods=2)
    assert wg.n == (27, 11, 432)
    plan = vie.Plan(wg.n, wg.h, wg.k0, wg.eps_b, fp32=True)
    try:
        plan.set_contrast(torch.from_numpy(wg.eps()).cuda())
        e = inputs.bragg_source(wg)
        b = plan.rhs(torch.from_numpy(e).cuda())
        x, info = plan.solve(b, tol=1e-9, precision=0)
        assert info["status"] == 0
        r = plan.residual(x, b)
        rel = (torch.linalg.vector_norm(r) / torch.linalg.vector_norm(b)).item()
        assert rel <= 1.5e-9
        T64 = observables.slice_transmission(experiments.bragg_slice_field(plan, wg, x, e), wg.h)
    finally:
        plan.close()
    print(f"lambda {lam} T {T:.6e} fp64 {T64:.6e} iters {res['iters'][0]}/{res['inner_iters'][0]} fp64 {info['iters']}")
    assert abs(T - T64) <= 1e-6 * T64
    # the block-circulant preconditioned solve gives the same transmission
    rc = experiments.bragg_transmission([lam * 1e3], periods=10, lead_periods=2, batch=1, circulant=True)
    assert rc["status"] == [0] and rc["rel_res"][0] <= 1e-8
    assert abs(rc["T"][0] - T64) <= 1e-6 * T64


def test_full_grating_reflects_in_its_band_gap():
    """The 100-period grating at the edge of the sweep and at the centre of its band gap
    (1547.5 nm in the full 1520-1570 nm sweep with these permittivities): the
    transmitted power there is below a third of that at 1520 nm."""
    _dev()
    res = experiments.bragg_transmission([1520.0, 1547.5], batch=2)
    assert res["status"] == [0, 0] and max(res["rel_res"]) <= 1e-8
    ratio = res["T"][1] / res["T"][0]
    print(f"T(1547.5) / T(1520) = {ratio:.3f}, outer steps {res['iters']}")
    assert ratio < 1 / 3


def test_absorber_inside_the_grating_stagnates():
    """Section V, slow light, at reduced length (absorbers of 3 and 10 periods against
    30): inside the grating the reflection barely falls with the absorber's length,
    while on the uniform strip it falls by orders of magnitude, as O(L^{-2(d+1)})."""
    _dev()
    res = experiments.bragg_slow_light_study(wavelengths_nm=(1520.0,), absorber_periods=(3, 10), ref_periods=30)
    g, s = res["runs"]["1520/grating"], res["runs"]["1520/strip"]
    for r in (g, s):
        assert r["status"] == 0 and r["max_rel_res"] <= 1e-8
    print(f"grating R {g['R']} strip R {s['R']}")
    assert g["R"][1] / g["R"][0] > 0.5
    assert s["R"][1] / s["R"][0] < 1e-2
    assert g["R"][0] > 100 * s["R"][0]


def test_absorber_inside_the_grating_reflects_most_at_the_band_edge():
    """Section V, slow light: with the absorber inside the grating (40 periods against a
    90-period reference, circulant-preconditioned solves) the reflection at the band
    edge (1540 nm with these permittivities) is several times that far from the band
    (1520 nm): the group velocity falls toward the edge."""
    _dev()
    res = experiments.bragg_slow_light_spectrum([1520.0, 1540.0])
    assert res["status"] == [0, 0] and max(res["rel_res"]) <= 1e-8
    print(f"R(1520) {res['R'][0]:.3e} R(1540) {res['R'][1]:.3e}")
    assert res["R"][1] > 5 * res["R"][0]
