"""The allocation-free solve entry point (vie_solve_noalloc) against vie_solve: the
same solution on two calls in a row, the second on a smaller system, both judged by
the oracle's own product; sizes beyond the static scratch are refused."""
import ctypes

import numpy as np
import pytest

from oracle import green, matvec as mv
from paper_1803_06237_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1803_06237_amd import vie
    vie.lib()
    return vie


def _system(vie, n, n_abs, core):
    wg = inputs.Waveguide(n=n, h=0.05, core_x=core, core_y=core, core_z=(0, n[2]), n_abs=n_abs, d=2,
                          sigma_max=2.0)
    kap = mv.kappa_of(wg.h, wg.k0, wg.eps_b)
    op = mv.Operator(green.green_table(wg.n, kap), mv.contrast(wg.eps(), wg.eps_b))
    plan = vie.Plan(wg.n, wg.h, wg.k0, wg.eps_b, fp32=False)
    plan.set_contrast(torch.from_numpy(wg.eps()).cuda())
    b = mv.rhs_from_field(wg.eps(), wg.eps_b, inputs.strip_small_dipole_rhs_field(wg), wg.h)
    b = b + 0.1 * inputs.gaussian_rhs(wg.n, 3) * mv.contrast(wg.eps(), wg.eps_b)[None]
    return wg, op, plan, b


def _check_pair(vie, wg, op, plan, b, precision):
    bd = torch.from_numpy(b).cuda()
    x_ref, info_ref = plan.solve(bd, tol=1e-8, restart=30, precision=precision)
    print(f"solve n={wg.n} p={precision}: {info_ref}", flush=True)
    x_na, info_na = plan.solve_noalloc(bd, tol=1e-8, restart=30, precision=precision)
    print(f"noalloc n={wg.n} p={precision}: {info_na}", flush=True)
    xr, xn = x_ref.cpu().numpy(), x_na.cpu().numpy()
    assert info_na["status"] == 0 and info_na["iters"] == info_ref["iters"]
    assert np.abs(xn - xr).max() <= 1e-12 * np.abs(xr).max()
    rr = np.linalg.norm(b.ravel() - op(xn.ravel())) / np.linalg.norm(b)
    assert rr <= 1.01e-8, rr


@pytest.mark.parametrize("precision", [0, 3], ids=["gmres", "circulant"])
def test_noalloc_solve_matches_solve_twice_second_smaller(precision):
    vie = _dev()
    big = _system(vie, (8, 8, 32), 8, (2, 6))
    small = _system(vie, (6, 6, 16), 4, (2, 4))
    for wg, op, plan, b in (big, small):
        if precision == 3:
            plan.build_circulant()
        _check_pair(vie, wg, op, plan, b, precision)


def test_noalloc_refuses_what_does_not_fit_and_other_tiers():
    vie = _dev()
    wg, op, plan, b = _system(vie, (8, 8, 32), 8, (2, 6))
    bd = torch.from_numpy(b).cuda()
    # restart 4096 on 3 |S| n3 = 1536 values: the basis alone is 100 MB > 64 MiB
    with pytest.raises(vie.VieError) as e:
        plan.solve_noalloc(bd, restart=4096)
    assert e.value.code == vie.VIE_EINVAL
    assert b"scratch" in vie.lib().vie_last_error(plan.handle)
    with pytest.raises(vie.VieError):
        plan.solve_noalloc(bd, precision=1)
    # still usable afterwards
    x, info = plan.solve_noalloc(bd, tol=1e-8, restart=30)
    rr = np.linalg.norm(b.ravel() - op(x.cpu().numpy().ravel())) / np.linalg.norm(b)
    assert info["status"] == 0 and rr <= 1.01e-8
