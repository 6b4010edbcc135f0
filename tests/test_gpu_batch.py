"""Batched solves (uneven grids, one launch per kernel shape, lockstep GMRES with
device-side masks, restart cycles replayed from a HIP graph), judged by the oracle."""
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


def _guides():
    """Uneven small guides: different n3, cross-sections and absorber profiles."""
    out = []
    for n, core, nabs, d in (((8, 8, 32), ((2, 6), (2, 6)), 8, 2), ((8, 8, 40), ((2, 6), (3, 5)), 6, 1),
                             ((6, 7, 24), ((1, 5), (2, 5)), 5, 0), ((5, 4, 37), ((1, 4), (1, 3)), 4, 3)):
        out.append(inputs.Waveguide(n=n, h=0.05, core_x=core[0], core_y=core[1], core_z=(0, n[2]), n_abs=nabs, d=d,
                                    sigma_max=2.0))
    return out


@pytest.fixture(scope="module")
def systems():
    vie = _dev()
    sys = []
    for i, wg in enumerate(_guides()):
        kap = mv.kappa_of(wg.h, wg.k0, wg.eps_b)
        op = mv.Operator(green.green_table(wg.n, kap), mv.contrast(wg.eps(), wg.eps_b))
        plan = vie.Plan(wg.n, wg.h, wg.k0, wg.eps_b, fp32=True)
        plan.set_contrast(torch.from_numpy(wg.eps()).cuda())
        b = inputs.gaussian_rhs(wg.n, 100 + i)
        sys.append((wg, op, plan, b))
    return sys


def _rel(op, b, x):
    return np.linalg.norm(b.ravel() - op(x.ravel())) / np.linalg.norm(b)


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_solutions_satisfy_the_oracle(systems, precision):
    vie = _dev()
    plans = [s[2] for s in systems]
    bs = [torch.from_numpy(s[3]).cuda() for s in systems]
    xs, infos, code = vie.solve_batch(plans, bs, tol=1e-8, restart=30, precision=precision, inner_restart=10,
                                      inner_tol=1e-3)
    assert code == vie.VIE_OK, infos
    for (wg, op, plan, b), x, info in zip(systems, xs, infos):
        rr = _rel(op, b, x.cpu().numpy())
        print(wg.n, info, rr)
        assert info["status"] == 0 and info["rel_res_true"] <= 1e-8
        assert rr <= 1.01e-8
        if precision == 1:
            assert info["inner_iters"] > 0


def test_graph_replays_match_eager_cycles(systems):
    """Short restarts force many cycles; every replay of the captured cycle must give
    the same iterates as launching the same kernels eagerly."""
    vie = _dev()
    plans = [s[2] for s in systems]
    bs = [torch.from_numpy(s[3]).cuda() for s in systems]
    for precision in (0, 1):
        xg, ig, cg = vie.solve_batch(plans, bs, tol=1e-8, restart=2, precision=precision, inner_restart=2,
                                     inner_tol=1e-2, use_graph=True)
        xe, ie, ce = vie.solve_batch(plans, bs, tol=1e-8, restart=2, precision=precision, inner_restart=2,
                                     inner_tol=1e-2, use_graph=False)
        print(precision, [(i["iters"], i["restarts"]) for i in ig])
        assert cg == ce == vie.VIE_OK
        assert max(i["restarts"] for i in ig) > 2      # the graph was replayed several times
        for a, b, i1, i2 in zip(xg, xe, ig, ie):
            assert i1["iters"] == i2["iters"] and i1["restarts"] == i2["restarts"]
            assert torch.equal(a, b)


@pytest.mark.parametrize("rhs", ["on_support", "everywhere"])
def test_batch_equals_single_solve_residual_level(systems, rhs):
    """The single and the batch solver both keep Krylov vectors compressed to the
    support columns and solve A_SS x_S = b_S - (A b_off)_S, so for b = h^{3/2} chi e
    (zero off the support) and for a Gaussian b (non-zero everywhere) the iterates
    agree to rounding."""
    vie = _dev()
    wg, op, plan, _ = systems[0]
    if rhs == "on_support":
        b = mv.rhs_from_field(wg.eps(), wg.eps_b, inputs.gaussian_rhs(wg.n, 7), wg.h)
    else:
        b = inputs.gaussian_rhs(wg.n, 7)
    x1, info1 = plan.solve(torch.from_numpy(b).cuda(), tol=1e-8, restart=30)
    xs, infos, code = vie.solve_batch([plan], [torch.from_numpy(b).cuda()], tol=1e-8, restart=30)
    assert code == vie.VIE_OK
    assert infos[0]["iters"] == info1["iters"]
    assert abs(infos[0]["rel_res_true"] - info1["rel_res_true"]) < 1e-12
    assert torch.linalg.norm(xs[0] - x1) / torch.linalg.norm(x1) < 1e-10
    assert _rel(op, b, xs[0].cpu().numpy()) <= 1.01e-8


def test_batch_resumes_from_x0(systems):
    """use_x0: a batch stopped by maxit continues from its iterates to the tolerance;
    the oracle judges the result, and an exact start needs no step."""
    vie = _dev()
    plans = [s[2] for s in systems]
    bs = [torch.from_numpy(s[3]).cuda() for s in systems]
    xs, infos, code = vie.solve_batch(plans, bs, tol=1e-8, restart=10, maxit=10)
    assert code == vie.VIE_ENOCONV
    xs, infos, code = vie.solve_batch(plans, bs, xs=xs, tol=1e-8, restart=30, use_x0=True)
    assert code == vie.VIE_OK, infos
    for (wg, op, plan, b), x, info in zip(systems, xs, infos):
        assert _rel(op, b, x.cpu().numpy()) <= 1.01e-8
        assert info["matvecs"] >= info["iters"] + 1
    again = [x.clone() for x in xs]
    xs2, infos2, code = vie.solve_batch(plans, bs, xs=again, tol=1e-6, restart=30, use_x0=True)
    assert code == vie.VIE_OK
    for x, x2, info in zip(xs, xs2, infos2):
        assert info["iters"] == 0 and info["rel_res_true"] <= 1.01e-8
        assert torch.equal(x, x2)


def test_batch_system_without_contrast(systems):
    """A guide whose permittivity is the background everywhere has no support: A is
    the identity and x = b, next to an ordinary system of the same batch."""
    vie = _dev()
    wg, op, plan, b = systems[2]
    empty = vie.Plan(wg.n, wg.h, wg.k0, wg.eps_b)
    empty.set_contrast(torch.full(wg.n, wg.eps_b, dtype=torch.complex128).cuda())
    b2 = torch.from_numpy(inputs.gaussian_rhs(wg.n, 300)).cuda()
    xs, infos, code = vie.solve_batch([plan, empty], [torch.from_numpy(b).cuda(), b2], tol=1e-8, restart=30)
    assert code == vie.VIE_OK
    assert _rel(op, b, xs[0].cpu().numpy()) <= 1.01e-8
    assert torch.equal(xs[1], b2) and infos[1]["iters"] == 0 and infos[1]["rel_res_true"] == 0


def test_one_plan_several_right_hand_sides(systems):
    vie = _dev()
    wg, op, plan, _ = systems[1]
    rhs = [inputs.gaussian_rhs(wg.n, 200 + k) for k in range(3)]
    xs, infos, code = vie.solve_batch([plan] * 3, [torch.from_numpy(r).cuda() for r in rhs], tol=1e-8, restart=40,
                                      precision=1, inner_restart=8, inner_tol=1e-3)
    assert code == vie.VIE_OK
    for r, x in zip(rhs, xs):
        assert _rel(op, r, x.cpu().numpy()) <= 1.01e-8


def test_batch_maxit_reports_noconv(systems):
    vie = _dev()
    plans = [s[2] for s in systems]
    bs = [torch.from_numpy(s[3]).cuda() for s in systems]
    xs, infos, code = vie.solve_batch(plans, bs, tol=1e-14, restart=4, maxit=8)
    assert code == vie.VIE_ENOCONV
    for (wg, op, plan, b), x, info in zip(systems, xs, infos):
        assert info["status"] == vie.VIE_ENOCONV and info["iters"] <= 8 + 4
        assert abs(_rel(op, b, x.cpu().numpy()) - info["rel_res_true"]) < 1e-9


def test_long_guides_family_batch():
    """32 x 32 x (192, 256, 320) guides with 0.5/1/1.5 um absorbers, FP32-inner mixed tier,
    every kernel shape of the batch (four-step z of lengths 512 and 1024, 64 x 64 xy)."""
    vie = _dev()
    plans, bs = [], []
    for L, d in ((0.5, 2), (1.0, 0), (1.5, 3)):
        wg = inputs.strip_family(L, d)
        p = vie.Plan(wg.n, wg.h, wg.k0, wg.eps_b, fp32=True)
        p.set_contrast(torch.from_numpy(wg.eps()).cuda())
        b = p.rhs(torch.from_numpy(inputs.transverse_dipole_field(wg)).cuda())
        plans.append(p)
        bs.append(b)
    xs, infos, code = vie.solve_batch(plans, bs, tol=1e-8, restart=50, precision=1, inner_restart=20,
                                      inner_tol=1e-3)
    print(infos)
    assert code == vie.VIE_OK
    for p, b, x, info in zip(plans, bs, xs, infos):
        r = p.residual(x, b)
        rel = (torch.linalg.norm(r) / torch.linalg.norm(b)).item()
        assert rel <= 1e-8 and abs(rel - info["rel_res_true"]) < 1e-12


def test_batch_circulant_tier(systems):
    """precision 3: each system's FGMRES preconditioned by its plan's block circulant;
    solutions judged by the oracle, fewer iterations than plain GMRES."""
    vie = _dev()
    plans = [s[2] for s in systems]
    for p in plans:
        p.build_circulant()
    bs = [torch.from_numpy(s[3]).cuda() for s in systems]
    x0, i0, c0 = vie.solve_batch(plans, bs, tol=1e-8, restart=30, precision=0)
    xs, infos, code = vie.solve_batch(plans, bs, tol=1e-8, restart=30, precision=3)
    assert code == vie.VIE_OK, infos
    for (wg, op, plan, b), x, info, info0 in zip(systems, xs, infos, i0):
        rr = _rel(op, b, x.cpu().numpy())
        print(wg.n, info["iters"], "vs plain", info0["iters"], rr)
        assert info["status"] == 0 and rr <= 1.01e-8
        assert info["iters"] < info0["iters"]
    plans[0].set_contrast(torch.from_numpy(systems[0][0].eps()).cuda())       # releases its preconditioner
    with pytest.raises(vie.VieError) as ei:
        vie.solve_batch(plans, bs, tol=1e-8, restart=30, precision=3)
    assert ei.value.code == vie.VIE_ESTATE
