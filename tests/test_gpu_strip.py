"""The strip reflection study (Section V-A) through the batched solver, at reduced
length: every system converges to the tolerance in FP64 terms, and the transition
reflection falls as the absorber grows (Section IV-C)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _oracle_residual(wg, b, x):
    """||b - A x|| / ||b|| with the oracle's own table (16 worker processes) and FFT product."""
    from oracle import green, matvec as mv
    kap = mv.kappa_of(wg.h, wg.k0, wg.eps_b)
    op = mv.Operator(green.green_table(wg.n, kap, workers=16), mv.contrast(wg.eps(), wg.eps_b))
    return np.linalg.norm(b.ravel() - op(x.ravel())) / np.linalg.norm(b)


def test_strip_study_converges_and_reflection_falls_with_length():
    """The paper's strip (30 x 12 voxels of 50/3 nm, one absorber at the far end,
    complex-source dipole; Section II-A, Section V-A) at reduced length.  The shortest
    guide's solution from the batched mixed-precision solve is judged by the oracle's
    residual, recomputed from its own table and product."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1803_06237_amd import experiments, vie
    vie.lib()
    res = experiments.strip_reflection_study(r_rts=(1e-10,), degrees=(2,), lengths=(0.45, 0.9, 1.8, 3.6),
                                             strip_len=120, keep=(0.45,))
    run = res["runs"]["1e-10/2"]
    sol = run.pop("solutions")
    print(run)
    assert run["status"] == vie.VIE_OK
    assert run["max_rel_res"] <= 1e-8
    R = run["R"]
    assert len(R) == 3 and all(np.isfinite(R))
    assert R[0] > R[1] > R[2]
    assert R[0] < 1.0
    wg, b, x = sol[0.45]
    assert wg.n == (30, 12, 147)
    rr = _oracle_residual(wg, b, x)
    print("oracle residual of the 0.45 um guide", rr)
    assert rr <= 1.01e-8


def test_matched_absorber_study_converges_and_reflection_falls_with_length():
    """The e&m variant through the JM-VIE at the same reduced length."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1803_06237_amd import experiments, vie
    vie.lib()
    kw = dict(r_rts=(1e-10,), degrees=(2,), lengths=(0.45, 0.9, 1.8, 3.6), strip_len=120)
    em = experiments.strip_reflection_study_em(**kw)["runs"]["1e-10/2"]
    e = experiments.strip_reflection_study(**kw)["runs"]["1e-10/2"]
    print("e&m", em)
    print("e", e["R"])
    assert em["status"] == vie.VIE_OK
    assert em["max_rel_res"] <= 1e-8
    R = em["R"]
    assert len(R) == 3 and all(np.isfinite(R))
    assert R[0] > R[1] > R[2]
