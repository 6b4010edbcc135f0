"""The strip reflection study (Section V-A) through the batched solver, at reduced
length: every system converges to the tolerance in FP64 terms, and the transition
reflection falls as the absorber grows (Section IV-C)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_strip_study_converges_and_reflection_falls_with_length():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1803_06237_amd import experiments, vie
    vie.lib()
    res = experiments.strip_reflection_study(r_rts=(1e-10,), degrees=(2,), lengths=(0.45, 0.9, 1.8, 3.6),
                                             strip_len=120)
    run = res["runs"]["1e-10/2"]
    print(run)
    assert run["status"] == vie.VIE_OK
    assert run["max_rel_res"] <= 1e-8
    R = run["R"]
    assert len(R) == 3 and all(np.isfinite(R))
    assert R[0] > R[1] > R[2]
    assert R[0] < 1.0


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
