"""Mixed precision against FP64 on observables (the absorber test case of Section V-A
at 8 x 8 x 32): the FP32-inner / FP64-outer solution must give the FP64 field to
well within the solver tolerance's effect and the same reflection R."""
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("precision", [1, 5], ids=["fp32-inner-arnoldi", "fp64-inner-arnoldi"])
def test_mixed_tier_reproduces_fp64_observables(precision):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1803_06237_amd import experiments
    r = experiments.mixed_vs_fp64(precision=precision)
    print(r)
    for d, l2, dR, r64, r32 in zip(r["degrees"], r["rel_l2"], r["rel_dR"], r["rel_res_fp64"], r["rel_res_mixed"]):
        assert r64 <= 1e-8 and r32 <= 1e-8, d
        assert l2 <= 1e-7, (d, l2)
        assert dR <= 1e-3, (d, dR)
    assert min(r["inner_iters"]) > 0
