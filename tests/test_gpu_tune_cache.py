"""The plan-time tuner's persistent cache (VIE_TUNE_CACHE): a plan that tunes appends
its choice per precision, and a later process takes a stored choice for its grid
instead of timing candidates; lines of another candidate set are not read."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1803_06237_amd import vie
    vie.lib()
    return vie


def test_tuner_writes_and_reads_its_cache(tmp_path):
    vie = _dev()
    path = tmp_path / "tune.txt"
    old = os.environ.get("VIE_TUNE_CACHE")
    os.environ["VIE_TUNE_CACHE"] = str(path)
    try:
        # a 64 x 32 cross-section (three xy candidates) no other test plans
        n = (18, 10, 40)
        plan = vie.Plan(n, 0.05, 2 * 3.141592653589793 / 1.55, 2.1, fp32=True)
        t64, t32 = plan.tune(0), plan.tune(1)
        plan.close()
    finally:
        if old is None:
            del os.environ["VIE_TUNE_CACHE"]
        else:
            os.environ["VIE_TUNE_CACHE"] = old
    lines = [l.split() for l in path.read_text().splitlines()]
    mine = [l for l in lines if l[1:4] == ["18", "10", "40"]]
    assert sorted(int(l[4]) for l in mine) == [8, 16]          # FP32 and FP64 complex values
    arch = mine[0][0]
    assert arch.endswith("/xy6432")
    for l in mine:
        t = t64 if l[4] == "16" else t32
        assert int(l[7]) == t["xy_variant"]

    # a fresh process with forced lines for another grid takes them without timing;
    # a line in the format of an older candidate set (no suffix) is ignored
    n2 = (19, 11, 33)
    seeded = tmp_path / "seeded.txt"
    base = arch.split("/")[0]
    seeded.write_text(f"{arch} 19 11 33 16 0 0 0\n{arch} 19 11 33 8 0 0 1\n{base} 19 11 33 16 0 0 2\n")
    child = (
        "import sys, torch; sys.path.insert(0, %r)\n"
        "from paper_1803_06237_amd import vie\n"
        "p = vie.Plan(%r, 0.05, 4.05, 2.1, fp32=True)\n"
        "print(p.tune(0)['xy_variant'], p.tune(1)['xy_variant'])\n" % (ROOT, n2))
    env = dict(os.environ, VIE_TUNE_CACHE=str(seeded))
    r = subprocess.run([sys.executable, "-c", child], env=env, capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr
    assert r.stdout.split() == ["0", "1"]
    # the process appended nothing: both precisions came from the file
    assert len(seeded.read_text().splitlines()) == 3
