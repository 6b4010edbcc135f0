"""Network training checkpoints: the raw-binary + JSON-header format round-trips
exactly and refuses foreign or truncated files (CPU); a network restored from a
checkpoint continues training with the losses and weights of the original (GPU)."""
import json

import numpy as np
import pytest

from paper_1803_06237_amd import learned


def test_checkpoint_round_trip_and_refusals(tmp_path):
    rng = np.random.default_rng(0)
    n = 1037
    w, m = rng.standard_normal(n).astype(np.float32), rng.standard_normal(n).astype(np.float32)
    v = rng.random(n).astype(np.float32)
    path = tmp_path / "ck.bin"
    learned.write_checkpoint(str(path), w, m, v, 17, {"grid": [16, 16, 32], "seed": 3, "lr": 1e-3})
    w2, m2, v2, step, meta = learned.read_checkpoint(str(path))
    assert step == 17 and meta == {"grid": [16, 16, 32], "seed": 3, "lr": 1e-3}
    assert np.array_equal(w, w2) and np.array_equal(m, m2) and np.array_equal(v, v2)
    head = json.loads(path.read_bytes().split(b"\n", 1)[0])
    assert head["num_params"] == n and head["parts"] == ["weights", "adam_m", "adam_v"]
    # truncated payload
    (tmp_path / "cut.bin").write_bytes(path.read_bytes()[:-4])
    with pytest.raises(ValueError):
        learned.read_checkpoint(str(tmp_path / "cut.bin"))
    # another format
    (tmp_path / "other.bin").write_bytes(b'{"format": "something else", "version": 1}\n')
    with pytest.raises(ValueError):
        learned.read_checkpoint(str(tmp_path / "other.bin"))
    with pytest.raises(ValueError):
        learned.write_checkpoint(str(tmp_path / "bad.bin"), w, m[:-1], v, 1)


@pytest.mark.gpu
def test_restored_network_continues_training_identically(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1803_06237_amd import vie
    grid = (16, 16, 16)
    rng = np.random.default_rng(5)
    N = int(np.prod(grid))

    def sample():
        r = torch.from_numpy(rng.standard_normal(3 * N) + 1j * rng.standard_normal(3 * N)).cuda()
        chi = torch.from_numpy(0.5 * rng.random(N) + 0j).cuda()
        t = torch.from_numpy(rng.standard_normal(3 * N) + 1j * rng.standard_normal(3 * N)).cuda()
        return r, chi, t

    batches = [[sample() for _ in range(2)] for _ in range(5)]
    a = vie.Net(grid, seed=11)
    for bt in batches[:3]:
        a.train_step([s[0] for s in bt], [s[1] for s in bt], [s[2] for s in bt], lr=1e-3)
    path = str(tmp_path / "net.ck")
    learned.save_net(a, path, {"grid": list(grid), "seed": 11})
    la = [a.train_step([s[0] for s in bt], [s[1] for s in bt], [s[2] for s in bt], lr=1e-3) for bt in batches[3:]]
    b = vie.Net(grid, seed=99)                      # other initial weights, overwritten by the checkpoint
    assert learned.load_net(b, path) == {"grid": list(grid), "seed": 11}
    assert b.get_state()[3] == 3
    lb = [b.train_step([s[0] for s in bt], [s[1] for s in bt], [s[2] for s in bt], lr=1e-3) for bt in batches[3:]]
    print(la, lb)
    assert np.allclose(la, lb, rtol=1e-6, atol=0)
    wa, ma, va, sa = a.get_state()
    wb, mb, vb, sb = b.get_state()
    assert sa == sb == 5
    assert np.max(np.abs(wa - wb)) <= 1e-6 * np.max(np.abs(wa))
    # a state with a negative second moment is refused and leaves the network unchanged
    with pytest.raises(vie.VieError):
        b.set_state(wb, mb, -np.ones_like(vb), 5)
    assert np.array_equal(b.get_state()[0], wb)
