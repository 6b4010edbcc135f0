"""Training and evaluation driver for the learned preconditioner.

Every numerical step runs in libvie.so (matvecs, solves, network forward,
backward and Adam); this module only generates seeded random inputs, orders
the calls and records timings.

Training pairs for a geometry with contrast chi:
* operator pairs (A v, v): v a smooth random complex field on the support of
  chi (a spatial Gaussian filter of white noise), A v one FP64 product -- the
  network learns to undo the operator without any solve;
* solution pairs (b, x*): b from a dipole source, x* from the mixed-precision
  solver to 1e-8.
Each pair is rotated by a random global phase (the operator is complex linear;
the network is not, so phases are shown during training).
"""
from __future__ import annotations

import time
from typing import Dict, List, Sequence

import numpy as np

from . import inputs, vie


CHECKPOINT_FORMAT = "vie-unet-training-state"


def write_checkpoint(path: str, w: np.ndarray, m: np.ndarray, v: np.ndarray, step: int, meta: Dict = None):
    """Training checkpoint without pickling: one JSON header line (format, parameter
    count, Adam step, caller's metadata such as grid, seeds and learning rate), then
    the FP32 weights, Adam m and Adam v as raw little-endian float32."""
    import json
    n = int(np.asarray(w).size)
    parts = [np.ascontiguousarray(a, dtype="<f4").ravel() for a in (w, m, v)]
    if any(a.size != n for a in parts):
        raise ValueError("weights and moments differ in size")
    head = {"format": CHECKPOINT_FORMAT, "version": 1, "num_params": n, "step": int(step),
            "dtype": "float32-le", "parts": ["weights", "adam_m", "adam_v"], "meta": meta or {}}
    with open(path, "wb") as f:
        f.write((json.dumps(head, sort_keys=True) + "\n").encode())
        for a in parts:
            f.write(a.tobytes())


def read_checkpoint(path: str):
    """(weights, m, v, step, meta) of a file written by write_checkpoint; refuses other
    formats and files whose payload does not match the header."""
    import json
    with open(path, "rb") as f:
        head = json.loads(f.readline().decode())
        if head.get("format") != CHECKPOINT_FORMAT or head.get("version") != 1:
            raise ValueError("not a network training checkpoint")
        n = int(head["num_params"])
        raw = f.read()
    if len(raw) != 3 * 4 * n:
        raise ValueError(f"checkpoint payload is {len(raw)} bytes, the header needs {12 * n}")
    a = np.frombuffer(raw, dtype="<f4").astype(np.float32)
    return a[:n].copy(), a[n:2 * n].copy(), a[2 * n:].copy(), int(head["step"]), head["meta"]


def save_net(net: "vie.Net", path: str, meta: Dict = None):
    """Checkpoint a network's training state (vie_net_get_state)."""
    w, m, v, step = net.get_state()
    write_checkpoint(path, w, m, v, step, meta)


def load_net(net: "vie.Net", path: str) -> Dict:
    """Restore a network's training state from a checkpoint; returns its metadata."""
    w, m, v, step, meta = read_checkpoint(path)
    net.set_state(w, m, v, step)
    return meta


def smooth_field(shape, mask: np.ndarray, rng: np.random.Generator, width: float = 3.0) -> np.ndarray:
    """Complex white noise filtered by a spatial Gaussian of `width` voxels, masked to the support."""
    from scipy.ndimage import gaussian_filter
    z = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    sig = (0, width, width, width)
    z = gaussian_filter(z.real, sig) + 1j * gaussian_filter(z.imag, sig)
    return z * mask[None]


class Trainer:
    def __init__(self, grid: Sequence[int], h: float, seed: int = 0):
        import torch
        self.torch = torch
        self.grid = tuple(grid)
        self.h = h
        self.plan = vie.Plan(self.grid, h, inputs.K0, inputs.EPS_B, fp32=True)
        self.net = vie.Net(self.grid, seed=seed)
        self.rng = np.random.default_rng(seed)
        self.data: List[tuple] = []

    def add_geometry(self, wg: inputs.Waveguide, n_operator_pairs: int, n_solution_pairs: int = 0,
                     tol: float = 1e-8):
        torch = self.torch
        self.plan.set_contrast(torch.from_numpy(wg.eps()).cuda())
        chi = self.plan.contrast()
        mask = wg.core_mask()
        for _ in range(n_operator_pairs):
            v = torch.from_numpy(smooth_field((3,) + self.grid, mask, self.rng)).cuda()
            r = self.plan.matvec(v)
            ph = complex(np.exp(1j * self.rng.uniform(0, 2 * np.pi)))
            self.data.append((r * ph, chi, v * ph))
        for _ in range(n_solution_pairs):
            b = self.plan.rhs(torch.from_numpy(inputs.transverse_dipole_field(wg)).cuda())
            x, info = self.plan.solve(b, tol=tol, restart=50, precision=1)
            ph = complex(np.exp(1j * self.rng.uniform(0, 2 * np.pi)))
            self.data.append((b * ph, chi, x * ph))

    def train(self, epochs: int, lr: float = 1e-3, batch: int = 4, lr_decay: float = 0.7) -> List[float]:
        losses = []
        order = np.arange(len(self.data))
        for ep in range(epochs):
            self.rng.shuffle(order)
            for i in range(0, len(order), batch):
                sel = [self.data[j] for j in order[i:i + batch]]
                losses.append(self.net.train_step([s[0] for s in sel], [s[1] for s in sel], [s[2] for s in sel],
                                                  lr))
            lr *= lr_decay
        return losses


def compare_tiers(plan: "vie.Plan", net: "vie.Net", b, tol: float = 1e-8, restart: int = 50,
                  maxit: int = 20000) -> Dict[str, dict]:
    """Wall time and iterations to the tolerance for FP64 GMRES, mixed FGMRES and learned FGMRES."""
    import torch
    out = {}
    plan.set_preconditioner(net)
    for name, prec in (("fp64", 0), ("mixed", 1), ("learned", 2)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = plan.solve(b, tol=tol, restart=restart, maxit=maxit, precision=prec)
        torch.cuda.synchronize()
        info["wall"] = time.perf_counter() - t0
        r = plan.residual(x, b)
        info["rel_res_fp64"] = (torch.linalg.norm(r) / torch.linalg.norm(b)).item()
        out[name] = info
    return out


class CirculantCorrectionStudy:
    """The learned preconditioner as a correction of the block circulant W (Section V-D):
    z = W^{-1} v + net(v, W^{-1} v, chi), trained on pairs the method itself produces on
    seeded rough-sidewall guides (32 x 32 x 256).

    Training pair of geometry s: b = the dipole right-hand side of inputs.rough_strip(s),
    x* = its solution by circulant-preconditioned FGMRES to 1e-8, w = W^{-1} b; the
    network learns x* - w.  Every pair stays on the device (about 42 MB each)."""

    def __init__(self, seed: int = 0, n3: int = 256):
        import torch
        self.torch = torch
        wg = inputs.rough_strip(0, n3=n3)
        self.grid = wg.n
        self.plan = vie.Plan(self.grid, wg.h, wg.k0, wg.eps_b, fp32=True)
        self.net = vie.Net(self.grid, seed=seed)
        self.rng = np.random.default_rng(seed)
        self.n3 = n3
        self.pairs: List[tuple] = []
        self.gen_seconds = 0.0

    def _geometry(self, s: int):
        torch = self.torch
        wg = inputs.rough_strip(s, n3=self.n3)
        self.plan.set_contrast(torch.from_numpy(wg.eps()).cuda())
        self.plan.build_circulant()
        b = self.plan.rhs(torch.from_numpy(inputs.transverse_dipole_field(wg)).cuda())
        return wg, b

    def generate(self, seeds: Sequence[int], tol: float = 1e-8, n_operator: int = 0, progress=None) -> dict:
        """One solver-generated pair per training geometry, plus n_operator pairs
        (A u, u) per geometry with u a smooth random field on the contrast's support
        (Gaussian filter of 1 to 4 voxels), which resemble the vectors FGMRES hands the
        preconditioner more than a dipole right-hand side does."""
        torch = self.torch
        t0 = time.perf_counter()
        its = []
        for s in seeds:
            wg, b = self._geometry(s)
            x, info = self.plan.solve(b, tol=tol, restart=50, precision=3)
            if info["status"] != vie.VIE_OK:
                continue
            chi = self.plan.contrast()
            w = self.plan.apply_circulant(b)
            ph = complex(np.exp(1j * self.rng.uniform(0, 2 * np.pi)))
            self.pairs.append((b * ph, w * ph, chi, x * ph))
            its.append(info["iters"])
            if progress is not None and len(its) % 100 == 0:
                progress(f"{len(its)} geometries, {len(self.pairs)} pairs, "
                         f"{time.perf_counter() - t0:.1f} s")
            mask = wg.core_mask()
            for _ in range(n_operator):
                u = torch.from_numpy(smooth_field((3,) + self.grid, mask, self.rng,
                                                  width=float(self.rng.uniform(1.0, 4.0)))).cuda()
                v = self.plan.matvec(u)
                self.pairs.append((v, self.plan.apply_circulant(v), chi, u))
        torch.cuda.synchronize()
        self.gen_seconds += time.perf_counter() - t0
        return {"pairs": len(self.pairs), "seconds": round(time.perf_counter() - t0, 2),
                "circulant_iters_mean": float(np.mean(its)) if its else None}

    def train(self, epochs: int, lr: float = 1e-3, batch: int = 4, lr_decay: float = 0.8, progress=None) -> List[float]:
        losses = []
        order = np.arange(len(self.pairs))
        for _ in range(epochs):
            self.rng.shuffle(order)
            ep = []
            for i in range(0, len(order), batch):
                sel = [self.pairs[j] for j in order[i:i + batch]]
                ep.append(self.net.train_step_base([p[0] for p in sel], [p[1] for p in sel],
                                                   [p[2] for p in sel], [p[3] for p in sel], lr))
            losses.append(float(np.mean(ep)))
            if progress is not None:
                progress(f"epoch {len(losses)} loss {losses[-1]:.4f}")
            lr *= lr_decay
        return losses

    def evaluate(self, seeds: Sequence[int], tol: float = 1e-8, restart: int = 50, progress=None) -> dict:
        """Iterations and wall time to tol on unseen geometries: FP64 GMRES (0), mixed
        FGMRES (1), circulant FGMRES (3) and the network correcting the circulant (4);
        each tier's residual recomputed with the FP64 product."""
        torch = self.torch
        self.plan.set_preconditioner(self.net)
        rows = []
        for s in seeds:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, b = self._geometry(s)
            torch.cuda.synchronize()
            setup = time.perf_counter() - t0
            row = {"seed": int(s), "circulant_setup_seconds": round(setup, 4)}
            for name, prec in (("fp64", 0), ("mixed", 1), ("circulant", 3), ("learned_circulant", 4)):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                x, info = self.plan.solve(b, tol=tol, restart=restart, maxit=20000, precision=prec)
                torch.cuda.synchronize()
                wall = time.perf_counter() - t0
                r = self.plan.residual(x, b)
                row[name] = {"seconds": round(wall, 5), "iters": info["iters"], "applications": info["inner_iters"],
                             "fallback": info["fallback"], "status": info["status"],
                             "rel_res_fp64": (torch.linalg.norm(r) / torch.linalg.norm(b)).item()}
            rows.append(row)
            if progress is not None and len(rows) % 10 == 0:
                progress(f"{len(rows)} test geometries")
        self.plan.set_preconditioner(None)
        agg = {}
        for name in ("fp64", "mixed", "circulant", "learned_circulant"):
            agg[name] = {"seconds_mean": float(np.mean([r[name]["seconds"] for r in rows])),
                         "iters_mean": float(np.mean([r[name]["iters"] for r in rows])),
                         "max_rel_res_fp64": float(max(r[name]["rel_res_fp64"] for r in rows)),
                         "fallbacks": int(sum(r[name]["fallback"] for r in rows))}
        return {"per_seed": rows, "mean": agg}
