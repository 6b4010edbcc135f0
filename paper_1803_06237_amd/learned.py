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
