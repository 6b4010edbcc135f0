"""The absorber-length family solved as one batch, and its reflection curve.

Section IV-C predicts that the transition reflection of a monomial absorber of
degree d falls as O(L^{-2(d+1)}) with its length L (coupled-mode argument), and
Section V-A measures it as R = ||E_inf - E_L||^2 / ||E_inf||^2 on the core axis
over the lossless part, with the longest absorber as reference.  This module
builds that family on synthetic 32 x 32 x n3 guides (h = 25 nm, 20 x 9 core),
solves all right-hand sides in one vie_solve_batch call and evaluates R(L).

All solver arithmetic runs in libvie.so; the reflection is post-processing of
the returned currents on the host.
"""
from __future__ import annotations

import itertools
import math
import time
from typing import Dict, List, Sequence

import numpy as np

from . import inputs, vie

LENGTHS = (0.5, 1.0, 2.0, 4.0, 8.0)   # um
DEGREES = (0, 1, 2, 3)


def family(lengths: Sequence[float] = LENGTHS, degrees: Sequence[int] = DEGREES, n_gauss: int = 44,
           r_rt: float = 1e-10):
    """(waveguide, kind, seed) for the dipole solves of every (L, d) and n_gauss seeded Gaussian
    right-hand sides spread over the combinations."""
    combos = list(itertools.product(lengths, degrees))
    items = [(inputs.strip_family(L, d, r_rt=r_rt), "dipole", 0, (L, d)) for L, d in combos]
    for s in range(n_gauss):
        L, d = combos[s % len(combos)]
        items.append((inputs.strip_family(L, d, r_rt=r_rt), "gauss", s, (L, d)))
    return items


def axis_field(wg: inputs.Waveguide, w: np.ndarray) -> np.ndarray:
    """E on the core's centre line over the lossless part: J = c_e (eps_r - 1) E with
    J = w h^{-3/2} on a voxel (constants dropped).  Shape (3, length)."""
    i1, i2 = wg.core_axis()
    z0 = wg.core_z[0] + wg.n_abs
    z1 = wg.core_z[1] - wg.n_abs
    eps_r = wg.eps()[i1, i2, z0:z1] / wg.eps_b
    return w[:, i1, i2, z0:z1] / (wg.h ** 1.5 * (eps_r - 1.0))[None]


def reflection_curve(fields: Dict[tuple, np.ndarray], lengths: Sequence[float] = LENGTHS,
                     degrees: Sequence[int] = DEGREES) -> Dict[int, List[float]]:
    """R(L) per degree, reference = the longest absorber."""
    out = {}
    Lref = max(lengths)
    for d in degrees:
        ref = fields[(Lref, d)]
        out[d] = [float(np.sum(np.abs(ref - fields[(L, d)]) ** 2) / np.sum(np.abs(ref) ** 2))
                  for L in lengths if L != Lref]
    return out


def fitted_slopes(curve: Dict[int, List[float]], lengths: Sequence[float], floor: float) -> Dict[int, float]:
    """Least-squares slope of log R vs log L, dropping points within 10x of the floor."""
    Ls = [L for L in lengths if L != max(lengths)]
    out = {}
    for d, R in curve.items():
        pts = [(np.log(L), np.log(r)) for L, r in zip(Ls, R) if r > 10 * floor]
        if len(pts) >= 2:
            x, y = np.array(pts).T
            out[d] = float(np.polyfit(x, y, 1)[0])
    return out


def run_family(precision: int = 1, tol: float = 1e-8, restart: int = 50, inner_restart: int = 20,
               inner_tol: float = 1e-3, n_gauss: int = 44, use_graph: bool = True) -> dict:
    """Build the 64 systems (plans shared per (L, d)), solve them in one batch, return timings,
    per-system info and the reflection curve of the dipole solves.  precision 3 builds each
    plan's block-circulant preconditioner first (timed apart)."""
    import torch
    items = family(n_gauss=n_gauss)
    plans: Dict[tuple, vie.Plan] = {}
    t0 = time.perf_counter()
    for wg, kind, seed, key in items:
        if key not in plans:
            p = vie.Plan(wg.n, wg.h, wg.k0, wg.eps_b, fp32=True)
            p.set_contrast(torch.from_numpy(wg.eps()).cuda())
            plans[key] = p
    plan_s = time.perf_counter() - t0
    precond_s = 0.0
    if precision == 3:
        t0 = time.perf_counter()
        for p in plans.values():
            p.build_circulant()
        precond_s = time.perf_counter() - t0
    bs, ps = [], []
    for wg, kind, seed, key in items:
        p = plans[key]
        if kind == "dipole":
            b = p.rhs(torch.from_numpy(inputs.transverse_dipole_field(wg)).cuda())
        else:
            b = torch.from_numpy(inputs.gaussian_rhs(wg.n, seed)).cuda()
        bs.append(b)
        ps.append(p)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xs, infos, code = vie.solve_batch(ps, bs, tol=tol, restart=restart, precision=precision,
                                      inner_restart=inner_restart, inner_tol=inner_tol, use_graph=use_graph)
    torch.cuda.synchronize()
    solve_s = time.perf_counter() - t0
    fields = {}
    for (wg, kind, seed, key), x in zip(items, xs):
        if kind == "dipole":
            fields[key] = axis_field(wg, x.cpu().numpy())
    curve = reflection_curve(fields)
    slopes = fitted_slopes(curve, LENGTHS, floor=1e-10)
    unknowns = sum(3 * wg.N for wg, _, _, _ in items)
    return {"status": code, "systems": len(items), "plan_seconds": plan_s, "solve_seconds": solve_s,
            "preconditioner_seconds": precond_s,
            "unknowns": unknowns, "grids": sorted({wg.n[2] for wg, _, _, _ in items}),
            "max_rel_res": max(i["rel_res_true"] for i in infos),
            "outer_iters": [i["iters"] for i in infos], "inner_iters": [i["inner_iters"] for i in infos],
            "reflection": {str(d): v for d, v in curve.items()}, "slopes": {str(d): v for d, v in slopes.items()},
            "lengths": list(LENGTHS)}


def iterations_vs_length(n3s: Sequence[int] = (128, 256, 512, 1024), d: int = 2, tol: float = 1e-8,
                         restart: int = 50) -> dict:
    """GMRES iterations to tol with and without the block-circulant preconditioner for
    straight guides of growing length (Section V-D: unpreconditioned counts grow with
    the length, preconditioned counts stay flat).  32 x 32 x n3 guides, h = 25 nm,
    80-voxel absorbers of degree d, x-dipole source."""
    import torch
    out = {"n3": list(n3s), "length_um": [], "plain_iters": [], "circulant_iters": [], "plain_seconds": [],
           "circulant_solve_seconds": [], "circulant_setup_seconds": []}
    for n3 in n3s:
        wg = inputs.strip_long(d=d, n3=n3)
        plan = vie.Plan(wg.n, wg.h, wg.k0, wg.eps_b, fp32=True)
        plan.set_contrast(torch.from_numpy(wg.eps()).cuda())
        b = plan.rhs(torch.from_numpy(inputs.transverse_dipole_field(wg)).cuda())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, i0 = plan.solve(b, tol=tol, restart=restart, precision=0)
        t_plain = time.perf_counter() - t0
        t0 = time.perf_counter()
        plan.build_circulant()
        t_setup = time.perf_counter() - t0
        t0 = time.perf_counter()
        _, i3 = plan.solve(b, tol=tol, restart=restart, precision=3)
        t_circ = time.perf_counter() - t0
        if i0["status"] != 0 or i3["status"] != 0:
            raise RuntimeError(f"solve did not converge at n3={n3}: {i0} {i3}")
        out["length_um"].append(round(n3 * wg.h, 3))
        out["plain_iters"].append(i0["iters"])
        out["circulant_iters"].append(i3["iters"])
        out["plain_seconds"].append(round(t_plain, 4))
        out["circulant_solve_seconds"].append(round(t_circ, 4))
        out["circulant_setup_seconds"].append(round(t_setup, 4))
        plan.close()
    return out


def mixed_vs_fp64(degrees: Sequence[int] = DEGREES, tol: float = 1e-8, ref_tol: float = 1e-10) -> dict:
    """The mixed tier against FP64 on the 8 x 8 x 32 guide (h = 50 nm, 4 x 4 core, 8-voxel
    absorbers, sigma_max = 2, z-dipole where the lossless core starts), per absorber degree:
    relative L2 distance of the two solutions, and the reflection R of each against an FP64
    reference with 64-voxel absorbers (8 x 8 x 144, same cross-section, same source plane
    relative to the lossless part), R as in Section V-A over the lossless part."""
    import torch
    out = {"degrees": list(degrees), "rel_l2": [], "R_fp64": [], "R_mixed": [], "rel_dR": [],
           "rel_res_fp64": [], "rel_res_mixed": [], "inner_iters": []}
    for d in degrees:
        wg = inputs.strip_small(d=d)
        ref = inputs.Waveguide(n=(8, 8, 144), h=wg.h, core_x=wg.core_x, core_y=wg.core_y, core_z=(0, 144),
                               n_abs=64, d=d, sigma_max=wg.sigma_max)
        kb = wg.k0 * math.sqrt(wg.eps_b)
        fields = {}
        for name, g in (("ref", ref), ("short", wg)):
            plan = vie.Plan(g.n, g.h, g.k0, g.eps_b, fp32=True)
            plan.set_contrast(torch.from_numpy(g.eps()).cuda())
            r0 = (g.h * 4, g.h * 4, g.h * g.n_abs)
            e = inputs.dipole_field(g.n, g.h, r0, (0, 0, 1), kb)
            b = plan.rhs(torch.from_numpy(e).cuda())
            if name == "ref":
                x, info = plan.solve(b, tol=ref_tol, restart=200, precision=0)
                fields["ref"] = axis_field(g, x.cpu().numpy())
            else:
                x64, i64 = plan.solve(b, tol=tol, restart=50, precision=0)
                x32, i32 = plan.solve(b, tol=tol, restart=50, precision=1, inner_restart=20, inner_tol=1e-4)
                a64, a32 = x64.cpu().numpy(), x32.cpu().numpy()
                out["rel_l2"].append(float(np.linalg.norm(a32 - a64) / np.linalg.norm(a64)))
                out["rel_res_fp64"].append(i64["rel_res_true"])
                out["rel_res_mixed"].append(i32["rel_res_true"])
                out["inner_iters"].append(i32["inner_iters"])
                fields["fp64"] = axis_field(g, a64)
                fields["mixed"] = axis_field(g, a32)
            plan.close()
        Eref = fields["ref"]
        R = {k: float(np.sum(np.abs(Eref - fields[k]) ** 2) / np.sum(np.abs(Eref) ** 2)) for k in ("fp64", "mixed")}
        out["R_fp64"].append(R["fp64"])
        out["R_mixed"].append(R["mixed"])
        out["rel_dR"].append(abs(R["mixed"] - R["fp64"]) / R["fp64"])
    return out
