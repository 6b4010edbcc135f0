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


def mixed_vs_fp64(degrees: Sequence[int] = DEGREES, tol: float = 1e-8, ref_tol: float = 1e-10,
                  precision: int = 1) -> dict:
    """The mixed tier against FP64 on the 8 x 8 x 32 guide (h = 50 nm, 4 x 4 core, 8-voxel
    absorbers, sigma_max = 2, z-dipole where the lossless core starts), per absorber degree:
    relative L2 distance of the two solutions, and the reflection R of each against an FP64
    reference with 64-voxel absorbers (8 x 8 x 144, same cross-section, same source plane
    relative to the lossless part), R as in Section V-A over the lossless part.
    precision 1: inner GMRES with FP32 Krylov vectors; 5: with FP64 Krylov vectors."""
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
                x32, i32 = plan.solve(b, tol=tol, restart=50, precision=precision, inner_restart=20,
                                      inner_tol=1e-4)
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


# ---------------------------------------------------------------------------
# The strip study of Section V-A on the paper's own geometry (Section II-A).
# ---------------------------------------------------------------------------

STRIP_LENGTHS = tuple(round(0.45 * k, 2) for k in range(1, 22))    # 450 .. 9450 nm in steps of 450 nm
LAMBDA_SI = inputs.LAMBDA0 / math.sqrt(inputs.EPS_SI)                # wavelength in the core, um
# Absorber length (silicon wavelengths) for R = 1e-8 with electric currents only, as the
# paper's table of Section V-A gives it (d = 0 and some d = 1 entries are extrapolations there)
PAPER_LENGTH_FOR_1E8 = {1e-25: {0: 13000.0, 1: 49.0, 2: 9.5, 3: 7.2}, 1e-10: {0: 4500.0, 1: 32.0, 2: 7.1, 3: 6.2}}
# the same with electric and magnetic currents and an impedance-matched absorber
PAPER_LENGTH_FOR_1E8_EM = {1e-25: {0: 350.0, 1: 14.0, 2: 5.1, 3: 5.9}, 1e-10: {0: 230.0, 1: 9.0, 2: 4.8, 3: 6.1}}


def strip_axis_field(wg: inputs.Waveguide, w: np.ndarray) -> np.ndarray:
    """E over the lossless part of the strip's centre line (Section V-A measures on
    y = 250 nm, z = 100 nm, a corner shared by four voxel columns): the mean of those four
    columns, E = J / (eps_r - 1) with J = w h^{-3/2} (constants dropped).  Shape (3, length)."""
    i1, i2 = wg.n[0] // 2, wg.n[1] // 2
    lo, hi = wg.lossless_range()
    eps_r = wg.eps_core / wg.eps_b
    J = sum(w[:, a, b, lo:hi] for a in (i1 - 1, i1) for b in (i2 - 1, i2)) / 4.0
    return J / (wg.h ** 1.5 * (eps_r - 1.0))


def length_for_reflection(lengths: Sequence[float], R: Sequence[float], target: float = 1e-8):
    """Absorber length at which R(L) first falls to target: linear interpolation of log R
    against log L between the bracketing points; beyond the last point, the straight line
    through the last two points is extended (as the paper extrapolates some of its entries).
    None when R never decreases toward target."""
    L = np.log(np.asarray(lengths, dtype=float))
    y = np.log(np.maximum(np.asarray(R, dtype=float), 1e-300))
    t = math.log(target)
    for i in range(len(L)):
        if y[i] <= t:
            if i == 0:
                return float(lengths[0])
            f = (t - y[i - 1]) / (y[i] - y[i - 1])
            return float(math.exp(L[i - 1] + f * (L[i] - L[i - 1])))
    if len(L) >= 2 and y[-1] < y[-2]:
        slope = (y[-1] - y[-2]) / (L[-1] - L[-2])
        return float(math.exp(L[-1] + (t - y[-1]) / slope))
    return None


def analyse_reflection(lengths: Sequence[float], R: Sequence[float], d: int, r_rt: float, l_ref: float,
                       lam: float = LAMBDA_SI, target: float = 1e-8) -> dict:
    """Post-processing of one R(L) curve of Section V-A.  Points within a factor 2 of the
    reference length are left out (E(L) approaches the reference there, which steepens
    R artificially), as are points below ten times the floor max(R_rt, 1e-11) (the
    stagnation the paper describes).  From L >= 2 silicon wavelengths on, the log-log
    slope is fitted (predicted -2(d+1), Section IV-C).  The length giving R = target is
    interpolated where the kept curve crosses it, otherwise extrapolated from its last
    point with the fitted slope and, for comparison, with the predicted one (the paper
    extrapolates some of its entries).  Lengths are returned in silicon wavelengths."""
    L = np.asarray(lengths, dtype=float)
    R = np.asarray(R, dtype=float)
    keep = L <= l_ref / 2 + 1e-9
    Lk, Rk = L[keep], R[keep]
    fit = (Lk >= 2 * lam) & (Rk > 10 * max(r_rt, 1e-11))
    slope = float(np.polyfit(np.log(Lk[fit]), np.log(Rk[fit]), 1)[0]) if fit.sum() >= 2 else None
    out = {"slope": slope, "predicted_slope": -2 * (d + 1), "fit_points": int(fit.sum())}
    crossed = np.nonzero(Rk <= target)[0]
    if len(crossed):
        i = crossed[0] + 1
        out["length_lambda"] = length_for_reflection(Lk[:i], Rk[:i], target) / lam
        out["method"] = "interpolated"
        return out

    def extrapolate(s):
        if s is None or s >= 0:
            return None
        return float(Lk[-1] * math.exp((math.log(target) - math.log(Rk[-1])) / s)) / lam

    out["length_lambda"] = extrapolate(slope)
    out["length_lambda_predicted_slope"] = extrapolate(-2.0 * (d + 1))
    out["method"] = "extrapolated"
    return out


def _strip_guide(L: float, d: int, r_rt: float, strip_len: int, magnetic: bool) -> inputs.Waveguide:
    wg = inputs.strip_paper(L, d, r_rt, magnetic=magnetic)
    if strip_len != inputs.STRIP_LEN:
        wg = inputs.Waveguide(n=(wg.n[0], wg.n[1], strip_len + wg.n_abs), h=wg.h, core_x=wg.core_x,
                              core_y=wg.core_y, core_z=(0, strip_len + wg.n_abs), n_abs=wg.n_abs, d=d,
                              sigma_max=wg.sigma_max, ends="right", magnetic=magnetic)
    return wg


def _reflection(fields: dict, lengths: Sequence[float]):
    """R(L) = |E_ref - E_L|^2 / |E_ref|^2 on the centre line, against the longest absorber."""
    Lref = max(lengths)
    ref = fields[Lref]
    Ls = [L for L in lengths if L != Lref]
    return Ls, [float(np.sum(np.abs(ref - fields[L]) ** 2) / np.sum(np.abs(ref) ** 2)) for L in Ls]


def strip_reflection_study_em(r_rts: Sequence[float] = (1e-25, 1e-10), degrees: Sequence[int] = DEGREES,
                              lengths: Sequence[float] = STRIP_LENGTHS, precision: int = 1, tol: float = 1e-8,
                              restart: int = 50, inner_restart: int = 20, inner_tol: float = 1e-3,
                              strip_len: int = inputs.STRIP_LEN, progress=None) -> dict:
    """The e&m columns of Section V-A: the same strip, source and lengths, with magnetic
    conductivity matched to the electric one (mu'' = eps''/eps', strength with D = 4) and the
    JM-VIE solved for both currents (the source's eta H as the magnetic right-hand side).
    One plan at a time: each length's plan serves every (R_rt, d), then is freed.
    progress, if given, is called with a line per finished length."""
    import torch
    out = {"lengths_um": list(lengths), "lambda_si_um": LAMBDA_SI, "strip_voxels": strip_len, "runs": {},
           "formulation": "JM-VIE, impedance-matched absorber"}
    groups = [(r_rt, d) for r_rt in r_rts for d in degrees]
    fields = {g: {} for g in groups}
    stats = {g: {"solve_seconds": 0.0, "max_rel_res": 0.0, "outer_iters": [], "inner_iters": [], "status": 0,
                 "unknowns": 0} for g in groups}
    t_all = time.perf_counter()
    for L in lengths:
        t0 = time.perf_counter()
        wg0 = _strip_guide(L, degrees[0], r_rts[0], strip_len, True)
        plan = vie.Plan(wg0.n, wg0.h, wg0.k0, wg0.eps_b, fp32=precision != 0)
        try:
            plan.set_contrast(torch.from_numpy(wg0.eps()).cuda())
            plan.jm_enable()
            e_inc = torch.from_numpy(inputs.strip_paper_source(wg0)).cuda()
            h_inc = torch.from_numpy(inputs.strip_paper_source_h(wg0)).cuda()
            setup_s = time.perf_counter() - t0
            for g in groups:
                r_rt, d = g
                wg = _strip_guide(L, d, r_rt, strip_len, True)
                plan.set_contrast(torch.from_numpy(wg.eps()).cuda())
                plan.set_permeability(torch.from_numpy(wg.mu()).cuda())
                b = plan.jm_rhs(e_inc, h_inc)
                t1 = time.perf_counter()
                x, info = plan.jm_solve(b, tol=tol, restart=restart, precision=precision,
                                        inner_restart=inner_restart, inner_tol=inner_tol)
                torch.cuda.synchronize()
                st = stats[g]
                st["solve_seconds"] += time.perf_counter() - t1
                st["max_rel_res"] = max(st["max_rel_res"], info["rel_res_true"])
                st["outer_iters"].append(info["iters"])
                st["inner_iters"].append(info["inner_iters"])
                st["unknowns"] += 6 * wg.N
                if info["status"] != vie.VIE_OK:
                    st["status"] = info["status"]
                w = x.view((6,) + wg.n)[:3].cpu().numpy()
                fields[g][L] = strip_axis_field(wg, w)
        finally:
            plan.close()
        if progress is not None:
            progress(f"L = {L} um: {6 * wg0.N} unknowns, setup {setup_s:.1f} s, "
                     f"{len(groups)} JM solves in {time.perf_counter() - t0 - setup_s:.1f} s")
    out["seconds"] = round(time.perf_counter() - t_all, 3)
    for g in groups:
        r_rt, d = g
        Ls, R = _reflection(fields[g], lengths)
        run = dict(stats[g])
        run["solve_seconds"] = round(run["solve_seconds"], 3)
        run.update({"r_rt": r_rt, "d": d, "R": R,
                    "paper_length_for_1e-8_lambda": PAPER_LENGTH_FOR_1E8_EM.get(r_rt, {}).get(d)})
        run.update(analyse_reflection(Ls, R, d, r_rt, max(lengths)))
        out["runs"][f"{r_rt:g}/{d}"] = run
    return out


def strip_reflection_study(r_rts: Sequence[float] = (1e-25, 1e-10), degrees: Sequence[int] = DEGREES,
                           lengths: Sequence[float] = STRIP_LENGTHS, precision: int = 1, tol: float = 1e-8,
                           restart: int = 50, inner_restart: int = 20, inner_tol: float = 1e-3,
                           strip_len: int = inputs.STRIP_LEN, progress=None, keep: Sequence[float] = ()) -> dict:
    """Section V-A on the strip of Section II-A: for each round-trip reflection and profile
    degree, the guide with every absorber length is solved in one vie_solve_batch call
    (complex-source dipole, electric currents only); R(L) against the longest absorber on
    the centre line, the fitted log-log slope (predicted -2(d+1), Section IV-C) and the
    length that gives R = 1e-8 in silicon wavelengths (the paper's table).  The grid
    depends on L only, so one plan per length serves every (R_rt, d) with its own
    contrast.  progress, if given, is called with each finished run.  For the lengths in
    keep, each run also returns the guide and the solution (host arrays) under
    "solutions" {L: (guide, b, x)}, for checks outside the library."""
    import torch

    def guide(L, d, r_rt):
        return _strip_guide(L, d, r_rt, strip_len, False)

    Lref = max(lengths)
    out = {"lengths_um": list(lengths), "lambda_si_um": LAMBDA_SI, "strip_voxels": strip_len, "runs": {}}
    t0 = time.perf_counter()
    plans = {}
    for L in lengths:
        wg = guide(L, 0, r_rts[0])
        plans[L] = vie.Plan(wg.n, wg.h, wg.k0, wg.eps_b, fp32=True)
    out["plan_seconds"] = round(time.perf_counter() - t0, 3)
    try:
        for r_rt in r_rts:
            for d in degrees:
                t0 = time.perf_counter()
                wgs, bs = [], []
                for L in lengths:
                    wg = guide(L, d, r_rt)
                    plans[L].set_contrast(torch.from_numpy(wg.eps()).cuda())
                    bs.append(plans[L].rhs(torch.from_numpy(inputs.strip_paper_source(wg)).cuda()))
                    wgs.append(wg)
                torch.cuda.synchronize()
                setup_s = time.perf_counter() - t0
                t0 = time.perf_counter()
                xs, infos, code = vie.solve_batch([plans[L] for L in lengths], bs, tol=tol, restart=restart,
                                                  precision=precision, inner_restart=inner_restart,
                                                  inner_tol=inner_tol)
                torch.cuda.synchronize()
                solve_s = time.perf_counter() - t0
                fields = {L: strip_axis_field(wg, x.cpu().numpy()) for L, wg, x in zip(lengths, wgs, xs)}
                Ls, R = _reflection(fields, lengths)
                run = {"r_rt": r_rt, "d": d, "status": code, "setup_seconds": round(setup_s, 3),
                       "solve_seconds": round(solve_s, 3), "unknowns": sum(3 * wg.N for wg in wgs),
                       "max_rel_res": max(i["rel_res_true"] for i in infos),
                       "outer_iters": [i["iters"] for i in infos], "inner_iters": [i["inner_iters"] for i in infos],
                       "R": R, "paper_length_for_1e-8_lambda": PAPER_LENGTH_FOR_1E8.get(r_rt, {}).get(d)}
                run.update(analyse_reflection(Ls, R, d, r_rt, Lref))
                if keep:
                    run["solutions"] = {L: (wg, b.cpu().numpy(), x.cpu().numpy())
                                        for L, wg, b, x in zip(lengths, wgs, bs, xs) if L in keep}
                out["runs"][f"{r_rt:g}/{d}"] = run
                if progress is not None:
                    progress(run)
                del xs, bs
    finally:
        for p in plans.values():
            p.close()
    return out


def bragg_slice_field(plan: "vie.Plan", wg: inputs.Waveguide, w, e_inc: np.ndarray) -> np.ndarray:
    """Total E on the transmission slice of a Bragg guide from its solved currents w
    (device, 3N values), including the background voxels at the slice, where w is zero.

    The discrete system reads w = M (h^{3/2} e_inc + N w) (Section III-A), so
    f = h^{3/2} e_inc + N w is the field's Galerkin coefficient scaled by eps_r on
    every voxel and E = f / (h^{3/2} eps_r).  N w comes from one product with a
    uniform contrast of 1/2 (eps = 2 eps_b everywhere): y = w - N w / 2.  This
    replaces the plan's contrast.  Returns shape (3, n1, n2)."""
    import torch
    z = inputs.bragg_slice(wg)
    plan.set_contrast(torch.full(wg.n, 2.0 * wg.eps_b, dtype=torch.complex128, device="cuda"))
    y = plan.matvec(w)
    nw = (2.0 * (w - y))[..., z].cpu().numpy()
    eps_r = wg.eps()[..., z] / wg.eps_b
    return (wg.h ** 1.5 * e_inc[..., z] + nw) / (wg.h ** 1.5 * eps_r)[None]


def band_gap(wavelengths_nm: Sequence[float], T: Sequence[float]) -> dict:
    """Band gap read off a transmission curve: the wavelength of least transmission and
    the contiguous range around it where the transmission stays below half of the
    curve's maximum."""
    lam = np.asarray(wavelengths_nm, dtype=float)
    t = np.asarray(T, dtype=float) / max(T)
    i = int(np.argmin(t))
    out = {"lambda_min_nm": float(lam[i]), "T_min_over_max": float(t[i])}
    if t[i] < 0.5:
        lo, hi = i, i
        while lo > 0 and t[lo - 1] < 0.5:
            lo -= 1
        while hi < len(t) - 1 and t[hi + 1] < 0.5:
            hi += 1
        out.update(gap_lo_nm=float(lam[lo]), gap_hi_nm=float(lam[hi]), gap_width_nm=float(lam[hi] - lam[lo]),
                   gap_centre_nm=float(0.5 * (lam[lo] + lam[hi])), gap_open_at_range_end=bool(lo == 0 or hi == len(t) - 1))
    return out


def bragg_transmission(wavelengths_nm: Sequence[float], periods: int = 100, lead_periods: int = 10, d: int = 2,
                       r_rt: float = 1e-10, precision: int = 1, tol: float = 1e-8, restart: int = 50,
                       inner_restart: int = 20, inner_tol: float = 1e-3, batch: int = 8, progress=None,
                       circulant: bool = False) -> dict:
    """Transmission through the Bragg grating of Section II-B against the free-space
    wavelength (Section V): for each wavelength the guide with quadratic absorbers of
    2.2 um on both ends is solved for the strip's complex-source dipole, and
    T = sum over the slice's voxels of |E|^2 h^2 (the integral of |E|^2 over a
    voxel-wide cross-section between the grating and the far absorber).  Each
    wavelength has its own operator (k0 h changes), so every wavelength gets a plan;
    `batch` of them are solved together in one vie_solve_batch call.  circulant=True
    solves with the block-circulant preconditioner of each plan's contrast
    (precision 3; FP32 inverse blocks, 12.7 GB per plan on the full grating)."""
    import torch
    out = {"wavelengths_nm": [float(v) for v in wavelengths_nm], "periods": periods, "lead_periods": lead_periods,
           "d": d, "r_rt": r_rt, "T": [], "iters": [], "inner_iters": [], "rel_res": [], "status": [],
           "plan_seconds": 0.0, "solve_seconds": 0.0, "circulant": circulant}
    if circulant:
        precision = 3
    for c0 in range(0, len(wavelengths_nm), batch):
        lams = list(wavelengths_nm[c0:c0 + batch])
        t0 = time.perf_counter()
        wgs = [inputs.bragg_grating(lam * 1e-3, periods=periods, lead_periods=lead_periods, d=d, r_rt=r_rt)
               for lam in lams]
        plans = [vie.Plan(wg.n, wg.h, wg.k0, wg.eps_b, fp32=True) for wg in wgs]
        try:
            eincs, bs = [], []
            for wg, p in zip(wgs, plans):
                p.set_contrast(torch.from_numpy(wg.eps()).cuda())
                e = inputs.bragg_source(wg)
                eincs.append(e)
                bs.append(p.rhs(torch.from_numpy(e).cuda()))
                if circulant:
                    p.build_circulant()
            torch.cuda.synchronize()
            out["plan_seconds"] += time.perf_counter() - t0
            t0 = time.perf_counter()
            xs, infos, code = vie.solve_batch(plans, bs, tol=tol, restart=restart, precision=precision,
                                              inner_restart=inner_restart, inner_tol=inner_tol)
            torch.cuda.synchronize()
            out["solve_seconds"] += time.perf_counter() - t0
            for lam, wg, p, x, e, info in zip(lams, wgs, plans, xs, eincs, infos):
                E = bragg_slice_field(p, wg, x, e)
                out["T"].append(float(np.sum(np.abs(E) ** 2) * wg.h ** 2))
                out["iters"].append(info["iters"])
                out["inner_iters"].append(info["inner_iters"])
                out["rel_res"].append(info["rel_res_true"])
                out["status"].append(info["status"])
                if progress is not None:
                    progress(lam, out["T"][-1], info)
            del xs, bs
        finally:
            for p in plans:
                p.close()
    out["plan_seconds"] = round(out["plan_seconds"], 3)
    out["solve_seconds"] = round(out["solve_seconds"], 3)
    out["T_norm"] = [t / max(out["T"]) for t in out["T"]]
    out.update(band_gap(out["wavelengths_nm"], out["T"]))
    return out


def bragg_axis_field(wg: inputs.Waveguide, w: np.ndarray) -> np.ndarray:
    """E on the core's centre line (the voxel column through the grid's centre, inside
    the core over the whole length) over the lossless part: E = J / (eps_r - 1) with
    J = w h^{-3/2}.  Shape (3, length)."""
    i1, i2 = wg.n[0] // 2, wg.n[1] // 2
    lo, hi = wg.lossless_range()
    eps_r = wg.eps_core / wg.eps_b
    return w[:, i1, i2, lo:hi] / (wg.h ** 1.5 * (eps_r - 1.0))


def bragg_slow_light_study(wavelengths_nm: Sequence[float] = (1520.0, 1538.0),
                           absorber_periods: Sequence[int] = (3, 5, 10, 20, 40), ref_periods: int = 90,
                           d: int = 2, r_rt: float = 1e-10, precision: int = 1, tol: float = 1e-8,
                           restart: int = 50, inner_restart: int = 20, inner_tol: float = 1e-3,
                           progress=None) -> dict:
    """Absorbers inside the periodic region (Section V, slow light): R(L) on the centre
    line of the lossless part against a ref_periods absorber, for the corrugated
    guide and for the uniform strip of the same lengths, at each wavelength.  All
    lengths of one (wavelength, guide) are solved in one vie_solve_batch call
    (uneven grids)."""
    import torch
    lengths = list(absorber_periods) + [ref_periods]
    out = {"absorber_periods": list(absorber_periods), "ref_periods": ref_periods, "d": d, "r_rt": r_rt,
           "period_um": inputs.BRAGG_PERIOD * inputs.BRAGG_H, "runs": {}}
    for lam in wavelengths_nm:
        for corrugated in (True, False):
            t0 = time.perf_counter()
            wgs = [inputs.bragg_slow_light(lam * 1e-3, P, d=d, r_rt=r_rt, corrugated=corrugated) for P in lengths]
            plans = [vie.Plan(wg.n, wg.h, wg.k0, wg.eps_b, fp32=True) for wg in wgs]
            try:
                bs = []
                for wg, p in zip(wgs, plans):
                    p.set_contrast(torch.from_numpy(wg.eps()).cuda())
                    bs.append(p.rhs(torch.from_numpy(inputs.bragg_source(wg)).cuda()))
                torch.cuda.synchronize()
                setup_s = time.perf_counter() - t0
                t0 = time.perf_counter()
                xs, infos, code = vie.solve_batch(plans, bs, tol=tol, restart=restart, precision=precision,
                                                  inner_restart=inner_restart, inner_tol=inner_tol)
                torch.cuda.synchronize()
                solve_s = time.perf_counter() - t0
                fields = {P: bragg_axis_field(wg, x.cpu().numpy()) for P, wg, x in zip(lengths, wgs, xs)}
                del xs, bs
            finally:
                for p in plans:
                    p.close()
            Ls, R = _reflection(fields, lengths)
            fit = np.polyfit(np.log(np.asarray(Ls, float)), np.log(np.asarray(R)), 1)[0] if len(Ls) >= 2 else None
            run = {"lambda_nm": float(lam), "corrugated": corrugated, "status": code,
                   "setup_seconds": round(setup_s, 3), "solve_seconds": round(solve_s, 3),
                   "max_rel_res": max(i["rel_res_true"] for i in infos), "outer_iters": [i["iters"] for i in infos],
                   "R": R, "loglog_slope": None if fit is None else float(fit), "predicted_slope": -2 * (d + 1)}
            out["runs"][f"{lam:g}/{'grating' if corrugated else 'strip'}"] = run
            if progress is not None:
                progress(run)
    return out


def bragg_slow_light_spectrum(wavelengths_nm: Sequence[float], absorber_periods: int = 40, ref_periods: int = 90,
                              d: int = 2, r_rt: float = 1e-10, tol: float = 1e-8, progress=None) -> dict:
    """R against the free-space wavelength for an absorber inside the grating (Section
    V, slow light): at each wavelength the guide with an absorber of absorber_periods
    and the reference with ref_periods are solved (block-circulant preconditioned
    FGMRES) and R = |E_ref - E|^2 / |E_ref|^2 on the centre line of the lossless part."""
    import torch
    out = {"wavelengths_nm": [float(v) for v in wavelengths_nm], "absorber_periods": absorber_periods,
           "ref_periods": ref_periods, "d": d, "r_rt": r_rt, "R": [], "iters": [], "rel_res": [], "status": []}
    t0 = time.perf_counter()
    for lam in wavelengths_nm:
        fields, its, res, st = {}, [], [], []
        for P in (absorber_periods, ref_periods):
            wg = inputs.bragg_slow_light(lam * 1e-3, P, d=d, r_rt=r_rt)
            plan = vie.Plan(wg.n, wg.h, wg.k0, wg.eps_b, fp32=True)
            try:
                plan.set_contrast(torch.from_numpy(wg.eps()).cuda())
                b = plan.rhs(torch.from_numpy(inputs.bragg_source(wg)).cuda())
                plan.build_circulant()
                x, info = plan.solve(b, tol=tol, precision=3)
                fields[P] = bragg_axis_field(wg, x.cpu().numpy())
            finally:
                plan.close()
            its.append(info["iters"])
            res.append(info["rel_res_true"])
            st.append(info["status"])
        ref = fields[ref_periods]
        R = float(np.sum(np.abs(ref - fields[absorber_periods]) ** 2) / np.sum(np.abs(ref) ** 2))
        out["R"].append(R)
        out["iters"].append(its)
        out["rel_res"].append(max(res))
        out["status"].append(max(abs(v) for v in st))
        if progress is not None:
            progress(lam, R, its)
    out["seconds"] = round(time.perf_counter() - t0, 3)
    return out


if __name__ == "__main__":
    import argparse
    import json
    ap = argparse.ArgumentParser(description="experiments of the paper run on the GPU path")
    ap.add_argument("which", choices=["strip", "bragg", "slowlight", "learned"],
                    help="strip: the reflection study of Section V-A; bragg: the grating's transmission; "
                         "slowlight: absorbers inside the grating; learned: the network correcting the "
                         "block circulant on rough guides (train seeds 0.., test seeds 10000..)")
    ap.add_argument("--train", type=int, default=2000, help="learned: solver-generated training pairs")
    ap.add_argument("--test", type=int, default=100, help="learned: test geometries")
    ap.add_argument("--epochs", type=int, default=8, help="learned: training epochs")
    ap.add_argument("--operator-pairs", type=int, default=2, help="learned: (A u, u) pairs per training geometry")
    ap.add_argument("--out", default=None, help="write the JSON result here")
    ap.add_argument("--quick", action="store_true", help="every other absorber length")
    ap.add_argument("--em", action="store_true", help="electric and magnetic currents, matched absorber")
    ap.add_argument("--r-rt", type=float, nargs="*", default=[1e-25, 1e-10], help="round-trip reflections")
    ap.add_argument("--step", type=float, default=1.0, help="bragg: wavelength step in nm (1520..1570)")
    ap.add_argument("--periods", type=int, default=100, help="bragg: grating periods")
    ap.add_argument("--circulant", action="store_true", help="bragg: block-circulant preconditioned solves")
    a = ap.parse_args()
    if a.which == "learned":
        from . import learned
        st = learned.CirculantCorrectionStudy(seed=0)
        say = lambda m: print(m, flush=True)
        gen = st.generate(range(a.train), n_operator=a.operator_pairs, progress=say)
        print("generated", gen, flush=True)
        t0 = time.perf_counter()
        losses = st.train(a.epochs, progress=say)
        train_s = time.perf_counter() - t0
        print("losses", losses, "train s", round(train_s, 1), flush=True)
        ev = st.evaluate(range(10000, 10000 + a.test), progress=say)
        res = {"generate": gen, "epochs": a.epochs, "losses": losses, "train_seconds": round(train_s, 2),
               "test": ev["mean"], "per_seed": ev["per_seed"]}
        print(json.dumps(ev["mean"]), flush=True)
        if a.out:
            with open(a.out, "w") as f:
                f.write(json.dumps(res, indent=1))
        raise SystemExit(0)
    if a.which == "slowlight":
        res = bragg_slow_light_study(progress=lambda r: print(r, flush=True))
        res["spectrum"] = bragg_slow_light_spectrum(
            np.arange(1520.0, 1570.0 + 1e-9, a.step),
            progress=lambda lam, R, its: print(f"{lam:.1f} nm R {R:.3e} outer steps {its}", flush=True))
        if a.out:
            with open(a.out, "w") as f:
                f.write(json.dumps(res, indent=1))
        raise SystemExit(0)
    if a.which == "bragg":
        lams = np.arange(1520.0, 1570.0 + 1e-9, a.step)
        res = bragg_transmission(lams, periods=a.periods, circulant=a.circulant, batch=4 if a.circulant else 8,
                                 progress=lambda lam, T, i: print(f"{lam:.1f} nm T {T:.4e} iters {i['iters']}/"
                                                                  f"{i['inner_iters']} res {i['rel_res_true']:.1e}",
                                                                  flush=True))
        print({k: v for k, v in res.items() if not isinstance(v, list)}, flush=True)
        if a.out:
            with open(a.out, "w") as f:
                f.write(json.dumps(res, indent=1))
        raise SystemExit(0)
    lengths = STRIP_LENGTHS[::2] if a.quick else STRIP_LENGTHS
    if lengths[-1] != STRIP_LENGTHS[-1]:
        lengths = tuple(lengths) + (STRIP_LENGTHS[-1],)

    def show(r):
        def fmt(v):
            return None if v is None else round(v, 2)
        print(f"{r['r_rt']:g}/{r['d']}", "slope", fmt(r["slope"]), "pred", r["predicted_slope"],
              "L(1e-8)/lambda", fmt(r["length_lambda"]), r["method"], "paper", r["paper_length_for_1e-8_lambda"],
              "solve s", r["solve_seconds"], "max res", f"{r['max_rel_res']:.1e}", flush=True)

    if a.em:
        res = strip_reflection_study_em(r_rts=tuple(a.r_rt), lengths=lengths, progress=lambda m: print(m, flush=True))
        for r in res["runs"].values():
            show(r)
    else:
        res = strip_reflection_study(r_rts=tuple(a.r_rt), lengths=lengths, progress=show)
    if a.out:
        with open(a.out, "w") as f:
            f.write(json.dumps(res, indent=1))
