#!/usr/bin/env python3
"""Throughput of the voxel J-VIE hot path on one MI355X.

A step is one FP64 product y = (I - M_eps N) x on the 32 x 32 x 512 voxel
waveguide (1.57 M unknowns, h = 25 nm, 500 x 225 nm silicon core in silica,
quadratic absorbers of 2 um at both ends): forward z FFT, xy FFT with the fused
Green product, inverse z FFT with the fused contrast.  Inputs are resident in
HBM before the timed region.  After the timed steps the same operator is solved
to a relative residual of 1e-8 from a dipole source with FP64 GMRES(50) and with
the FP32-inner / FP64-outer flexible GMRES, and the oracle's FFT matvec is timed
on the host as the CPU baseline.  The JM-VIE products and the J-VIE product on
the paper's 30 x 12 x 1377 strip are timed beside it.  Unless skipped, the
64-system absorber family is solved as one batch (reflection slopes reported)
and the learned preconditioner is trained and compared on 32 x 32 x 256 rough
guides.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-solve] [--no-cpu]

Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "VIE matvecs/s + HBM %peak; time-to-1e-8 residual: mixed/learned vs FP64"


def pass_bytes(n, M, cs):
    """Algorithmic HBM bytes of the three passes for complex element size cs."""
    n1, n2, n3 = n
    M1, M2, M3 = M
    N = n1 * n2 * n3
    U = 3 * n1 * n2 * M3 * cs
    G = 6 * (M1 // 2 + 1) * (M2 // 2 + 1) * (M3 // 2 + 1) * cs
    return [3 * N * cs + U,                      # pass 1: read x, write U
            2 * U + G,                           # pass 2: read/write U, read spectrum octant
            U + 3 * N * cs + N * cs + 3 * N * cs]  # pass 3: read U, x, chi; write y


def jm_pass_bytes(n, M, cs, fused):
    """Algorithmic HBM bytes of the JM-VIE product (6N unknowns) per kernel: the z passes
    run once per half; the cross-section work is one fused kernel (spectra in LDS) or the
    forward transforms, the product and the inverse transforms through full spectra."""
    n1, n2, n3 = n
    M1, M2, M3 = M
    N = n1 * n2 * n3
    U = 3 * n1 * n2 * M3 * cs
    H = (M1 // 2 + 1) * (M2 // 2 + 1) * (M3 // 2 + 1)
    G, K = 6 * H * cs, 3 * H * cs
    S3 = 3 * M1 * M2 * M3 * cs
    z = {"z forward (x2)": 2 * (3 * N * cs + U), "z inverse (x2)": 2 * (U + 7 * N * cs)}
    if fused:
        z["k_jm_xy"] = 4 * U + G + K
    else:
        z["k_jm_xyfwd (x2)"] = 2 * (U + S3)
        z["k_jm_product"] = 4 * S3 + G + K
        z["k_jm_xyinv (x2)"] = 2 * (S3 + U)
    return z


def jm_measurement(steps: int):
    """JM-VIE products (Section III: electric and magnetic currents, 6N unknowns) timed
    with HIP events on the plan's stream: the bench guide with impedance-matched magnetic
    absorbers, and the paper's strip (30 x 12 x 1377, the longest absorber of the e&m study)."""
    import numpy as np
    import torch

    from paper_1803_06237_amd import inputs, vie
    wg_bench = inputs.strip_long(d=2)
    wg_bench.magnetic = True
    cases = (("32x32x512 guide, matched absorbers", wg_bench),
             ("30x12x1377 strip, matched 9.45 um absorber", inputs.strip_paper(9.45, 2, 1e-10, magnetic=True)))
    out = {}
    for name, wg in cases:
        plan = vie.Plan(wg.n, wg.h, wg.k0, wg.eps_b, fp32=True)
        plan.set_contrast(torch.from_numpy(wg.eps()).cuda())
        plan.jm_enable()
        plan.set_permeability(torch.from_numpy(wg.mu()).cuda())
        rng = np.random.default_rng(1)
        xh = rng.standard_normal(6 * wg.N) + 1j * rng.standard_normal(6 * wg.N)
        res = {"grid": list(wg.n), "unknowns": 6 * wg.N}
        for prec, label in ((0, "fp64"), (1, "fp32")):
            x = torch.from_numpy(xh).cuda()
            if prec:
                x = x.to(torch.complex64)
            y = torch.empty_like(x)
            f = plan.jm_matvec if prec == 0 else plan.jm_matvec_c64
            for _ in range(5):
                f(x, y)
            t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0.record()
            for _ in range(steps):
                f(x, y)
            t1.record()
            t1.synchronize()
            ms = t0.elapsed_time(t1) / steps
            fused = plan.jm_route(prec)
            by = jm_pass_bytes(wg.n, circulant(wg.n), 16 if prec == 0 else 8, fused)
            tot = sum(by.values())
            res[label] = {"avg_us": round(ms * 1e3, 2), "matvecs_per_s": round(1e3 / ms, 1),
                          "route": "fused" if fused else "through HBM", "modelled_bytes": tot,
                          "GBs": round(tot / (ms * 1e-3) / 1e9, 1),
                          "frac": round(tot / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "bytes_by_kernel": by}
        plan.close()
        out[name] = res
    return out


def strip_measurement(steps: int):
    """J-VIE products on the paper's strip with its longest absorber (30 x 12 x 1377,
    circulant 64 x 32 x 4096: generic cross-section pass, long z pencils), FP64 and
    FP32, timed with HIP events on the plan's stream after one device copy of a
    3N-value FP64 vector (counter calibration, bytes known)."""
    import numpy as np
    import torch

    from paper_1803_06237_amd import inputs, vie
    wg = inputs.strip_paper(9.45, 2)
    plan = vie.Plan(wg.n, wg.h, wg.k0, wg.eps_b, fp32=True)
    plan.set_contrast(torch.from_numpy(wg.eps()).cuda())
    rng = np.random.default_rng(2)
    x = torch.from_numpy(rng.standard_normal(3 * wg.N) + 1j * rng.standard_normal(3 * wg.N)).cuda()
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    M = circulant(wg.n)
    out = {"grid": list(wg.n), "circulant": list(M), "calibration_copy_bytes_each_way": 3 * wg.N * 16}
    for prec, label in ((0, "fp64"), (1, "fp32")):
        xx = x if prec == 0 else x.to(torch.complex64)
        yy = torch.empty_like(xx)
        f = plan.matvec if prec == 0 else plan.matvec_c64
        for _ in range(5):
            f(xx, yy)
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(steps):
            f(xx, yy)
        t1.record()
        t1.synchronize()
        ms = t0.elapsed_time(t1) / steps
        by = pass_bytes(wg.n, M, 16 if prec == 0 else 8)
        out[label] = {"avg_us": round(ms * 1e3, 2), "modelled_bytes": sum(by), "bytes_by_pass": by,
                      "frac": round(sum(by) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "tune": plan.tune(prec)}
    plan.close()
    return out


KERNEL_SOURCES = {
    "k_xy64<double, 0>": ["xy64.hip", "fft_device.hpp", "block_maps.hpp"],
    "k_xy64<double, 1>": ["xy64.hip", "fft_device.hpp", "block_maps.hpp"],
    "k_xy64<double, 2>": ["xy64.hip", "fft_device.hpp", "block_maps.hpp"],
    "k_zfwd4<double, 32, 32>": ["zpass.hip", "dft_reg.hpp", "fft_device.hpp", "block_maps.hpp"],
    "k_zinv4<double, 32, 32, 0>": ["zpass.hip", "dft_reg.hpp", "fft_device.hpp", "block_maps.hpp"],
}


def profiled_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/matvec_32x32x512_fp64.md), or None when the kernel's sources have
    changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "matvec_32x32x512_fp64.md")
    if kernel not in KERNEL_SOURCES or not os.path.exists(path):
        return None
    m = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        m.update(open(os.path.join(ROOT, "paper_1803_06237_amd", "csrc", f), "rb").read())
    digest = m.hexdigest()[:16]
    for line in open(path):
        if line.startswith(f"traffic_bytes {kernel} ="):
            val, sha = line.split("=", 1)[1].split(";")
            if sha.split("=")[1].strip() == digest:
                return int(float(val))
    return None


def circulant(n):
    out = []
    for v in n:
        m = 1
        while m < 2 * v - 1:
            m *= 2
        out.append(m)
    return tuple(out)


def cpu_baseline(n, seconds_budget=30.0):
    """The oracle's FFT matvec at the same grid, host cores, bounded sample."""
    import numpy as np

    from oracle import matvec as mv
    rng = np.random.default_rng(0)
    M = tuple(2 * v for v in n)
    spec = rng.standard_normal((6,) + M) + 1j * rng.standard_normal((6,) + M)
    chi = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x = rng.standard_normal((3,) + n) + 1j * rng.standard_normal((3,) + n)
    t0 = time.perf_counter()
    runs = 0
    while True:
        mv.matvec_fft(spec, chi, x)
        runs += 1
        el = time.perf_counter() - t0
        if el > seconds_budget / 2 or runs >= 3:
            break
    model, cores = host_cpu()
    return {"value": runs / el, "unit": "matvecs/s", "cores": 1, "kind": "oracle",
            "sample": f"{runs} oracle FFT matvec(s) at {n[0]}x{n[1]}x{n[2]} (own radix-2 FFT, numpy, "
                      f"one thread) with a synthetic spectrum of the full circulant shape; table build excluded; "
                      f"{el:.1f} s on {model}, {cores} cores available"}


def host_cpu():
    """Model name and the number of cores this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def cpu_protocol(repeats: int = 5):
    """The CPU baselines of the measurement plan: the oracle's own-FFT FP64 matvec (one
    thread) and the same matvec with scipy.fft on every host core, each the median of
    `repeats` runs after one warm-up, at 8x8x32, 32x32x256 and 32x32x512 (synthetic
    spectra of the circulant shape; table build excluded), and the oracle's GMRES(50) to
    a relative residual of 1e-8 on the 8x8x32 guide from its dipole source (oracle table,
    spectrum and solve).  Takes a few minutes; `bench.py --cpu-full`."""
    import statistics

    import numpy as np

    from oracle import green, matvec as mv, solve
    from paper_1803_06237_amd import inputs
    model, cores = host_cpu()
    out = {"cpu_model": model, "nproc": cores, "repeats": repeats, "matvec": {}}

    def med(f):
        f()
        ts = []
        for _ in range(repeats):
            t0 = time.perf_counter()
            f()
            ts.append(time.perf_counter() - t0)
        return statistics.median(ts)

    for n in ((8, 8, 32), (32, 32, 256), (32, 32, 512)):
        rng = np.random.default_rng(0)
        M = tuple(2 * v for v in n)
        spec = rng.standard_normal((6,) + M) + 1j * rng.standard_normal((6,) + M)
        chi = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        x = rng.standard_normal((3,) + n) + 1j * rng.standard_normal((3,) + n)
        t_or = med(lambda: mv.matvec_fft(spec, chi, x))
        t_sc = med(lambda: cpu_tuned_matvec(spec, chi, x, cores))
        out["matvec"]["x".join(map(str, n))] = {"oracle_seconds": round(t_or, 5), "oracle_matvecs_per_s":
                                                 round(1 / t_or, 4), "scipy_seconds": round(t_sc, 5),
                                                 "scipy_matvecs_per_s": round(1 / t_sc, 3)}
    wg = inputs.strip_small(d=2)
    kap = mv.kappa_of(wg.h, wg.k0, wg.eps_b)
    b = mv.rhs_from_field(wg.eps(), wg.eps_b, inputs.strip_small_dipole_rhs_field(wg), wg.h)
    holder = {}

    def gm():
        op = mv.Operator(green.green_table(wg.n, kap), mv.contrast(wg.eps(), wg.eps_b))
        holder["res"] = solve.gmres(op, b.ravel(), tol=1e-8, restart=50)
    t_gm = med(gm)
    res = holder["res"]
    info = res[1]
    out["gmres_8x8x32"] = {"seconds": round(t_gm, 4), "iterations": int(getattr(info, "iters", -1)),
                           "includes": "oracle Green table, spectrum and GMRES(50) to 1e-8"}
    return out


def cpu_tuned_matvec(spec, chi, x, workers):
    """The same FFT matvec with scipy.fft on `workers` threads (FP64): zero-padded 3-D
    transforms of the three components, the symmetric 3 x 3 product with the full
    spectrum (components xx, xy, xz, yy, yz, zz), inverse transforms, crop, contrast."""
    import numpy as np
    import scipy.fft as sf
    n = x.shape[1:]
    M = spec.shape[1:]
    X = sf.fftn(x, s=M, axes=(1, 2, 3), workers=workers)
    Y = np.empty_like(X)
    Y[0] = spec[0] * X[0] + spec[1] * X[1] + spec[2] * X[2]
    Y[1] = spec[1] * X[0] + spec[3] * X[1] + spec[4] * X[2]
    Y[2] = spec[2] * X[0] + spec[4] * X[1] + spec[5] * X[2]
    u = sf.ifftn(Y, axes=(1, 2, 3), workers=workers)[:, :n[0], :n[1], :n[2]]
    return x - chi[None] * u


def cpu_tuned_baseline(n, seconds_budget=10.0):
    """The FFT matvec on all host cores with scipy.fft (the tuned CPU baseline beside
    the oracle's own FFT), at the same grid, bounded sample."""
    import numpy as np
    workers = len(os.sched_getaffinity(0))
    rng = np.random.default_rng(0)
    M = tuple(2 * v for v in n)
    spec = rng.standard_normal((6,) + M) + 1j * rng.standard_normal((6,) + M)
    chi = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x = rng.standard_normal((3,) + n) + 1j * rng.standard_normal((3,) + n)
    cpu_tuned_matvec(spec, chi, x, workers)            # plans and page-in
    t0 = time.perf_counter()
    runs = 0
    while True:
        cpu_tuned_matvec(spec, chi, x, workers)
        runs += 1
        el = time.perf_counter() - t0
        if el > seconds_budget / 2 or runs >= 10:
            break
    return {"value": runs / el, "unit": "matvecs/s", "cores": workers, "kind": "scipy.fft",
            "sample": f"{runs} FFT matvec(s) at {n[0]}x{n[1]}x{n[2]} with scipy.fft on {workers} threads "
                      f"(products and contrast in numpy), synthetic spectrum of the full circulant shape; {el:.1f} s"}


# Forward FLOPs of one network application at grid n: 2 V_l 27 cin cout per 3x3x3 layer
# (padded channel counts, as the matrix cores compute them) plus the 1x1x1 output layer.
NN_LAYERS = [(27, 16, 16, 0), (27, 16, 16, 0), (27, 16, 32, 1), (27, 32, 32, 1), (27, 32, 48, 2), (27, 48, 48, 2),
             (27, 48, 64, 3), (27, 64, 64, 3), (27, 112, 48, 2), (27, 48, 48, 2), (27, 80, 32, 1), (27, 32, 32, 1),
             (27, 48, 16, 0), (27, 16, 16, 0), (1, 16, 16, 0)]


def nn_flops(n):
    V = n[0] * n[1] * n[2]
    return sum(2 * (V >> (3 * lev)) * t * ci * co for t, ci, co, lev in NN_LAYERS)


def nn_measurement(steps: int):
    """The learned network at 32x32x256: average application time (HIP events on the
    network's stream) and one training step, with the forward FLOP rate."""
    import numpy as np
    import torch

    from paper_1803_06237_amd import vie
    n = (32, 32, 256)
    s = torch.cuda.current_stream()
    net = vie.Net(n, seed=0)
    rng = np.random.default_rng(0)
    r = torch.from_numpy(rng.standard_normal((3,) + n) + 1j * rng.standard_normal((3,) + n)).cuda()
    chi = torch.from_numpy((rng.uniform(0, 1, n) < 0.2) * (0.8 + 0.1j)).cuda()
    w = torch.from_numpy(rng.standard_normal((3,) + n) + 1j * rng.standard_normal((3,) + n)).cuda()
    for _ in range(3):
        net.apply_base(r, w, chi)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(steps):
        net.apply_base(r, w, chi)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    net.train_step_base([r], [w], [chi], [r], 1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        net.train_step_base([r], [w], [chi], [r], 1e-4)
    torch.cuda.synchronize()
    tr = (time.perf_counter() - t0) / 3
    f = nn_flops(n)
    return {"grid": list(n), "apply_ms": round(ms, 4), "forward_gflop": round(f / 1e9, 2),
            "forward_tflops": round(f / (ms * 1e-3) / 1e12, 1), "train_step_ms": round(tr * 1e3, 2)}


def learned_comparison(n_train: int = 96, epochs: int = 3, n_test: int = 4):
    """The learned preconditioner as a correction of the block circulant on seeded rough
    guides (32x32x256): n_train solver-generated pairs (training seeds 0..), a few
    epochs, then time to 1e-8 on unseen guides (test seeds 10000..) for FP64 GMRES(50),
    mixed FGMRES, circulant FGMRES and the network correcting the circulant.  A reduced
    version of the study `python -m paper_1803_06237_amd.experiments learned` (2000
    pairs, 100 test guides)."""
    import numpy as np

    from paper_1803_06237_amd import learned
    t0 = time.perf_counter()
    st = learned.CirculantCorrectionStudy(seed=0)
    gen = st.generate(range(n_train))
    losses = st.train(epochs)
    train_s = time.perf_counter() - t0
    ev = st.evaluate(range(10000, 10000 + n_test))
    m = ev["mean"]
    return {"workload": "32x32x256 rough-sidewall guides (sigma 1 voxel, corr 8), quadratic 1 um absorbers; "
                        f"network correcting the block circulant, {gen['pairs']} solver-generated pairs, "
                        f"{epochs} epochs, {n_test} test guides",
            "generate_and_train_seconds": round(train_s, 2), "losses": [round(x, 4) for x in losses],
            "test_mean": m,
            "learned_circulant_speedup_vs_fp64": round(m["fp64"]["seconds_mean"] /
                                                       m["learned_circulant"]["seconds_mean"], 3),
            "learned_circulant_speedup_vs_circulant": round(m["circulant"]["seconds_mean"] /
                                                            m["learned_circulant"]["seconds_mean"], 3),
            "mixed_speedup_vs_fp64": round(m["fp64"]["seconds_mean"] / m["mixed"]["seconds_mean"], 3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-family", action="store_true", help="skip the 64-system absorber-family batch")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-preconditioner comparison")
    ap.add_argument("--cpu-full", action="store_true",
                    help="only the CPU baselines: medians of 5 runs at 8x8x32, 32x32x256, 32x32x512 and the "
                         "oracle's GMRES on 8x8x32 (a few minutes, no GPU)")
    ap.add_argument("--profile", action="store_true",
                    help="profiler run: one device copy of a vector (counter calibration, bytes known) and the "
                         "timed FP64 products only")
    ap.add_argument("--profile-jm", action="store_true",
                    help="profiler run: the JM-VIE products only (both grids, both precisions)")
    ap.add_argument("--profile-strip", action="store_true",
                    help="profiler run: J-VIE products on the paper's strip 30x12x1377 only (FP64, FP32)")
    ap.add_argument("--profile-nn", action="store_true",
                    help="profiler run: the learned network at 32x32x256 (applications and training steps)")
    args = ap.parse_args()
    if args.cpu_full:
        print(json.dumps({"cpu_protocol": cpu_protocol()}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the solver is single-GPU.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1803_06237_amd import inputs, vie
    torch.cuda.set_device(0)
    if args.profile_jm:
        print(json.dumps({"jm_matvec": jm_measurement(args.steps)}), flush=True)
        return
    if args.profile_strip:
        print(json.dumps({"strip_matvec": strip_measurement(args.steps)}), flush=True)
        return
    if args.profile_nn:
        print(json.dumps({"nn": nn_measurement(args.steps)}), flush=True)
        return
    wg = inputs.strip_long(d=2)
    n = wg.n
    M = circulant(n)
    t0 = time.perf_counter()
    plan = vie.Plan(n, wg.h, wg.k0, wg.eps_b, fp32=True)
    plan_s = time.perf_counter() - t0
    plan.set_contrast(torch.from_numpy(wg.eps()).cuda())
    rng = np.random.default_rng(0)
    xh = rng.standard_normal((3,) + n) + 1j * rng.standard_normal((3,) + n)
    x = torch.from_numpy(xh).cuda()
    y = torch.empty_like(x)
    if args.profile:
        y.copy_(x)        # calibration: reads and writes exactly 3N * 16 bytes
        torch.cuda.synchronize()
        args.no_solve = args.no_cpu = args.no_family = args.no_learned = True
    for _ in range(args.warmup):
        plan.matvec(x, y)
    torch.cuda.synchronize()
    # timed region: K FP64 products through the C ABI, nothing else on the stream
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.matvec(x, y)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_step = el / args.steps * 1e3
    value = args.steps / el
    # per-pass breakdown in a separate run: HIP events around each pass on the plan's stream
    pass_ms, tot_ms = plan.profile_matvec(x, y, args.steps, precision=0)
    torch.cuda.synchronize()

    b64 = pass_bytes(n, M, 16)
    z4 = M[2] in (512, 1024)
    tune64 = plan.tune(0)
    names = ["k_zfwd4<double, 32, 32>" if z4 else "k_zfwd<double>",
             f"k_xy64<double, {tune64['xy_variant']}>" if M[0] == 64 and M[1] == 64 else "k_xyg<double>",
             "k_zinv4<double, 32, 32, 0>" if z4 else "k_zinv<double, 0>"]
    dom = int(np.argmax(pass_ms))
    achieved = b64[dom] / (pass_ms[dom] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": profiled_traffic(names[dom]),
                "kernel": names[dom],
                "algorithmic_bytes": b64[dom], "avg_ms": round(pass_ms[dom], 5)}
    passes = {names[i]: {"avg_us": round(pass_ms[i] * 1e3, 2), "bytes": b64[i],
                         "GBs": round(b64[i] / (pass_ms[i] * 1e-3) / 1e9, 1)} for i in range(3)}
    matvec_bytes = sum(b64)

    # FP32 product (mixed tier inner operator)
    x32 = x.to(torch.complex64)
    y32 = torch.empty_like(x32)
    for _ in range(args.warmup):
        plan.matvec_c64(x32, y32)
    torch.cuda.synchronize()
    # back-to-back products as for FP64 (the per-pass run below adds events between passes)
    k32 = max(20, args.steps // 2)
    t0 = time.perf_counter()
    for _ in range(k32):
        plan.matvec_c64(x32, y32)
    torch.cuda.synchronize()
    t32 = (time.perf_counter() - t0) / k32 * 1e3
    p32, _ = plan.profile_matvec(x32, y32, k32, precision=1)
    b32 = pass_bytes(n, M, 8)

    out = {"metric": METRIC, "value": round(value, 2), "unit": "matvecs/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 5),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "32x32x512 voxel J-VIE matvec (1.57M unknowns), h=25nm, 20x9-voxel Si core "
                                  "in SiO2, quadratic absorbers 80 voxels each end, FP64",
                      "grid": list(n), "circulant": list(M), "unknowns": 3 * wg.N, "parallelism": "1 GPU"},
           "roofline": roofline,
           "matvec_hbm": {"modelled_bytes": matvec_bytes,
                          "GBs": round(matvec_bytes / (ms_step * 1e-3) / 1e9, 1),
                          "frac": round(matvec_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                          "event_timed_us": round(tot_ms * 1e3, 2)},
           "passes": passes,
           "launch_shapes": {"fp64": tune64, "fp32": plan.tune(1)},
           "fp32_matvec": {"matvecs_per_s": round(1e3 / t32, 1), "avg_us": round(t32 * 1e3, 2),
                           "GBs": round(sum(b32) / (t32 * 1e-3) / 1e9, 1),
                           "passes_us_event_timed": [round(v * 1e3, 2) for v in p32]},
           "plan_seconds": round(plan_s, 3)}

    if not args.profile:
        out["jm_matvec"] = jm_measurement(max(10, args.steps // 4))
        # the paper's strip (Section II-A, 9.45 um absorber): 64 x 32 cross-section pass
        sm = strip_measurement(max(10, args.steps // 4))
        out["strip_matvec"] = {"workload": "J-VIE product, strip 30x12x1377, circulant 64x32x4096",
                               **{k: sm[k] for k in ("fp64", "fp32")}}

    if not args.no_solve:
        e_inc = inputs.transverse_dipole_field(wg)
        b = plan.rhs(torch.from_numpy(e_inc).cuda())
        res = {}
        for name, prec in (("fp64_gmres50", 0), ("mixed_fgmres", 1), ("mixed_fgmres_fp64_inner_arnoldi", 5)):
            plan.solve(b, tol=1e-8, restart=50, maxit=200, precision=prec)   # warm (allocations)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            xs, info = plan.solve(b, tol=1e-8, restart=50, maxit=20000, precision=prec)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            its = info["iters"] + info["inner_iters"]
            res[name] = {"seconds": round(dt, 4), "outer_iters": info["iters"],
                         "inner_iters": info["inner_iters"], "rel_res_true_fp64": info["rel_res_true"],
                         "status": info["status"],
                         "unknown_iterations_per_s": round(3 * wg.N * its / dt, 1)}
        res["mixed_speedup_vs_fp64"] = round(res["fp64_gmres50"]["seconds"] / res["mixed_fgmres"]["seconds"], 3)
        res["mixed_fp64_inner_arnoldi_speedup_vs_fp64"] = round(
            res["fp64_gmres50"]["seconds"] / res["mixed_fgmres_fp64_inner_arnoldi"]["seconds"], 3)
        # block-circulant preconditioner (Section V-D): set-up timed apart from the solve
        plan.build_circulant()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cinfo = plan.build_circulant()
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        r = torch.randn_like(b)
        z = plan.apply_circulant(r)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(20):
            plan.apply_circulant(r, z)
        torch.cuda.synchronize()
        t_apply = (time.perf_counter() - t0) / 20
        plan.solve(b, tol=1e-8, restart=50, maxit=5, precision=3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xs, info = plan.solve(b, tol=1e-8, restart=50, maxit=20000, precision=3)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res["circulant_fgmres"] = {"seconds": round(dt, 4), "setup_seconds": round(t_setup, 4),
                                   "total_seconds": round(dt + t_setup, 4), "outer_iters": info["iters"],
                                   "rel_res_true_fp64": info["rel_res_true"], "status": info["status"],
                                   "block_size": cinfo["block_size"], "blocks": cinfo["blocks"],
                                   "inverse_bytes": cinfo["bytes"], "apply_ms": round(t_apply * 1e3, 4)}
        res["circulant_speedup_vs_fp64_incl_setup"] = round(res["fp64_gmres50"]["seconds"] / (dt + t_setup), 3)
        out["solve_to_1e-8"] = res
        from paper_1803_06237_amd import experiments
        out["iterations_vs_length"] = experiments.iterations_vs_length()
        out["mixed_vs_fp64_observables"] = experiments.mixed_vs_fp64()
        out["mixed_fp64_inner_arnoldi_vs_fp64_observables"] = experiments.mixed_vs_fp64(precision=5)

    if not args.no_family:
        from paper_1803_06237_amd import experiments
        fam = experiments.run_family(precision=1, restart=30)
        out["batched_family"] = {
            "workload": "64 systems, 32x32x{192,256,320,512,832}, absorbers L in {0.5,1,2,4,8} um x d in 0..3, "
                        "20 dipole + 44 Gaussian rhs, FP32-inner/FP64-outer FGMRES, one vie_solve_batch call",
            "solve_seconds": round(fam["solve_seconds"], 3), "plan_seconds": round(fam["plan_seconds"], 3),
            "unknowns_total": fam["unknowns"], "max_rel_res_fp64": fam["max_rel_res"],
            "reflection_slopes": fam["slopes"], "predicted_slopes": {str(d): -2 * (d + 1) for d in range(4)},
            "reflection": fam["reflection"]}
        famc = experiments.run_family(precision=3, restart=30)
        out["batched_family_circulant"] = {
            "workload": "the same 64 systems, FP64 FGMRES preconditioned by each plan's block circulant",
            "solve_seconds": round(famc["solve_seconds"], 3),
            "preconditioner_seconds": round(famc["preconditioner_seconds"], 3),
            "max_rel_res_fp64": famc["max_rel_res"], "max_outer_iters": max(famc["outer_iters"]),
            "reflection_slopes": famc["slopes"],
            "speedup_vs_mixed_incl_setup": round(fam["solve_seconds"] /
                                                 (famc["solve_seconds"] + famc["preconditioner_seconds"]), 3)}

    if not args.no_learned:
        out["learned_preconditioner"] = learned_comparison()

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(n)
        out["cpu_tuned"] = cpu_tuned_baseline(n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
