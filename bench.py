"""Benchmark of the gfx950 MFM hydro pass.

    python bench.py [--steps K] [--warmup W] [--workload clustered|turbulence|shock_tube|...]
    python bench.py --copy-probe        # plain device copy of known size (counter calibration)
    python bench.py --adjoint-only      # forward + adjoint of 10 steps on the 64^3 box only

Metric: unordered particle-pair interactions per second per hydro pass (kernel
length + gradients + fluxes on particles already in the library's spatial
order), FP64, with the mixed form and its per-field error beside it, the
finite-volume (MFV) form of the same pass, and the forward + adjoint time of
10 fixed-dt steps on the 64^3 jittered box.

Inputs are seeded synthetic particle sets resident in HBM before timing starts.
Every timed pass starts the kernel-length solve cold (H = 0), so each step
redoes all of the pass's work.  Stage times come from HIP events on the stream
the library launches on; the dominant kernel's own duration comes from the
library's per-kernel event pairs (mfm_set_kernel_timing), which bracket that
kernel alone on the same stream.  Prints one JSON line on stdout.
"""
from __future__ import annotations

import argparse
import contextlib
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-pair interactions/s per hydro pass, FP64 vs mixed at stated error; fwd+adj time"

PEAK_HBM = 8.0e12          # B/s, MI355X HBM3E
# Vector peaks from the unit counts: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA)
# x 2.4 GHz = 78.6 TFLOP/s FP64; FP32 twice that with packed FP32 instructions.
PEAK_FP64_VALU = 78.6e12   # flop/s, FP64 vector
PEAK_FP32_VALU = 157.3e12  # flop/s, FP32 vector (packed)

# Algorithmic work per unit, the per-unit figures of the hot-path scope's
# measurement section: each particle's inputs read once and outputs written
# once (neighbour data are re-reads and not counted).  n particles, G gather
# entries (self excluded), F directed flux-list entries (= 2 pairs), P
# unordered pairs, I mean kernel-length iterations per particle.
#   solve_h:   48 B per particle (x 24 B in; H, n, V 24 B out); 20 flops per
#              gather neighbour per Newton iteration.
#   gradients: 264 B per particle (x, H, V, m, v, u in; B, rho, P and the five
#              gradients out); 65 flops per gather neighbour.
#   fluxes:    288 B per particle (the gradient outputs, x, H, V and v in; dp,
#              dE, vsig out); 400 flops per unordered pair (two sqrt, ~3 div).
#   fluxes, finite-volume form: dm (8 B) more out, and the full HLLC flux of the
#              selected side and the lab-frame boost add ~75 flops per pair.
# The neighbour-list indices the implementation reads (4 B per gather or flux
# entry) are reported separately as list_bytes.
def algorithmic(kernel, n, G, F, P, iters=5.0):
    """(bytes, flops, list_bytes) per launch."""
    if kernel == "solve_h":
        return 48.0 * n, 20.0 * G * iters, 4.0 * G
    if kernel == "gradients":
        return 264.0 * n, 65.0 * G, 4.0 * F
    if kernel == "hydro_fluxes":
        return 288.0 * n, 400.0 * P, 4.0 * F
    if kernel == "hydro_fluxes_mfv":
        return 296.0 * n, 475.0 * P, 4.0 * F
    raise KeyError(kernel)


def binding(frac_hbm, frac_alu):
    """The roof a kernel is closer to at its algorithmic counts."""
    return "alu" if frac_alu >= frac_hbm else "hbm"


KERNEL_NAMES = {"solve_h": "k_solve_h<false> + k_solve_h_wave + k_solve_h_fallback",
                "gradients": "k_gradients<false, false>", "hydro_fluxes": "k_fluxes_f64"}
KERNEL_SOURCES = ("paper_1712_01294_amd/csrc/pass.hip", "paper_1712_01294_amd/csrc/device.h",
                  "paper_1712_01294_amd/csrc/kernels.h")

# HBM traffic per launch from rocprofv3 FETCH_SIZE and WRITE_SIZE passes over
# this benchmark, scaled by what the same counters read for plain copies of
# known size (bench.py --copy-probe).  Keyed by workload and kernel, and valid
# only for the kernel sources whose fingerprint is recorded with it.
TRAFFIC = {
    ("clustered", "solve_h"): {"bytes_per_launch": 1.2331e+11, "fingerprint": "4d9f0a385d8119e7"},
    ("clustered", "gradients"): {"bytes_per_launch": 3.0494e+10, "fingerprint": "4d9f0a385d8119e7"},
    ("clustered", "hydro_fluxes"): {"bytes_per_launch": 1.3791e+10, "fingerprint": "4d9f0a385d8119e7"},
    ("clustered", "solve_h_mixed"): {"bytes_per_launch": 1.2331e+11, "fingerprint": "4d9f0a385d8119e7"},
    ("clustered", "gradients_mixed"): {"bytes_per_launch": 2.7638e+10, "fingerprint": "4d9f0a385d8119e7"},
    ("clustered", "hydro_fluxes_mixed"): {"bytes_per_launch": 1.5502e+10, "fingerprint": "4d9f0a385d8119e7"},
    ("clustered", "hydro_fluxes_mfv"): {"bytes_per_launch": 1.4172e+10, "fingerprint": "4d9f0a385d8119e7"},
    ("clustered", "hydro_fluxes_mfv_mixed"): {"bytes_per_launch": 1.5410e+10, "fingerprint": "4d9f0a385d8119e7"},
}

# VALU counters per launch from rocprofv3 --pmc passes over this benchmark:
# executed FP64 and FP32 flops (SQ_INSTS_VALU_FLOPS_FP64/FP32), VALU busy
# percentage (SQ_ACTIVE_INST_VALU over GRBM_GUI_ACTIVE, 256 CUs) and VALU
# instructions issued.  Keyed and fingerprinted like TRAFFIC.
COUNTERS = {
    ("clustered", "solve_h"): {"valu_busy_pct": 70.6, "fp64_flops_per_launch": 7.3894e+11, "fp32_flops_per_launch": 6.2724e+09, "valu_insts_per_launch": 1.7271e+10, "fingerprint": "4d9f0a385d8119e7"},
    ("clustered", "gradients"): {"valu_busy_pct": 27.7, "fp64_flops_per_launch": 1.0868e+11, "fp32_flops_per_launch": 0.0000e+00, "valu_insts_per_launch": 2.1952e+09, "fingerprint": "4d9f0a385d8119e7"},
    ("clustered", "hydro_fluxes"): {"valu_busy_pct": 52.4, "fp64_flops_per_launch": 3.6667e+11, "fp32_flops_per_launch": 0.0000e+00, "valu_insts_per_launch": 5.7054e+09, "fingerprint": "4d9f0a385d8119e7"},
    ("clustered", "solve_h_mixed"): {"valu_busy_pct": 70.6, "fp64_flops_per_launch": 7.3894e+11, "fp32_flops_per_launch": 6.2724e+09, "valu_insts_per_launch": 1.7271e+10, "fingerprint": "4d9f0a385d8119e7"},
    ("clustered", "gradients_mixed"): {"valu_busy_pct": 30.1, "fp64_flops_per_launch": 9.3961e+10, "fp32_flops_per_launch": 1.4820e+10, "valu_insts_per_launch": 2.2503e+09, "fingerprint": "4d9f0a385d8119e7"},
    ("clustered", "hydro_fluxes_mixed"): {"valu_busy_pct": 77.4, "fp64_flops_per_launch": 6.8311e+10, "fp32_flops_per_launch": 2.7785e+11, "valu_insts_per_launch": 5.8521e+09, "fingerprint": "4d9f0a385d8119e7"},
    ("clustered", "hydro_fluxes_mfv"): {"valu_busy_pct": 61.8, "fp64_flops_per_launch": 4.8855e+11, "fp32_flops_per_launch": 0.0000e+00, "valu_insts_per_launch": 7.2402e+09, "fingerprint": "4d9f0a385d8119e7"},
    ("clustered", "hydro_fluxes_mfv_mixed"): {"valu_busy_pct": 95.6, "fp64_flops_per_launch": 7.0260e+10, "fp32_flops_per_launch": 3.9681e+11, "valu_insts_per_launch": 7.3923e+09, "fingerprint": "4d9f0a385d8119e7"},
}


def source_fingerprint():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="clustered")
    ap.add_argument("--tree-levels", type=int, default=0)
    ap.add_argument("--max-ngb", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-mfv", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-limited", action="store_true")
    ap.add_argument("--no-hier", action="store_true")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only the forward + adjoint timing of 10 steps on the 64^3 box")
    ap.add_argument("--hier-only", action="store_true",
                    help="only the timing of hierarchical steps with active subsets on the workload")
    return ap.parse_args()


def copy_probe():
    """Counter calibration: five plain copies of a 1 GiB device buffer by the
    runtime's copy kernel, then five by a PyTorch elementwise kernel (b = a * 1):
    each launch fetches 1 GiB and writes 1 GiB."""
    import torch
    nbytes = 1 << 30
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    for _ in range(5):
        torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_per_launch": nbytes, "launches": 5,
                      "kernels": ["__amd_rocclr_copyBuffer", "elementwise mul"]}), flush=True)


def copy_ceiling(stream):
    """Measured HBM ceiling: a 1 GiB device-to-device copy (1 GiB read, 1 GiB
    written per launch), best of the copy and an elementwise kernel, median of
    five launches each, timed with HIP events on the stream."""
    import torch
    nbytes = 1 << 30
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    best = 0.0
    for op in (lambda: b.copy_(a), lambda: torch.mul(a, 1.0, out=b)):
        op()
        ts = []
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            op()
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e-3)
        best = max(best, 2.0 * nbytes / float(np.median(ts)))
    del a, b
    torch.cuda.empty_cache()
    return best


def timed_pass(ctx, st, steps, warmup, stream):
    """Warmup + timed passes, each from a cold kernel-length solve.  Returns the
    mean per-stage HIP-event durations (ms) of the timed passes and the
    per-kernel totals of the library's event pairs over the timed passes."""
    import torch
    stages = ("build", "solve_h", "gradients", "fluxes")
    acc = {k: [] for k in stages}
    for it in range(warmup + steps):
        if it == warmup:
            ctx.set_kernel_timing(True)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        st.H.zero_()
        ev[0].record(stream)
        ctx.build_neighbours(st)
        ev[1].record(stream)
        ctx.solve_h(st)
        ev[2].record(stream)
        ctx.gradients(st)
        ev[3].record(stream)
        ctx.hydro_fluxes(st)
        ev[4].record(stream)
        if it >= warmup:
            torch.cuda.synchronize()
            for k, s in enumerate(stages):
                acc[s].append(ev[k].elapsed_time(ev[k + 1]))
    torch.cuda.synchronize()
    kern = {}
    for k in ("solve_h", "gradients", "hydro_fluxes"):
        ms, launches = ctx.kernel_time(k)
        kern[k] = {"ms_total": ms, "launches": launches, "ms_avg": ms / max(launches, 1)}
    ctx.set_kernel_timing(False)
    return {k: float(np.mean(v)) for k, v in acc.items()}, kern


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"cpu_model": model, "host_cpus": os.cpu_count(), "cpus_available": avail}


CPU_QUANTILES = (0.2, 0.4, 0.6, 0.8)


def cpu_sample(w, side=0.125, quantiles=CPU_QUANTILES):
    """Sub-cubes of side `side` (of the unit box) whose particle counts sit at
    the given quantiles of all sub-cubes' counts, each as an open box with its
    own origin: bounded pieces of the same particle set, spread over its
    density range, that the oracle can pass over whole."""
    from paper_1712_01294_amd import workloads
    nc = int(round(1.0 / side))
    X = np.stack([w.x, w.y, w.z]) / np.array(w.box)[:, None]
    c = np.minimum((X * nc).astype(np.int64), nc - 1)
    cell = (c[0] * nc + c[1]) * nc + c[2]
    counts = np.bincount(cell, minlength=nc ** 3)
    order = np.argsort(counts, kind="stable")
    subs = []
    for q in quantiles:
        pick = int(order[min(len(order) - 1, int(q * len(order)))])
        sel = np.flatnonzero(cell == pick)
        o = np.array([pick // (nc * nc), (pick // nc) % nc, pick % nc]) * side
        subs.append((workloads.Workload(name=w.name + "[sub-cube]", x=w.x[sel] - o[0], y=w.y[sel] - o[1],
                                        z=w.z[sel] - o[2], m=w.m[sel], vx=w.vx[sel], vy=w.vy[sel],
                                        vz=w.vz[sel], u=w.u[sel], gamma=w.gamma, box=(side, side, side),
                                        periodic=(0, 0, 0), n_ngb=w.n_ngb), pick))
    return subs


def cpu_baseline(w):
    """The FP64 oracle's whole-set pass (kernel lengths, gradients, fluxes) on a
    bounded sample of the workload: four sub-cubes of the benchmark's own set,
    each treated as an open box and passed over whole; pairs summed over the
    four, divided by their summed time.  Single-threaded, then the OpenMP build
    of the same oracle on every thread OpenMP is given."""
    from oracle import oracle as O
    subs = cpu_sample(w)
    info = host_cpu()
    runs = {}
    for kind in ("oracle", "oracle_omp"):
        pairs, t, parts = 0, 0.0, []
        with (O.openmp() if kind == "oracle_omp" else contextlib.nullcontext()):
            cores = O.threads()
            for sub, pick in subs:
                t0 = time.perf_counter()
                out = O.hydro_pass(O.Setup.of(sub), sub.arrays())
                dt = time.perf_counter() - t0
                pairs += out["pairs"]
                t += dt
                parts.append(f"cube {pick}: {sub.n} particles, {out['pairs']} pairs, {dt:.2f} s")
        runs[kind] = {"value": pairs / t, "unit": "pairs/s", "cores": cores, "kind": kind,
                      "sample": "whole-set oracle passes (cold kernel lengths) over four sub-cubes (side 1/8 "
                                "of the box, open boundaries) of the same " + str(w.n) + "-particle set, at the "
                                "20/40/60/80th percentiles of the 512 sub-cubes' particle counts; "
                                + "; ".join(parts),
                      **info}
    return runs["oracle"], runs["oracle_omp"]


# Algorithmic traffic of forward + adjoint per particle (10 fixed-dt steps,
# taped): forward = the initial pass (600 B: 48 + 264 + 288) and 10 steps of a
# pass plus the kick-drift-kick streaming (~160 B: x, v, u, m, dp, dE in; x, v,
# u and the predicted v, u out), one checkpoint copy (192 B read and written)
# and the tape written (~465 B: 42 doubles, 3 int32 and the ~29 used list
# entries); backward = per step the tape read (465 B), the reverse pass (the
# pass's 600 B plus 88 B of adjoints in and out) and the reverse step streaming
# (~200 B), then the initial pass recomputed and reversed (1,288 B).  One
# step's working set on the 64^3 box (~100 MB) fits in the 256 MB Infinity
# Cache, so this is a traffic-equivalent rate, not an HBM measurement.
ADJ_BYTES_PER_PARTICLE = (600 + 10 * (600 + 160 + 192 + 465)) + (10 * (465 + 688 + 200) + 1288)


def adjoint_timing(reps=3):
    """Forward (initial pass + 10 fixed-dt steps with checkpoints) and backward
    (hand-written adjoint with recomputation) on the 64^3 jittered box, FP64."""
    import torch

    from paper_1712_01294_amd import autodiff, workloads
    w = workloads.adjoint_box()
    evo = autodiff.Evolution(w, w.steps, w.dt)
    m = torch.tensor(w.m, device="cuda")
    v0 = torch.tensor(np.stack([w.vx, w.vy, w.vz]), device="cuda")
    u0 = torch.tensor(w.u, device="cuda")
    fw, bw = [], []
    for it in range(reps + 1):
        vr = v0.clone().requires_grad_(True)
        ur = u0.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        vk, uk = autodiff.MFMSteps.apply(vr, ur, evo)
        L = (m * (vk * vk).sum(0)).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        L.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if it:
            fw.append(t1 - t0)
            bw.append(t2 - t1)
    evo.ctx.check()
    fwd, adj = float(np.median(fw)) * 1e3, float(np.median(bw)) * 1e3
    b = ADJ_BYTES_PER_PARTICLE * float(w.n)
    rate = b / ((fwd + adj) * 1e-3)
    return {"workload": f"jittered box 64^3 = {w.n} particles, {w.steps} fixed steps of dt = {w.dt}, "
                        "L = sum m |v|^2 at the end, gradient w.r.t. (v0, u0)",
            "fwd_ms": fwd, "adj_ms": adj, "fwd_adj_ms": fwd + adj, "reps": reps,
            "roofline": {"bound": "hbm", "achieved": rate / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                         "frac": rate / PEAK_HBM, "algorithmic_bytes": b,
                         "note": "algorithmic bytes of forward + adjoint over their wall time; the set fits "
                                 "in the Infinity Cache"},
            "note": "wall clock with the stream synchronised at both ends; forward keeps one checkpoint and one tape per step, the backward reads the tapes"}


def run_precision(mfm, w, prec, kw, args, stream, scheme=0):
    ctx = mfm.Context(mfm.config_of(w, precision=prec, scheme=scheme, **kw), w.n)
    st = mfm.State.from_arrays(w.arrays(), ids=True, dm=scheme == mfm.SCHEME_MFV)
    ctx.build_neighbours(st)
    ctx.hydro_pass(st)
    ctx.check(allow_illcond=True)
    tm, kern = timed_pass(ctx, st, args.steps, args.warmup, stream)
    ctx.check(allow_illcond=True)
    cnt = ctx.counters()
    return ctx, st, tm, kern, cnt


def hier_bins(cfg, st, max_bin, ctx):
    """Time bins from the state's last pass on ctx (the hierarchical leg's
    binning), in the particles' current order:
    dt_i = min(cfl H_i / vsig_i, sqrt(2 cfl H_i / |a_i|)) with a_i = dp_i / m_i,
    bin_i = max_bin - floor(log2(dt_i / dt_min)) clamped to [0, max_bin];
    then the neighbour limiter of individual time-step schemes
    (mfm_limit_bins): each bin is raised to at least its flux neighbours' bins
    minus one, until no bin changes, so neighbours step at most a factor 2
    apart.  Returns (bins,
    T = 2^max_bin dt_min, dt_min, number of bins the limiter raised)."""
    import torch
    acc = torch.sqrt((st.dp * st.dp).sum(0)) / st.m
    dti = torch.minimum(cfg.cfl * st.H / st.vsig, torch.sqrt(2.0 * cfg.cfl * st.H / acc)).double()
    dtmin = float(dti.min())
    if not (dtmin > 0.0 and np.isfinite(dtmin)):
        raise RuntimeError(f"hierarchical leg: no finite step (min {dtmin})")
    bins = (max_bin - torch.floor(torch.log2(dti / dtmin))).clamp(0, max_bin).to(torch.int64).contiguous()
    raised = ctx.limit_bins(st, bins, max_bin)
    return bins, dtmin * (1 << max_bin), dtmin, raised


def hierarchical_timing(mfm, w, kw, max_bin=3, reps=3, active_only=False):
    """Hierarchical power-of-two steps on the same set.  Each particle's bin
    comes from its step of an initial pass, the smaller of the Courant step
    cfl H_i / vsig_i (the step the library takes when dt <= 0) and the step in
    which its acceleration a_i = dp_i / m_i alone moves it by cfl H_i,
    sqrt(2 cfl H_i / |a_i|): with dt_min the smallest,
    bin_i = max_bin - floor(log2(dt_i / dt_min)), clamped to [0, max_bin], so
    it steps by T / 2^bin_i <= dt_i within the system step T = 2^max_bin dt_min;
    the neighbour limiter then keeps flux neighbours within one bin of each
    other (hier_bins).  One system step (2^max_bin sub-steps, each pass evaluating only the due
    pairs' fluxes) is timed against the 2^max_bin global steps of dt_min that
    cover the same time from the same state; every timed call is logged and
    followed by the counters' check, so a state that went non-finite ends the
    leg with an error instead of slowing the solves."""
    import torch
    cfg = mfm.config_of(w, **kw)
    ctx = mfm.Context(cfg, w.n)
    st = mfm.State.from_arrays(w.arrays())
    ctx.build_neighbours(st)
    ctx.hydro_pass(st)
    bins, T, dtmin, raised = hier_bins(cfg, st, max_bin, ctx)
    hist = torch.bincount(bins, minlength=max_bin + 1).tolist()
    log(f"hierarchical: cfl {cfg.cfl}, dt_min {dtmin:.3e}, T {T:.3e}, particles per bin {hist} "
        f"({raised} raised by the neighbour limiter)")
    start = {k: getattr(st, k).clone() for k in ("x", "y", "z", "vx", "vy", "vz", "u", "id")}
    b0 = bins.clone()

    def restore():
        for k, v in start.items():
            getattr(st, k).copy_(v)
        bins.copy_(b0)
        st.H.zero_()
        ctx.build_neighbours(st)
        ctx.hydro_pass(st)

    def timed(name, fn):
        ts = []
        for it in range(reps + 1):
            restore()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            ctx.check(allow_illcond=True)
            log(f"hierarchical: {name} {'warm-up' if it == 0 else 'run'} {it}: {ms:.1f} ms")
            if it:
                ts.append(ms)
        return float(np.median(ts))

    act = timed("system step, active subsets", lambda: ctx.step_hier(st, bins, max_bin, T, rebin=True, active=True))
    if active_only:
        return {"max_bin": max_bin, "bin_counts": hist, "limiter_raised": raised, "ms_per_system_step_active": act}
    hier = timed("system step, every particle", lambda: ctx.step_hier(st, bins, max_bin, T, rebin=True))
    glob = timed(f"{1 << max_bin} global steps", lambda: [ctx.step(st, dtmin) for _ in range(1 << max_bin)])
    del ctx, st
    torch.cuda.empty_cache()
    return {"max_bin": max_bin, "sub_steps": 1 << max_bin, "bin_counts": hist, "limiter_raised": raised,
            "T": T, "dt_min": dtmin,
            "ms_per_system_step_active": act, "ms_per_system_step": hier, "global_ms": glob,
            "speedup_vs_global_active": glob / act, "speedup_vs_global": glob / hier,
            "note": "wall clock of one system step (the levelled pass of every level at its start included) "
                    "against the global steps of the smallest step over the same time; with active "
                    "subsets a sub-step recomputes kernel lengths and gradients of the due bins' particles "
                    "only, without them of every particle; either way the flux kernel skips the pairs not due"}


def kernel_table(w, kern, n, G, F, P, iters, fp, mixed):
    """Per-kernel rates against the roofs at the algorithmic counts, with the
    measured traffic and VALU counters of the same sources when recorded."""
    kernels = {}
    for k, v in kern.items():
        b, f, lb = algorithmic(k, n, G, F, P, iters)
        s = v["ms_avg"] * 1e-3
        # the mixed flux kernel's pair arithmetic is FP32; everything else FP64
        peak = PEAK_FP32_VALU if (mixed and k == "hydro_fluxes") else PEAK_FP64_VALU
        fh, fa = b / s / PEAK_HBM, f / s / peak
        e = {"kernel": KERNEL_NAMES[k], "ms_avg": v["ms_avg"], "launches": v["launches"],
             "algorithmic_bytes": b, "list_bytes": lb, "algorithmic_flops": f,
             "GBps": b / s / 1e9, "frac_hbm": fh, "GFLOPps": f / s / 1e9,
             "alu_peak_TFLOPps": peak / 1e12, "frac_alu": fa, "bound": binding(fh, fa)}
        key = (w.name, k + ("_mixed" if mixed else ""))
        tr = TRAFFIC.get(key)
        e["traffic"] = tr["bytes_per_launch"] if tr and tr["fingerprint"] == fp else None
        if e["traffic"] is not None:
            e["traffic_GBps"] = e["traffic"] / s / 1e9
            e["traffic_frac_hbm"] = e["traffic"] / s / PEAK_HBM
        ct = COUNTERS.get(key)
        if ct and ct["fingerprint"] == fp:
            e["counters"] = {"valu_busy_pct": ct["valu_busy_pct"],
                             "executed_fp64_TFLOPps": ct["fp64_flops_per_launch"] / s / 1e12,
                             "executed_fp32_TFLOPps": ct["fp32_flops_per_launch"] / s / 1e12,
                             "valu_insts_per_launch": ct["valu_insts_per_launch"]}
        kernels[k] = e
    return kernels


def roofline_of(dk, fp):
    """The bench line's roofline object for one kernel: the roof it is closer to
    at its algorithmic counts, the other roof beside it."""
    alu = {"achieved": dk["GFLOPps"] / 1e3, "peak": dk["alu_peak_TFLOPps"], "unit": "TFLOP/s",
           "frac": dk["frac_alu"], "flops_per_launch": dk["algorithmic_flops"]}
    hbm = {"achieved": dk["GBps"], "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": dk["frac_hbm"],
           "bytes_per_launch": dk["algorithmic_bytes"], "list_bytes_per_launch": dk["list_bytes"]}
    top = alu if dk["bound"] == "alu" else hbm
    r = {"kernel": dk["kernel"], "bound": dk["bound"], "achieved": top["achieved"], "peak": top["peak"],
         "unit": top["unit"], "frac": top["frac"], "traffic": dk["traffic"], "ms_avg": dk["ms_avg"],
         "hbm": hbm, "alu": alu, "source_fingerprint": fp}
    if "counters" in dk:
        r["counters"] = dk["counters"]
    return r


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU (asked for --gpus {args.gpus}); this build has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "no GPU"
    if args.copy_probe:
        copy_probe()
        return
    if args.adjoint_only:
        print(json.dumps({"adjoint": adjoint_timing()}), flush=True)
        return

    from paper_1712_01294_amd import mfm, workloads
    t0 = time.time()
    w = workloads.by_name(args.workload)
    log(f"workload {w.name}: n={w.n} generated in {time.time() - t0:.1f}s")
    kw = {}
    if args.tree_levels:
        kw["tree_levels"] = args.tree_levels
    if args.max_ngb:
        kw["max_ngb"] = args.max_ngb
    stream = torch.cuda.current_stream()
    if args.hier_only:
        print(json.dumps({"hierarchical": hierarchical_timing(mfm, w, kw, active_only=True)}), flush=True)
        return

    ctx, st64, tm, kern, cnt = run_precision(mfm, w, mfm.FP64, kw, args, stream)
    log(f"fp64: pairs={cnt['pairs']} gather={cnt['gather_entries']} list_max={cnt['list_max']} "
        f"h_rounds_max={cnt['h_rounds_max']} h_fallback={cnt['h_fallback']} illcond={cnt['illcond']} "
        + " ".join(f"{k}={v:.3f}ms" for k, v in tm.items()))
    del ctx
    n, P, F, G = w.n, cnt["pairs"], cnt["list_entries"], cnt["gather_entries"]
    iters = cnt["h_iters"] / n
    pass_ms = tm["solve_h"] + tm["gradients"] + tm["fluxes"]
    fp = source_fingerprint()
    kernels = kernel_table(w, kern, n, G, F, P, iters, fp, mixed=False)
    dom = max(kernels, key=lambda k: kernels[k]["ms_avg"])
    roofline = roofline_of(kernels[dom], fp)
    ceiling = copy_ceiling(stream)
    roofline["hbm"]["measured_copy_ceiling_GBps"] = ceiling / 1e9

    out = {
        "metric": METRIC,
        "value": P / (pass_ms * 1e-3),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": pass_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n_particles": n, "unordered_pairs": P, "gather_entries": G,
                   "n_ngb": w.n_ngb, "gamma": w.gamma, "box": list(w.box), "h_start": "cold (H = 0)"},
        "stage_ms": tm,
        "value_incl_build": P / ((pass_ms + tm["build"]) * 1e-3),
        "roofline": roofline,
        "kernels": kernels,
    }

    if not args.no_mixed:
        ctx, stmx, tmx, kmx, cmx = run_precision(mfm, w, mfm.MIXED, kw, args, stream)
        del ctx
        mx_ms = tmx["solve_h"] + tmx["gradients"] + tmx["fluxes"]
        same = torch.equal(st64.id, stmx.id)
        errs = None
        if same:
            errs = {}
            for k in ("dp", "dE", "vsig", "grad", "B", "rho", "P", "H"):
                a = getattr(st64, k).double()
                b = getattr(stmx, k).double()
                errs[k] = float((a - b).abs().max() / a.abs().max())
        pm = torch.tensor([float((st64.dp[c]).sum()) for c in range(3)])
        kx = kernel_table(w, kmx, n, G, F, P, cmx["h_iters"] / n, fp, mixed=True)
        mdom = max(kx, key=lambda k: kx[k]["ms_avg"])
        out["mixed"] = {"value": cmx["pairs"] / (mx_ms * 1e-3), "unit": "pairs/s", "dtype": "f32/f64",
                        "ms_per_step": mx_ms, "stage_ms": tmx,
                        "kernel_ms": {k: v["ms_avg"] for k, v in kmx.items()},
                        "kernels": kx, "roofline": roofline_of(kx[mdom], fp),
                        "speedup_vs_fp64": pass_ms / mx_ms,
                        "normwise_error_vs_fp64": errs,
                        "momentum_sum_mixed": [float(stmx.dp[c].sum()) for c in range(3)],
                        "momentum_sum_fp64": pm.tolist()}
        log(f"mixed: " + " ".join(f"{k}={v:.3f}ms" for k, v in tmx.items()) + f" errs={errs}")
        del stmx
    del st64
    torch.cuda.empty_cache()

    if not args.no_mfv:
        ctx, stv, tv, kv, cv = run_precision(mfm, w, mfm.FP64, kw, args, stream, scheme=mfm.SCHEME_MFV)
        del ctx
        v_ms = tv["solve_h"] + tv["gradients"] + tv["fluxes"]
        fk = kv["hydro_fluxes"]
        b, f, lb = algorithmic("hydro_fluxes_mfv", n, cv["gather_entries"], cv["list_entries"], cv["pairs"])
        s = fk["ms_avg"] * 1e-3
        dm = stv.dm
        out["mfv"] = {"value": cv["pairs"] / (v_ms * 1e-3), "unit": "pairs/s", "dtype": "f64",
                      "ms_per_step": v_ms, "stage_ms": tv,
                      "flux_kernel": {"kernel": "k_fluxes_mfv", "ms_avg": fk["ms_avg"], "launches": fk["launches"],
                                      "algorithmic_bytes": b, "list_bytes": lb, "GBps": b / s / 1e9,
                                      "frac_hbm": b / s / PEAK_HBM,
                                      "algorithmic_flops": f, "GFLOPps": f / s / 1e9,
                                      "frac_fp64": f / s / PEAK_FP64_VALU},
                      "mass_rate_sum_rel": float(dm.sum().abs() / dm.abs().sum()),
                      "flux_kernel_traffic": (TRAFFIC[(w.name, "hydro_fluxes_mfv")]["bytes_per_launch"]
                                              if (w.name, "hydro_fluxes_mfv") in TRAFFIC
                                              and TRAFFIC[(w.name, "hydro_fluxes_mfv")]["fingerprint"] == fp
                                              else None),
                      "fallbacks": cv["fallbacks"]}
        log(f"mfv: " + " ".join(f"{k}={v:.3f}ms" for k, v in tv.items())
            + f" flux kernel {fk['ms_avg']:.3f} ms")
        if not args.no_mixed:
            ctx, stvm, tvm, kvm, cvm = run_precision(mfm, w, mfm.MIXED, kw, args, stream, scheme=mfm.SCHEME_MFV)
            del ctx
            vm_ms = tvm["solve_h"] + tvm["gradients"] + tvm["fluxes"]
            errs = None
            if torch.equal(stv.id, stvm.id):
                errs = {k: float((getattr(stv, k) - getattr(stvm, k)).abs().max() / getattr(stv, k).abs().max())
                        for k in ("dm", "dp", "dE")}
            out["mfv"]["mixed"] = {"value": cvm["pairs"] / (vm_ms * 1e-3), "unit": "pairs/s", "dtype": "f32/f64",
                                   "ms_per_step": vm_ms, "flux_kernel_ms": kvm["hydro_fluxes"]["ms_avg"],
                                   "normwise_error_vs_fp64": errs}
            log(f"mfv mixed: flux kernel {kvm['hydro_fluxes']['ms_avg']:.3f} ms errs={errs}")
            del stvm
        del stv
        torch.cuda.empty_cache()

    if not args.no_limited:
        # the optional limiters (pairwise face limiter and condition-adaptive
        # beta): FP64 and mixed in both schemes, the mixed form's error against
        # FP64 under the same limiters, and the first-order switches each takes
        lk = dict(kw, limiter=1, beta=2.0, beta_min=1.0, cond_lo=10.0, cond_hi=1000.0)
        out["limited"] = {"params": {k: lk[k] for k in ("limiter", "beta", "beta_min", "cond_lo", "cond_hi")}}
        for name, sch in (("mfm", mfm.SCHEME_MFM), ("mfv", mfm.SCHEME_MFV)):
            ctx, s64, t64, _, c64 = run_precision(mfm, w, mfm.FP64, lk, args, stream, scheme=sch)
            del ctx
            ctx, s32, t32, _, c32 = run_precision(mfm, w, mfm.MIXED, lk, args, stream, scheme=sch)
            del ctx
            ms64 = t64["solve_h"] + t64["gradients"] + t64["fluxes"]
            ms32 = t32["solve_h"] + t32["gradients"] + t32["fluxes"]
            errs = None
            if torch.equal(s64.id, s32.id):
                errs = {k: float((getattr(s64, k) - getattr(s32, k)).abs().max() / getattr(s64, k).abs().max())
                        for k in (("dm", "dp", "dE") if name == "mfv" else ("dp", "dE"))}
            out["limited"][name] = {"value": c64["pairs"] / (ms64 * 1e-3), "unit": "pairs/s", "dtype": "f64",
                                    "ms_per_step": ms64, "first_order_faces": c64["fallbacks"],
                                    "mixed": {"value": c32["pairs"] / (ms32 * 1e-3), "unit": "pairs/s",
                                              "dtype": "f32/f64", "ms_per_step": ms32,
                                              "first_order_faces": c32["fallbacks"],
                                              "normwise_error_vs_fp64": errs}}
            log(f"limited {name}: fp64 {ms64:.3f} ms, mixed {ms32:.3f} ms, errs={errs}")
            del s64, s32
            torch.cuda.empty_cache()

    if not args.no_hier:
        out["hierarchical"] = hierarchical_timing(mfm, w, kw)
        hh = out["hierarchical"]
        log(f"hierarchical: {hh['ms_per_system_step_active']:.1f} ms per system step of {hh['sub_steps']} sub-steps "
            f"with active subsets, {hh['ms_per_system_step']:.1f} ms without, "
            f"{hh['global_ms']:.1f} ms for the same time in global steps")

    if not args.no_adjoint:
        log("adjoint ...")
        out["adjoint"] = adjoint_timing()
        log(f"adjoint: {out['adjoint']['fwd_ms']:.1f} ms fwd + {out['adjoint']['adj_ms']:.1f} ms adj")
    if not args.no_cpu:
        log("cpu baseline ...")
        out["cpu_baseline"], out["cpu_baseline_omp"] = cpu_baseline(w)
        log(f"cpu baseline: {out['cpu_baseline']['value']:.3e} pairs/s on 1 thread, "
            f"{out['cpu_baseline_omp']['value']:.3e} on {out['cpu_baseline_omp']['cores']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
