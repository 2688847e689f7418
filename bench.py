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
PEAK_FP64_VALU = 78.6e12   # flop/s, FP64 vector
PEAK_FP32_VALU = 157.3e12  # flop/s, FP32 vector (packed)

# Algorithmic work per unit (each particle's inputs read once and its outputs
# written once; neighbour data are re-reads).  n particles, G gather entries
# (self excluded), F directed flux-list entries (= 2 pairs), P unordered pairs.
#   solve_h:   x (24 B) + H guess (8 B) in; H, n, V (24 B) + two list lengths (8 B)
#              out; one 4 B index per gather entry.  Flops: distance and root
#              (sqrt) 9 + two spline evaluations (f, f') 24 per gather entry.
#   gradients: x, H, V, n, m, v, u (88 B) and the gather list in; B (48 B),
#              rho, P (16 B), five gradients (120 B) and the transposed flux-list
#              entries (4 B each) out.  Flops: about 75 per gather entry
#              (distance, W, E and the 15 weighted differences, extrema) and 200
#              per particle (inverse, products, limiter).
#   fluxes:    x, H, V, B, rho, P, v, gradients (248 B) and the flux list in;
#              dp, dE, vsig (40 B) out.  Flops: 236 per unordered pair (kernel
#              weights 20, faces 52, reconstruction 70, frame 22, HLLC 31, flux
#              6, distance 9, accumulation and signal speed 26), add/mul/div/sqrt
#              counted as one and fma as two.
#   fluxes, finite-volume form: dm (8 B) more out; the full HLLC flux of the
#              selected side (state, physical flux, star correction) and the
#              lab-frame boost replace the P* flux: about 310 flops per pair.
def algorithmic(kernel, n, G, F, P):
    if kernel == "solve_h":
        return 64.0 * n + 4.0 * G, 33.0 * G
    if kernel == "gradients":
        return 272.0 * n + 4.0 * F, 75.0 * G + 200.0 * n
    if kernel == "hydro_fluxes":
        return 288.0 * n + 4.0 * F, 236.0 * P
    if kernel == "hydro_fluxes_mfv":
        return 296.0 * n + 4.0 * F, 310.0 * P
    raise KeyError(kernel)


KERNEL_NAMES = {"solve_h": "k_solve_h + k_solve_h_wave + k_solve_h_fallback", "gradients": "k_gradients<false>",
                "hydro_fluxes": "k_fluxes_f64"}
KERNEL_SOURCES = ("paper_1712_01294_amd/csrc/pass.hip", "paper_1712_01294_amd/csrc/device.h",
                  "paper_1712_01294_amd/csrc/kernels.h")

# HBM traffic per launch from rocprofv3 FETCH_SIZE and WRITE_SIZE passes over
# this benchmark, scaled by what the same counters read for a plain copy of
# known size (bench.py --copy-probe).  Keyed by workload and kernel, and valid
# only for the kernel sources whose fingerprint is recorded with it.
TRAFFIC = {
    ("clustered", "solve_h"): {"bytes_per_launch": 141.36e9, "fingerprint": "cadc716193b0a796"},
    ("clustered", "gradients"): {"bytes_per_launch": 30.52e9, "fingerprint": "cadc716193b0a796"},
    ("clustered", "hydro_fluxes"): {"bytes_per_launch": 13.80e9, "fingerprint": "cadc716193b0a796"},
    ("clustered", "hydro_fluxes_mfv"): {"bytes_per_launch": 14.18e9, "fingerprint": "cadc716193b0a796"},
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
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="clustered")
    ap.add_argument("--tree-levels", type=int, default=0)
    ap.add_argument("--max-ngb", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-mfv", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only the forward + adjoint timing of 10 steps on the 64^3 box")
    return ap.parse_args()


def copy_probe():
    """Five copies of a 1 GiB device buffer: 1 GiB fetched and 1 GiB written per launch."""
    import torch
    nbytes = 1 << 30
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_per_launch": nbytes, "launches": 5}), flush=True)


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


def cpu_baseline(w, budget_s):
    """The FP64 oracle on a bounded sample of the same workload: the particles of a
    sub-box (all their dependencies computed), pairs of the sample per second."""
    from oracle import oracle as O
    s = O.Setup.of(w)
    X = np.stack([w.x, w.y, w.z], 1)
    box = np.array(w.box)
    order = np.argsort(((X / box) ** 2).sum(1))   # nearest the origin corner first

    def run(k):
        H, nk, V, _ = O.solve_h(s, w.x, w.y, w.z, None, mask=_mask(order[:k], w.n))
        t0 = time.perf_counter()
        out = O.sampled_pass(s, w.arrays(), order[:k], h_bound=_hbound(H))
        return time.perf_counter() - t0, out

    def _mask(idx, n):
        m = np.zeros(n, dtype=bool)
        m[idx] = True
        return m

    def _hbound(H):
        h = H[H > 0]
        return float(h.max()) * 1.5

    # double the sample while the next run, extrapolated with the growth of the
    # last doubling, stays within the budget (the dependency closure, and so the
    # cost per target, grows with the largest kernel length in the sample)
    k = 500
    t, out = run(k)
    growth = 2.0
    while k < w.n and t * growth <= budget_s:
        t_prev = t
        t_new, out_new = run(int(min(w.n, 2 * k)))
        k, t, out = int(min(w.n, 2 * k)), t_new, out_new
        growth = max(2.0, t / max(t_prev, 1e-9))
    pairs = out["pair_entries"] / 2.0
    return {"value": pairs / t, "unit": "pairs/s", "cores": 1, "kind": "oracle",
            "sample": f"{k} targets nearest one box corner of the same {w.n}-particle set, with every "
                      f"particle they depend on; {out['pair_entries']} directed flux entries in {t:.1f} s"}


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
    return {"workload": f"jittered box 64^3 = {w.n} particles, {w.steps} fixed steps of dt = {w.dt}, "
                        "L = sum m |v|^2 at the end, gradient w.r.t. (v0, u0)",
            "fwd_ms": fwd, "adj_ms": adj, "fwd_adj_ms": fwd + adj, "reps": reps,
            "note": "wall clock with the stream synchronised at both ends; forward keeps one checkpoint per step"}


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

    ctx, st64, tm, kern, cnt = run_precision(mfm, w, mfm.FP64, kw, args, stream)
    log(f"fp64: pairs={cnt['pairs']} gather={cnt['gather_entries']} list_max={cnt['list_max']} "
        f"h_rounds_max={cnt['h_rounds_max']} h_fallback={cnt['h_fallback']} illcond={cnt['illcond']} "
        + " ".join(f"{k}={v:.3f}ms" for k, v in tm.items()))
    del ctx
    n, P, F, G = w.n, cnt["pairs"], cnt["list_entries"], cnt["gather_entries"]
    pass_ms = tm["solve_h"] + tm["gradients"] + tm["fluxes"]

    kernels = {}
    for k, v in kern.items():
        b, f = algorithmic(k, n, G, F, P)
        s = v["ms_avg"] * 1e-3
        kernels[k] = {"kernel": KERNEL_NAMES[k], "ms_avg": v["ms_avg"], "launches": v["launches"],
                      "algorithmic_bytes": b, "algorithmic_flops": f,
                      "GBps": b / s / 1e9, "frac_hbm": b / s / PEAK_HBM,
                      "GFLOPps": f / s / 1e9, "frac_fp64": f / s / PEAK_FP64_VALU}
    fp = source_fingerprint()
    for k, v in kernels.items():
        tr = TRAFFIC.get((w.name, k))
        v["traffic"] = tr["bytes_per_launch"] if tr and tr["fingerprint"] == fp else None
    dom = max(kernels, key=lambda k: kernels[k]["ms_avg"])
    dk = kernels[dom]
    traffic = dk["traffic"]
    # the pass is memory-side at algorithmic intensity (flop/B below the FP64 ridge)
    roofline = {"kernel": dk["kernel"], "bound": "hbm", "achieved": dk["GBps"], "peak": PEAK_HBM / 1e9,
                "unit": "GB/s", "frac": dk["frac_hbm"], "traffic": traffic,
                "algorithmic_bytes_per_launch": dk["algorithmic_bytes"], "ms_avg": dk["ms_avg"],
                "fp64_alu": {"achieved": dk["GFLOPps"] / 1e3, "peak": PEAK_FP64_VALU / 1e12,
                             "unit": "TFLOP/s", "frac": dk["frac_fp64"]},
                "source_fingerprint": fp}

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
        out["mixed"] = {"value": cmx["pairs"] / (mx_ms * 1e-3), "unit": "pairs/s", "dtype": "f32/f64",
                        "ms_per_step": mx_ms, "stage_ms": tmx,
                        "kernel_ms": {k: v["ms_avg"] for k, v in kmx.items()},
                        # the pair arithmetic of the mixed flux kernel is FP32: its flops
                        # against the FP32 vector peak
                        "flux_GFLOPps": algorithmic("hydro_fluxes", n, G, F, P)[1] / (kmx["hydro_fluxes"]["ms_avg"] * 1e-3) / 1e9,
                        "flux_frac_fp32": algorithmic("hydro_fluxes", n, G, F, P)[1]
                        / (kmx["hydro_fluxes"]["ms_avg"] * 1e-3) / PEAK_FP32_VALU,
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
        b, f = algorithmic("hydro_fluxes_mfv", n, cv["gather_entries"], cv["list_entries"], cv["pairs"])
        s = fk["ms_avg"] * 1e-3
        dm = stv.dm
        out["mfv"] = {"value": cv["pairs"] / (v_ms * 1e-3), "unit": "pairs/s", "dtype": "f64",
                      "ms_per_step": v_ms, "stage_ms": tv,
                      "flux_kernel": {"kernel": "k_fluxes_mfv", "ms_avg": fk["ms_avg"], "launches": fk["launches"],
                                      "algorithmic_bytes": b, "GBps": b / s / 1e9, "frac_hbm": b / s / PEAK_HBM,
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

    if not args.no_adjoint:
        log("adjoint ...")
        out["adjoint"] = adjoint_timing()
        log(f"adjoint: {out['adjoint']['fwd_ms']:.1f} ms fwd + {out['adjoint']['adj_ms']:.1f} ms adj")
    if not args.no_cpu:
        log("cpu baseline ...")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
