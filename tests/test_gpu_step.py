"""Kick-drift-kick step of the HIP path against the oracle's step, and the
planar shock tube at full size against the exact Riemann solution."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from oracle import riemann_exact as R
from paper_1712_01294_amd import workloads as W

from .gpu_util import in_input_order, nerr

pytestmark = pytest.mark.gpu

LEFT = (1.0, 0.0, 1.0)
RIGHT = (0.125, 0.0, 0.1)


def _gpu_run(w, steps, dt=0.0, precision=0):
    import torch

    from paper_1712_01294_amd import mfm
    ctx = mfm.Context(mfm.config_of(w, precision=precision), w.n)
    st = mfm.State.from_arrays(w.arrays())
    ctx.build_neighbours(st)
    ctx.hydro_pass(st)
    ctx.check()
    dts = []
    for _ in range(steps):
        dts.append(ctx.step(st, dt))
    ctx.check()
    torch.cuda.synchronize()
    return ctx, st, dts


def _periodic_err(a, b, L):
    d = a - b
    d -= L * np.round(d / L)
    return float(np.abs(d).max())


@pytest.mark.parametrize("jitter,steps", [(0.2, 50), (0.0, 10)])
def test_step_matches_oracle_small_tube(jitter, steps):
    """CFL steps of a 10,368-particle shock tube: positions, velocities and
    energies within 1e-10 normwise of the oracle's step.  The jittered tube is
    held for all 50 steps of the configuration.  The perfect-lattice tube only
    for 10: its contact layer amplifies any asymmetric rounding by about 3x per
    step (pinned on the oracle alone in test_oracle_riemann), so past ~15 steps
    two correct implementations part by more than the bar."""
    w = W.shock_tube(n_yz=12, l_yz=12 / 64, jitter=jitter)
    ref = O.Stepper(w)
    ref.start()
    rdt = [ref.step() for _ in range(steps)]
    ctx, st, gdt = _gpu_run(w, steps)
    print("dt gpu", gdt[-1], "oracle", rdt[-1], flush=True)
    assert np.allclose(gdt, rdt, rtol=1e-12, atol=0)
    for k, L in (("x", w.box[0]), ("y", w.box[1]), ("z", w.box[2])):
        e = _periodic_err(in_input_order(st, k), ref.st[k], L)
        assert e <= 1e-10 * L, (k, e)
    for k in ("vx", "vy", "vz"):
        scale = np.abs(ref.st["vx"]).max()
        assert np.abs(in_input_order(st, k) - ref.st[k]).max() <= 1e-10 * scale, k
    assert nerr(in_input_order(st, "u"), ref.st["u"]) <= 1e-10
    assert nerr(in_input_order(st, "dp"), ref.last["dp"]) <= 1e-10
    assert nerr(in_input_order(st, "dE"), ref.last["dE"]) <= 1e-10


def test_mixed_step_matches_oracle_small_tube():
    """The mixed form's step (FP32 pair fluxes, FP64 state and sums) against the
    FP64 oracle's step over 10 CFL steps of the jittered small tube.  Each
    pass's flux error is within eps_F = 1e-5 of max|flux| (the mixed pass bar);
    a kick moves v by dt dp/m, and dt max|dp/m| stays below the largest
    velocity the run reaches, so after k steps the velocity error is at most
    k eps_F of max|v| when the map does not amplify differences (the jittered
    tube does not: test_oracle_riemann).  Bar: k eps_F = 1e-4 on v, u, dp
    and dE normwise, and positions within t k eps_F max|v|."""
    from paper_1712_01294_amd import mfm
    k = 10
    w = W.shock_tube(n_yz=12, l_yz=12 / 64)
    ref = O.Stepper(w)
    ref.start()
    rdt = [ref.step() for _ in range(k)]
    ctx, st, gdt = _gpu_run(w, k, precision=mfm.MIXED)
    bar = k * 1e-5
    vmax = float(np.abs(ref.st["vx"]).max())
    errs = {q: nerr(in_input_order(st, q), ref.st[q]) for q in ("vx", "u")}
    errs.update({q: nerr(in_input_order(st, q), ref.last[q]) for q in ("dp", "dE")})
    errs["v_transverse"] = max(float(np.abs(in_input_order(st, q) - ref.st[q]).max()) for q in ("vy", "vz")) / vmax
    errs["x"] = max(_periodic_err(in_input_order(st, q), ref.st[q], L)
                    for q, L in (("x", w.box[0]), ("y", w.box[1]), ("z", w.box[2]))) / (sum(rdt) * vmax)
    errs["dt"] = float(np.max(np.abs(np.array(gdt) / np.array(rdt) - 1.0)))
    print("mixed step vs oracle", " ".join(f"{q}={e:.2e}" for q, e in errs.items()), flush=True)
    for q, e in errs.items():
        assert e <= bar, (q, e)
    m = st.m.cpu().numpy()
    vx = st.vx.cpu().numpy()
    assert abs(float((m * vx).sum())) <= 1e-13 * float(np.abs(m * vx).sum())


def test_fixed_dt_steps_conserve_on_jittered_box():
    """Fixed dt on the jittered sine box: total momentum stays at round-off and
    total energy is conserved to round-off (the flux is antisymmetric pair by pair)."""
    w = W.jittered_sine(n_side=16, seed=W.SEED_BASE + 90)
    ref = O.Stepper(w)
    ref.start()
    for _ in range(5):
        ref.step(1e-3)
    ctx, st, _ = _gpu_run(w, 5, dt=1e-3)
    m = st.m.cpu().numpy()
    v = [getattr(st, k).cpu().numpy() for k in ("vx", "vy", "vz")]
    u = st.u.cpu().numpy()
    p0 = [float((w.m * getattr(w, k)).sum()) for k in ("vx", "vy", "vz")]
    E0 = float((w.m * (w.u + 0.5 * (w.vx ** 2 + w.vy ** 2 + w.vz ** 2))).sum())
    E = float((m * (u + 0.5 * (v[0] ** 2 + v[1] ** 2 + v[2] ** 2))).sum())
    mv = float(np.abs(m * v[0]).sum())
    for c in range(3):
        assert abs(float((m * v[c]).sum()) - p0[c]) <= 1e-13 * mv
    assert E == pytest.approx(E0, rel=1e-13)
    for k in ("vx", "vy", "vz", "u"):
        assert nerr(in_input_order(st, k), ref.st[k]) <= 1e-11, k


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_shock_tube_full_size_against_exact_riemann(precision):
    """The 294,912-particle tube (left 256 x 32 x 32 at spacing 1/256, right at
    1/128, both jittered by +-0.2 spacing), 50 CFL steps, in FP64 and in the
    mixed form: a convergence check against the exact Riemann solution
    (reported, not parity).  At t ~ 0.036 the post-shock gas between the
    contact and the shock spans about eight lattice planes.  The means over the
    middle 40% of that region must match the exact v and rho within 5% and P
    within 8%; the binned velocity profile on 0.9 <= x <= 1.15 within a mean
    absolute error of 0.07; the shock within two right-hand spacings of the
    exact one; momentum along the tube at round-off."""
    w = W.shock_tube()
    ctx, st, dts = _gpu_run(w, 50, precision=precision)
    t = float(np.sum(dts))
    gam = w.gamma
    p, u = R.star_state(LEFT, RIGHT, gam)
    _, rr = R.star_densities(LEFT, RIGHT, gam)
    S = R.wave_speeds(LEFT, RIGHT, gam)["right_shock"]
    x = st.x.cpu().numpy()
    vx = st.vx.cpu().numpy()
    rho = st.rho.cpu().numpy()
    P = st.P.cpu().numpy()
    lo = 1.0 + (u + 0.3 * (S - u)) * t
    hi = 1.0 + (S - 0.3 * (S - u)) * t
    sel = (x > lo) & (x < hi)
    bins = np.linspace(0.9, 1.15, 26)
    xc = 0.5 * (bins[1:] + bins[:-1])
    exact_v = R.sample(LEFT, RIGHT, gam, (xc - 1.0) / t)[1]
    b = np.digitize(x, bins) - 1
    prof = np.array([vx[b == k].mean() for k in range(len(xc))])
    l1 = float(np.mean(np.abs(prof - exact_v)))
    print(f"precision={precision} t={t:.5f} n_sel={sel.sum()} v={vx[sel].mean():.4f} (exact {u:.4f}) "
          f"P={P[sel].mean():.4f} ({p:.4f}) rho={rho[sel].mean():.4f} ({rr:.4f}) L1(v)={l1:.4f}", flush=True)
    assert sel.sum() > 300
    assert vx[sel].mean() == pytest.approx(u, rel=0.05)
    assert P[sel].mean() == pytest.approx(p, rel=0.08)
    assert rho[sel].mean() == pytest.approx(rr, rel=0.05)
    assert l1 <= 0.07
    order = np.argsort(x)
    xs, rs = x[order], rho[order]
    win = (xs > 1.0 + u * t) & (xs < 1.5)
    mid = 0.5 * (rr + RIGHT[0])
    cross = xs[win][np.flatnonzero(rs[win] < mid)[0]]
    assert abs(cross - (1.0 + S * t)) < 2 * w.extra["spacing_right"]
    m = st.m.cpu().numpy()
    assert abs(float((m * vx).sum())) <= 1e-13 * float(np.abs(m * vx).sum())
    c = ctx.counters()
    assert c["floors"] == 0


@pytest.mark.parametrize("scheme", [0, 1])
def test_fixed_dt_step_replays_from_a_hip_graph(scheme):
    """A fixed-dt step makes no host synchronisation, allocation or memset, so
    it can be captured into a HIP graph once and replayed.  The captured step
    is replayed four times, with eager steps of a second context and host
    synchronisations between the replays; after every replay the graph's
    state equals the eagerly stepped state bit for bit."""
    import torch

    from paper_1712_01294_amd import mfm
    w = W.jittered_sine(n_side=16, seed=W.SEED_BASE + 95)
    dt = 1e-3
    runs = []
    for _ in range(2):
        ctx = mfm.Context(mfm.config_of(w, scheme=scheme), w.n)
        st = mfm.State.from_arrays(w.arrays(), dm=scheme == 1)
        ctx.build_neighbours(st)
        ctx.hydro_pass(st)
        runs.append((ctx, st))
    torch.cuda.synchronize()
    (cg, sg), (ce, se) = runs
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        cg.step(sg, dt)
    torch.cuda.synchronize()
    names = ("x", "y", "z", "m", "vx", "vy", "vz", "u", "H", "dp", "dE", "vsig", "id") + (("dm",) if scheme else ())
    for r in range(4):
        g.replay()
        ce.step(se, dt)
        float(se.u.sum())                  # eager work and a synchronisation between replays
        torch.cuda.synchronize()
        for k in names:
            assert torch.equal(getattr(sg, k), getattr(se, k)), (r, k)
    cg.check()
    ce.check()
