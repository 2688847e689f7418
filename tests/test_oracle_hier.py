"""Pins of the oracle's hierarchical power-of-two time steps (R25, R26; no GPU).

* One bin for every particle: the hierarchical step is the global
  kick-drift-kick step (R17), bit for bit.
* Mixed bins: momentum and energy are conserved to rounding (every pair kick
  is applied with opposite signs to its two particles).
* Two groups that share no pair, in bins 0 and 1: each follows the global
  step of its own size (one step of T, two of T/2) to rounding.
* Coupled bins: the step converges at second order to classical RK4 on the
  semi-discrete system (which knows nothing about bins).

Active subsets (R26), where a sub-step's pass recomputes kernel lengths,
densities, volumes, gradient matrices and limited gradients only for the
particles of the due bins:

* With every particle due at every boundary, bit for bit the full passes.
* Along a three-level system step, the active particles' values equal an
  independent cold solve and gradient pass at that boundary, and the inactive
  ones' are bit for bit those of their last active boundary.
* Conservation to rounding, and a result that differs from R25's.
* The decoupled groups still follow their own global steps.
* Convergence to RK4, each halving of the step cutting the error by more
  than 2.5.
"""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_1712_01294_amd import workloads as W

T_END = 0.02


@pytest.fixture(scope="module")
def smooth_box():
    w0 = W.jittered_sine(n_side=8, seed=W.SEED_BASE + 61)
    tp = 2.0 * np.pi
    return dataclasses.replace(w0, vx=0.5 * np.sin(tp * w0.y), vy=0.5 * np.sin(tp * w0.z),
                               vz=0.5 * np.sin(tp * w0.x))


def _totals(st):
    m = st["m"]
    v = np.stack([st["vx"], st["vy"], st["vz"]])
    return (m * v).sum(1), float((m * (st["u"] + 0.5 * (v * v).sum(0))).sum()), np.abs(m * v).sum()


def test_one_bin_is_the_global_step_bitwise(smooth_box):
    w = smooth_box
    a = O.Stepper(w, u_floor=0.0)
    a.start()
    b = O.Stepper(w, u_floor=0.0)
    b.set_bins(np.zeros(w.n, dtype=np.int64))
    for _ in range(3):
        a.step(0.004)
        b.hier_step(0.004)
    for k in a.st:
        assert np.array_equal(a.st[k], b.st[k]), k
    for k in ("dp", "dE", "H"):
        assert np.array_equal(a.last[k], b.last[k]), k


@pytest.mark.parametrize("levels", [2, 3])
def test_mixed_bins_conserve_momentum_and_energy(smooth_box, levels):
    w = smooth_box
    bins = np.minimum((w.x * levels).astype(np.int64), levels - 1)
    s = O.Stepper(w, u_floor=0.0)
    s.set_bins(bins)
    p0, E0, _ = _totals(s.st)
    for _ in range(2):
        s.hier_step(0.004)
    p1, E1, scale = _totals(s.st)
    assert np.abs(p1 - p0).max() <= 1e-14 * scale.max()
    assert E1 == pytest.approx(E0, rel=1e-14)
    assert s.floors == 0


def _clump(origin, nside, spacing, rng):
    x, y, z = W.lattice_sites(nside, nside, nside, spacing, origin=origin)
    j = rng.uniform(-0.2, 0.2, size=(3, x.size)) * spacing
    return x + j[0], y + j[1], z + j[2]


def test_two_groups_without_common_pairs_follow_their_own_global_steps():
    rng = np.random.default_rng(41)
    sp = 0.04
    a = _clump((0.1, 0.1, 0.1), 6, sp, rng)
    b = _clump((0.62, 0.62, 0.62), 6, sp, rng)
    n = a[0].size
    X = [np.concatenate([a[c], b[c]]) for c in range(3)]
    N = 2 * n
    v = rng.normal(0, 0.05, size=(3, N))
    u = 1.0 + 0.1 * rng.uniform(size=N)
    kw = dict(gamma=5 / 3, box=(1.0, 1.0, 1.0), periodic=(0, 0, 0))
    both = W.Workload(name="two", x=X[0], y=X[1], z=X[2], m=np.full(N, sp ** 3), vx=v[0], vy=v[1], vz=v[2],
                      u=u, **kw)
    ga, gb = both.subset(np.arange(n)), both.subset(np.arange(n, N))
    # no pair crosses between the groups at any stage: the gap exceeds every kernel length
    s = O.Setup.of(both, cell=0.0)
    H, _, _, _ = O.solve_h(s, both.x, both.y, both.z)
    gap = np.sqrt(((np.stack(a, 1)[:, None, :] - np.stack(b, 1)[None, :, :]) ** 2).sum(-1)).min()
    assert gap > 2.0 * H.max()
    T = 0.01
    h = O.Stepper(both, u_floor=0.0)
    h.set_bins(np.concatenate([np.zeros(n, dtype=np.int64), np.ones(n, dtype=np.int64)]))
    h.hier_step(T)
    ra = O.Stepper(ga, u_floor=0.0)
    ra.start()
    ra.step(T)
    rb = O.Stepper(gb, u_floor=0.0)
    rb.start()
    rb.step(0.5 * T)
    rb.step(0.5 * T)
    for k in ("x", "y", "z", "vx", "vy", "vz", "u"):
        got = h.st[k]
        want = np.concatenate([ra.st[k], rb.st[k]])
        scale = np.abs(want).max() if k in ("x", "y", "z", "u") else np.abs(v).max()
        assert np.abs(got - want).max() <= 1e-13 * scale, k
    # and the coarse group's velocities moved (the check is not vacuous)
    assert np.abs(ra.st["vx"] - ga.vx).max() > 1e-6


def _rk4(w, nsteps=32):
    s = O.Setup.of(w)
    L = np.array(w.box)[:, None]
    m = w.m

    def rates(X, Pm, E):
        v = Pm / m
        u = E / m - 0.5 * (v * v).sum(0)
        Xw = X - L * np.floor(X / L)
        out = O.hydro_pass(s, dict(x=Xw[0], y=Xw[1], z=Xw[2], m=m, vx=v[0], vy=v[1], vz=v[2], u=u))
        return v, out["dp"], out["dE"]

    V0 = np.stack([w.vx, w.vy, w.vz])
    Y = [np.stack([w.x, w.y, w.z]), m * V0, m * (w.u + 0.5 * (V0 * V0).sum(0))]
    h = T_END / nsteps
    for _ in range(nsteps):
        k1 = rates(*Y)
        k2 = rates(*[y + 0.5 * h * k for y, k in zip(Y, k1)])
        k3 = rates(*[y + 0.5 * h * k for y, k in zip(Y, k2)])
        k4 = rates(*[y + h * k for y, k in zip(Y, k3)])
        Y = [y + h / 6.0 * (a + 2.0 * b + 2.0 * c + d) for y, a, b, c, d in zip(Y, k1, k2, k3, k4)]
    return Y


@pytest.mark.parametrize("levels", [2, 3])
def test_hierarchical_step_converges_at_second_order(smooth_box, levels):
    w = smooth_box
    Y = _rk4(w)
    bins = np.minimum((w.x * levels).astype(np.int64), levels - 1)
    L = np.array(w.box)[:, None]

    def err(nsys):
        s = O.Stepper(w, u_floor=0.0)
        s.set_bins(bins)
        for _ in range(nsys):
            s.hier_step(T_END / nsys)
        q = s.st
        V = np.stack([q["vx"], q["vy"], q["vz"]])
        got = [np.stack([q["x"], q["y"], q["z"]]), q["m"] * V, q["m"] * (q["u"] + 0.5 * (V * V).sum(0))]
        dX = got[0] - Y[0]
        dX -= L * np.round(dX / L)
        return np.array([np.abs(dX).max()] + [np.abs(g - y).max() / np.abs(y).max() for g, y in zip(got[1:], Y[1:])])

    e2, e4 = err(2), err(4)
    print("hierarchical", levels, e2, e4, e2 / e4)
    assert np.all(e2 / e4 > 3.0), (e2, e4)
    assert np.all(e4 < 1e-3), e4


# ------------------------------------------------------------------ R26
# Active subsets: a sub-step's pass recomputes kernel lengths, densities,
# volumes, gradient matrices and limited gradients only for the particles of
# the due bins; the others keep those of their last active boundary.


def test_active_subsets_with_every_particle_due_are_the_full_passes_bitwise(smooth_box):
    """Every particle in bin 1 of two levels: each boundary has all of them
    active, so the masked solve and gradients and the densities and pressures
    rebuilt from n give the full passes bit for bit."""
    w = smooth_box
    bins = np.ones(w.n, dtype=np.int64)
    a = O.Stepper(w, u_floor=0.0)
    a.set_bins(bins)
    b = O.Stepper(w, u_floor=0.0)
    b.set_bins(bins)
    for _ in range(2):
        a.hier_step(0.004)
        b.hier_step(0.004, active=True)
    for k in a.st:
        assert np.array_equal(a.st[k], b.st[k]), k
    assert np.array_equal(a.lev, b.lev)


def test_active_subsets_recompute_the_due_bins_and_keep_the_rest(smooth_box):
    """Along one system step of three levels: at each boundary with lmin > 0,
    an active particle's H, n and V equal an independent solve at that
    boundary's positions (a cold start, no mask) and its gradient matrix equals
    an independent gradient pass on those; an inactive particle's H, n, V, B and
    limited gradients are bit for bit those of its last active boundary."""
    w = smooth_box
    bins = np.minimum((w.x * 3).astype(np.int64), 2)
    s = O.Stepper(w, u_floor=0.0)
    first = s.set_bins(bins)
    last = {k: np.array(first[k], copy=True) for k in O.FROZEN}
    trace = []
    s.hier_step(0.004, active=True, trace=trace)
    checked = 0
    for t in trace:
        lmin = t["lmin"]
        act = bins >= lmin
        if lmin > 0:
            assert 0 < act.sum() < w.n
            H, nk, V, _ = O.solve_h(s.s, t["x"], t["y"], t["z"])
            for k, ref in (("H", H), ("nk", nk), ("V", V)):
                assert np.abs(t[k][act] - ref[act]).max() <= 1e-11 * np.abs(ref).max(), k
            g = O.gradients(s.s, dict(t, m=s.st["m"]), H, nk, V)
            assert np.abs(t["B"][:, act] - g["B"][:, act]).max() <= 1e-9 * np.abs(g["B"]).max()
            for k in O.FROZEN:
                assert np.array_equal(t[k][..., ~act], last[k][..., ~act]), k
            checked += 1
        for k in O.FROZEN:
            last[k][..., act] = t[k][..., act]
    assert checked == 3   # boundaries 1, 2 and 3 of 4


@pytest.mark.parametrize("levels", [2, 3])
def test_active_subsets_conserve_and_differ_from_full_passes(smooth_box, levels):
    w = smooth_box
    bins = np.minimum((w.x * levels).astype(np.int64), levels - 1)
    a = O.Stepper(w, u_floor=0.0)
    a.set_bins(bins)
    b = O.Stepper(w, u_floor=0.0)
    b.set_bins(bins)
    p0, E0, _ = _totals(b.st)
    for _ in range(2):
        a.hier_step(0.004)
        b.hier_step(0.004, active=True)
    p1, E1, scale = _totals(b.st)
    assert np.abs(p1 - p0).max() <= 1e-14 * scale.max()
    assert E1 == pytest.approx(E0, rel=1e-14)
    # the kept values enter the fluxes: the result is not R25's
    assert np.abs(a.st["vx"] - b.st["vx"]).max() > 1e-6


def test_active_subsets_two_groups_without_common_pairs():
    """The decoupled groups of the R25 pin with active subsets: the coarse
    group, inactive at the middle boundary, has no due pair there, so each
    group still follows its own global steps."""
    rng = np.random.default_rng(43)
    sp = 0.04
    a = _clump((0.1, 0.1, 0.1), 6, sp, rng)
    b = _clump((0.62, 0.62, 0.62), 6, sp, rng)
    n = a[0].size
    X = [np.concatenate([a[c], b[c]]) for c in range(3)]
    N = 2 * n
    v = rng.normal(0, 0.05, size=(3, N))
    u = 1.0 + 0.1 * rng.uniform(size=N)
    kw = dict(gamma=5 / 3, box=(1.0, 1.0, 1.0), periodic=(0, 0, 0))
    both = W.Workload(name="two", x=X[0], y=X[1], z=X[2], m=np.full(N, sp ** 3), vx=v[0], vy=v[1], vz=v[2],
                      u=u, **kw)
    ga, gb = both.subset(np.arange(n)), both.subset(np.arange(n, N))
    T = 0.01
    h = O.Stepper(both, u_floor=0.0)
    h.set_bins(np.concatenate([np.zeros(n, dtype=np.int64), np.ones(n, dtype=np.int64)]))
    h.hier_step(T, active=True)
    ra = O.Stepper(ga, u_floor=0.0)
    ra.start()
    ra.step(T)
    rb = O.Stepper(gb, u_floor=0.0)
    rb.start()
    rb.step(0.5 * T)
    rb.step(0.5 * T)
    for k in ("x", "y", "z", "vx", "vy", "vz", "u"):
        got = h.st[k]
        want = np.concatenate([ra.st[k], rb.st[k]])
        scale = np.abs(want).max() if k in ("x", "y", "z", "u") else np.abs(v).max()
        assert np.abs(got - want).max() <= 1e-13 * scale, k


@pytest.mark.parametrize("levels", [2, 3])
def test_active_subsets_converge(smooth_box, levels):
    """Against RK4 of the semi-discrete system: a kept kernel length or
    gradient lags its particle's drift by less than one of its own steps, an
    error of first order that is small beside the scheme's second-order one
    at these steps; halving the system step cuts the error by more than 2.5
    (3.5 to 4.6 measured)."""
    w = smooth_box
    Y = _rk4(w)
    bins = np.minimum((w.x * levels).astype(np.int64), levels - 1)
    L = np.array(w.box)[:, None]

    def err(nsys):
        s = O.Stepper(w, u_floor=0.0)
        s.set_bins(bins)
        for _ in range(nsys):
            s.hier_step(T_END / nsys, active=True)
        q = s.st
        V = np.stack([q["vx"], q["vy"], q["vz"]])
        got = [np.stack([q["x"], q["y"], q["z"]]), q["m"] * V, q["m"] * (q["u"] + 0.5 * (V * V).sum(0))]
        dX = got[0] - Y[0]
        dX -= L * np.round(dX / L)
        return np.array([np.abs(dX).max()] + [np.abs(g - y).max() / np.abs(y).max() for g, y in zip(got[1:], Y[1:])])

    e2, e4 = err(2), err(4)
    print("active subsets", levels, e2, e4, e2 / e4)
    assert np.all(e2 / e4 > 2.5), (e2, e4)
    assert np.all(e4 < 1e-3), e4
