"""Exact Riemann solver pins and the oracle's time step on a planar shock tube (no GPU)."""
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from oracle import riemann_exact as R
from paper_1712_01294_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")
LEFT = (1.0, 0.0, 1.0)
RIGHT = (0.125, 0.0, 0.1)


def _golden(name):
    vals = {}
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()[:2]
            vals[k] = float(v)
    return vals


def test_sod_textbook_values():
    g = _golden("riemann_sod.txt")
    p, u = R.star_state(LEFT, RIGHT, 1.4)
    rl, rr = R.star_densities(LEFT, RIGHT, 1.4)
    assert p == pytest.approx(g["pstar"], abs=6e-6)
    assert u == pytest.approx(g["ustar"], abs=6e-6)
    assert rl == pytest.approx(g["rhoL_star"], abs=6e-6)
    assert rr == pytest.approx(g["rhoR_star"], abs=6e-6)


def test_jump_conditions_gamma_five_thirds():
    """Right shock satisfies Rankine-Hugoniot; left fan is isentropic and keeps
    the Riemann invariant u + 2c/(gamma-1)."""
    gam = 5.0 / 3.0
    p, u = R.star_state(LEFT, RIGHT, gam)
    rl, rr = R.star_densities(LEFT, RIGHT, gam)
    S = R.wave_speeds(LEFT, RIGHT, gam)["right_shock"]
    r0, u0, p0 = RIGHT
    m0 = r0 * (u0 - S)
    m1 = rr * (u - S)
    assert m1 == pytest.approx(m0, rel=1e-13)
    assert r0 * (u0 - S) ** 2 + p0 == pytest.approx(rr * (u - S) ** 2 + p, rel=1e-13)
    e0 = p0 / ((gam - 1) * r0) + 0.5 * (u0 - S) ** 2 + p0 / r0
    e1 = p / ((gam - 1) * rr) + 0.5 * (u - S) ** 2 + p / rr
    assert e1 == pytest.approx(e0, rel=1e-13)
    assert p / rl ** gam == pytest.approx(LEFT[2] / LEFT[0] ** gam, rel=1e-13)
    cl0 = math.sqrt(gam * LEFT[2] / LEFT[0])
    cl1 = math.sqrt(gam * p / rl)
    assert u + 2 * cl1 / (gam - 1) == pytest.approx(LEFT[1] + 2 * cl0 / (gam - 1), rel=1e-13)


def test_sample_is_continuous_through_the_fan():
    gam = 5.0 / 3.0
    ws = R.wave_speeds(LEFT, RIGHT, gam)
    a, b = ws["left_head"], ws["left_tail"]
    e = 1e-9
    for s in (a, b):
        lo = R.sample(LEFT, RIGHT, gam, np.array([s - e]))
        hi = R.sample(LEFT, RIGHT, gam, np.array([s + e]))
        for k in range(3):
            assert lo[k][0] == pytest.approx(hi[k][0], rel=1e-6, abs=1e-8)


@pytest.fixture(scope="module")
def small_tube():
    w = W.shock_tube(n_yz=12, l_yz=12 / 64)
    st = O.Stepper(w)
    st.start()
    tot0 = dict(px=float((w.m * w.vx).sum()),
                E=float((w.m * (w.u + 0.5 * (w.vx ** 2 + w.vy ** 2 + w.vz ** 2))).sum()))
    t = 0.0
    for _ in range(40):
        t += st.step()
    return w, st, t, tot0


def test_tube_conserves_momentum_and_energy(small_tube):
    w, st, t, tot0 = small_tube
    s = st.st
    m = s["m"]
    E = float((m * (s["u"] + 0.5 * (s["vx"] ** 2 + s["vy"] ** 2 + s["vz"] ** 2))).sum())
    assert st.floors == 0
    assert abs(float((m * s["vx"]).sum()) - tot0["px"]) < 1e-14
    assert abs(float((m * s["vy"]).sum())) < 1e-14
    assert E == pytest.approx(tot0["E"], rel=1e-13)


def test_tube_tracks_exact_solution(small_tube):
    """Coarse convergence check (reported, not parity): between the contact and the
    shock the particles carry the exact star velocity, pressure and density to a few
    per cent, and the shock sits where the exact solution puts it."""
    w, st, t, _ = small_tube
    gam = w.gamma
    p, u = R.star_state(LEFT, RIGHT, gam)
    _, rr = R.star_densities(LEFT, RIGHT, gam)
    S = R.wave_speeds(LEFT, RIGHT, gam)["right_shock"]
    x = st.st["x"]
    lo = 1.0 + (u + 0.3 * (S - u)) * t
    hi = 1.0 + (S - 0.3 * (S - u)) * t
    sel = (x > lo) & (x < hi)
    assert sel.sum() > 50
    assert np.mean(st.st["vx"][sel]) == pytest.approx(u, rel=0.06)
    assert np.mean(st.last["P"][sel]) == pytest.approx(p, rel=0.10)
    assert np.mean(st.last["rho"][sel]) == pytest.approx(rr, rel=0.10)
    # shock position: half-way density crossing between rho*_R and rho_R
    xs = np.sort(x[(x > 1.0 + u * t) & (x < 1.5)])
    rho_s = st.last["rho"][np.argsort(x)][np.searchsorted(np.sort(x), xs)]
    mid = 0.5 * (rr + RIGHT[0])
    cross = xs[np.flatnonzero(rho_s < mid)[0]]
    dx = 2 * w.extra["spacing_right"]
    assert abs(cross - (1.0 + S * t)) < dx
