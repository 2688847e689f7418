"""Pin of the oracle's MFM kick-drift-kick step (R17) against an independent
integrator of the same semi-discrete system (no GPU).

The pass defines dx/dt = v, d(m v)/dt = dp, dE/dt = dE with constant masses,
v = p/m and u = E/m - |v|^2/2.  Classical RK4 on that system with small steps
is the reference.  A kick-drift-kick step with a predicted state is second
order, so halving dt must cut its error by about 4.  A predictor or drift of
the wrong order (a full-step predicted kick, a drift with the start-of-step
velocity) is first order and cuts it by about 2; the controls below plant
those mistakes in a copy of the step and show that the check separates them.
"""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_1712_01294_amd import workloads as W

T = 0.02


@pytest.fixture(scope="module")
def smooth_box():
    """8^3 jittered box with smooth velocities of amplitude 0.5 (sound speed
    about 1.3), so the limiter and the first-order fallback rarely switch."""
    w0 = W.jittered_sine(n_side=8, seed=W.SEED_BASE + 61)
    tp = 2.0 * np.pi
    w = dataclasses.replace(w0, vx=0.5 * np.sin(tp * w0.y), vy=0.5 * np.sin(tp * w0.z),
                            vz=0.5 * np.sin(tp * w0.x))
    return w


def _rk4_reference(w, nsteps=32):
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
    h = T / nsteps
    for _ in range(nsteps):
        k1 = rates(*Y)
        k2 = rates(*[y + 0.5 * h * k for y, k in zip(Y, k1)])
        k3 = rates(*[y + 0.5 * h * k for y, k in zip(Y, k2)])
        k4 = rates(*[y + h * k for y, k in zip(Y, k3)])
        Y = [y + h / 6.0 * (a + 2.0 * b + 2.0 * c + d) for y, a, b, c, d in zip(Y, k1, k2, k3, k4)]
    return Y


@pytest.fixture(scope="module")
def reference(smooth_box):
    return _rk4_reference(smooth_box)


class _Planted(O.Stepper):
    """The MFM step written out again with two knobs: the fraction of dt in the
    predicted kick (1/2 is correct) and the velocity of the drift (the
    half-step one is correct).  With the correct knobs it must equal the
    oracle's own step bit for bit (checked below)."""

    def __init__(self, w, pred=0.5, drift="half"):
        super().__init__(w, u_floor=0.0)
        self.pred, self.drift = pred, drift

    def step(self, dt=None):
        if self.last is None:
            self.start()
        st, last = self.st, self.last
        m = st["m"]
        v0 = [st[k] for k in ("vx", "vy", "vz")]
        E = m * (st["u"] + 0.5 * (v0[0] ** 2 + v0[1] ** 2 + v0[2] ** 2))
        v = [v0[c] + 0.5 * dt * last["dp"][c] / m for c in range(3)]
        E = E + 0.5 * dt * last["dE"]
        x = self._drift(v if self.drift == "half" else v0, dt)
        vp = [v[c] + self.pred * dt * last["dp"][c] / m for c in range(3)]
        Ep = E + self.pred * dt * last["dE"]
        up = np.maximum(Ep / m - 0.5 * (vp[0] ** 2 + vp[1] ** 2 + vp[2] ** 2), self.u_floor)
        out = self._pass(x[0], x[1], x[2], vp[0], vp[1], vp[2], up)
        v = [v[c] + 0.5 * dt * out["dp"][c] / m for c in range(3)]
        E = E + 0.5 * dt * out["dE"]
        u = np.maximum(E / m - 0.5 * (v[0] ** 2 + v[1] ** 2 + v[2] ** 2), self.u_floor)
        st.update(x=x[0], y=x[1], z=x[2], vx=v[0], vy=v[1], vz=v[2], u=u)
        self.last = out
        return dt


def _kdk_error(w, Y, nsteps, make=None):
    st = make(w) if make else O.Stepper(w, u_floor=0.0)
    st.start()
    for _ in range(nsteps):
        st.step(T / nsteps)
    q = st.st
    L = np.array(w.box)[:, None]
    V = np.stack([q["vx"], q["vy"], q["vz"]])
    got = [np.stack([q["x"], q["y"], q["z"]]), q["m"] * V, q["m"] * (q["u"] + 0.5 * (V * V).sum(0))]
    dX = got[0] - Y[0]
    dX -= L * np.round(dX / L)
    return np.array([np.abs(dX).max()] + [np.abs(g - y).max() / np.abs(y).max()
                                           for g, y in zip(got[1:], Y[1:])])


def test_mfm_step_converges_at_second_order_to_the_semi_discrete_solution(smooth_box, reference):
    """e(dt) / e(dt/2) > 3 on positions, momenta and energies: second order."""
    e4, e8 = _kdk_error(smooth_box, reference, 4), _kdk_error(smooth_box, reference, 8)
    print("mfm kdk errors", e4, e8, e4 / e8)
    assert np.all(e4 / e8 > 3.0), (e4, e8)
    assert np.all(e8 < 1e-3), e8
    assert np.array_equal(_kdk_error(smooth_box, reference, 4, make=lambda w: _Planted(w)), e4)


@pytest.mark.parametrize("knobs", [dict(pred=1.0), dict(drift="start")])
def test_planted_first_order_steps_fail_the_convergence_check(smooth_box, reference, knobs):
    """Controls: the same check on a step with a full-dt predicted kick, or a
    drift with the start-of-step velocity, sees first-order convergence."""
    make = lambda w: _Planted(w, **knobs)
    e4, e8 = _kdk_error(smooth_box, reference, 4, make), _kdk_error(smooth_box, reference, 8, make)
    print("planted", knobs, e4 / e8)
    assert not np.all(e4 / e8 > 3.0), (knobs, e4, e8)
