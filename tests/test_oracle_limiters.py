"""Pins of the oracle's optional limiters (no GPU): the pairwise face limiter
(R23) and the condition-adaptive limiter constant (R24), by closed forms and
by the properties they exist for (positive face states, untouched linear
fields, conservation)."""
import dataclasses
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1712_01294_amd import workloads as W

PSI1, PSI2 = 0.5, 0.25


@pytest.mark.parametrize("f,pk,po,want", [
    # side K below the other particle: at most the midpoint + psi2 D, at least lo - psi1 D
    (5.0, 1.0, 3.0, 2.0 + PSI2 * 2.0),
    (-9.0, 2.0, 3.0, 2.0 - PSI1 * 1.0),
    # lo - psi1 D = 0 would not keep a positive field positive: lo / (1 + psi1 D / |lo|)
    (-9.0, 1.0, 3.0, 1.0 / (1.0 + PSI1 * 2.0 / 1.0)),
    (1.7, 1.0, 3.0, 1.7),                       # inside the bounds: untouched
    # side K above: at least the midpoint - psi2 D, at most hi + psi1 D
    (0.0, 3.0, 1.0, 2.0 - PSI2 * 2.0),
    (9.0, 3.0, 1.0, 3.0 + PSI1 * 2.0),
    # lo - psi1 D would change the sign of lo: lo / (1 + psi1 D / |lo|) instead
    (-2.0, 0.1, 3.0, 0.1 / (1.0 + PSI1 * 2.9 / 0.1)),
    # negative field: hi + psi1 D would turn positive
    (5.0, -0.1, -1.1, -0.1 / (1.0 + PSI1 * 1.0 / 0.1)),
    # equal centre values: the centre value
    (7.0, 2.0, 2.0, 2.0),
])
def test_pair_limit_closed_forms(oracle_lib, f, pk, po, want):
    assert O.pair_limit(f, pk, po) == pytest.approx(want, rel=1e-15, abs=1e-300)


def test_limiter_beta_interpolates_in_log_condition_number(oracle_lib):
    s = O.Setup(gamma=5 / 3, n_ngb=32, box=(1, 1, 1), periodic=(1, 1, 1), beta=0.6, limiter=1,
                beta_min=0.2, cond_lo=1.0, cond_hi=9.0)
    assert O.limiter_beta(s, 0.5) == 0.6
    assert O.limiter_beta(s, 1.0) == 0.6
    assert O.limiter_beta(s, 3.0) == pytest.approx(0.4, rel=1e-15)
    assert O.limiter_beta(s, 9.0) == pytest.approx(0.2, rel=1e-15)
    assert O.limiter_beta(s, 1e6) == pytest.approx(0.2, rel=1e-15)
    assert O.limiter_beta(s, float("nan")) == pytest.approx(0.2, rel=1e-15)
    assert O.limiter_beta(dataclasses.replace(s, limiter=0), 3.0) == 0.6


def test_adaptive_beta_closed_form_on_the_lattice(oracle_lib):
    """Interior of an open perfect lattice: E = e I, so cond(E) = ||E||_F ||E^-1||_F
    = 3 exactly.  With beta 0.6 at cond <= 1 and 0.2 at cond >= 9, R24 gives 0.4
    (half way in log cond), and a linear field along x limits to
    alpha = 0.4 * D / (sqrt(3) D / 2)."""
    nside = 16
    x, y, z = W.lattice_sites(nside, nside, nside, 1.0 / nside)
    n = x.size
    g = 0.7
    w = W.Workload(name="lat", x=x, y=y, z=z, m=np.ones(n), vx=g * x, vy=np.zeros(n), vz=np.zeros(n),
                   u=np.ones(n), gamma=5 / 3, box=(1, 1, 1), periodic=(0, 0, 0))
    s = O.Setup.of(w, cell=0.0, beta=0.6, limiter=1, beta_min=0.2, cond_lo=1.0, cond_hi=9.0)
    H, nk, V, _ = O.solve_h(s, w.x, w.y, w.z)
    gr = O.gradients(s, w.arrays(), H, nk, V)
    inner = np.all(np.stack([x, y, z]) > 2.4 / nside, 0) & np.all(np.stack([x, y, z]) < 1 - 2.4 / nside, 0)
    assert np.abs(gr["cond"][inner] - 3.0).max() < 1e-12
    want = 0.4 * 2.0 / math.sqrt(3.0)
    assert np.abs(gr["alpha"][1][inner] - want).max() < 1e-12
    # without R24 the same set keeps beta = 0.6
    s0 = dataclasses.replace(s, limiter=0)
    gr0 = O.gradients(s0, w.arrays(), H, nk, V)
    assert np.abs(gr0["alpha"][1][inner] - 0.6 * 2.0 / math.sqrt(3.0)).max() < 1e-12


@pytest.fixture(scope="module")
def steep():
    """A clustered set with pressure contrasts large enough that linear
    extrapolation gives non-positive face states on many faces."""
    return W.clustered(n_side=16, seed=W.SEED_BASE + 160)


@pytest.mark.parametrize("scheme", ["mfm", "mfv"])
def test_pairwise_limiter_keeps_face_states_positive_and_conserves(oracle_lib, steep, scheme):
    w = steep
    s0 = dataclasses.replace(O.Setup.of(w), scheme=scheme)
    s1 = dataclasses.replace(s0, limiter=1)
    off = O.hydro_pass(s0, w.arrays())
    on = O.hydro_pass(s1, w.arrays())
    assert off["fallbacks"] > 0
    assert on["fallbacks"] == 0
    assert np.array_equal(off["H"], on["H"])
    eps = np.finfo(np.float64).eps
    for c in range(3):
        assert abs(on["dp"][c].sum()) <= 10 * eps * np.abs(on["dp"][c]).sum()
    assert abs(on["dE"].sum()) <= 10 * eps * np.abs(on["dE"]).sum()
    if scheme == "mfv":
        assert abs(on["dm"].sum()) <= 10 * eps * np.abs(on["dm"]).sum()


def test_pairwise_limiter_leaves_linear_fields_alone(oracle_lib):
    """Linear fields on an open perfect lattice: every interior face value is
    the midpoint interpolant, inside R23's bounds, and R24 keeps beta = 1
    (beta_min = 1), so deep-interior particles get the same fluxes bit for bit
    with and without the optional limiters."""
    rng = np.random.default_rng(8)
    nside = 16
    x, y, z = W.lattice_sites(nside, nside, nside, 1.0 / nside)
    n = x.size
    w = W.Workload(name="lat", x=x, y=y, z=z, m=np.ones(n), vx=np.zeros(n), vy=np.zeros(n),
                   vz=np.zeros(n), u=np.ones(n), gamma=5 / 3, box=(1, 1, 1), periodic=(0, 0, 0))
    s0 = O.Setup.of(w, cell=0.0)
    H, nk, V, _ = O.solve_h(s0, w.x, w.y, w.z)
    X = np.stack([x, y, z], 1)
    gv = 0.5 * rng.normal(size=(5, 3))
    phi = np.array([5.0, 0.2, -0.1, 0.4, 8.0])[None, :] + X @ gv.T
    assert phi[:, 0].min() > 0 and phi[:, 4].min() > 0
    st = dict(x=x, y=y, z=z, m=phi[:, 0] / nk, vx=phi[:, 1], vy=phi[:, 2], vz=phi[:, 3],
              u=phi[:, 4] / ((s0.gamma - 1) * phi[:, 0]))
    deep = np.all(X > 4.6 / nside, 1) & np.all(X < 1 - 4.6 / nside, 1)
    assert deep.sum() == 6 ** 3
    a = O.hydro_pass(s0, st)
    b = O.hydro_pass(dataclasses.replace(s0, limiter=1), st)
    for k in ("dp", "dE"):
        assert np.array_equal(a[k][..., deep], b[k][..., deep]), k
