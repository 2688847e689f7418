"""Python driver of the plain C FP64 oracle (``mfm_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline leg of the benchmark, never by the product path.

The release paper names a Lagrangian mesh-free finite-volume Godunov method
whose mesh moves with the fluid (abstract; "Arbitrary (Moving) Meshes").
The pass here follows the standard meshless finite-mass formulation it refers
to, in the numbered readings R1-R18 that the C file lists and the GPU
library's header shares: kernel length, gradient matrix and limited
gradients, faces, HLLC fluxes, accumulation, and the kick-drift-kick step
with a predicted state.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mfm_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")   # the same source built with -fopenmp

_dp = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)
_u8p = C.POINTER(C.c_uint8)


class OrParams(C.Structure):
    _fields_ = [("gamma", C.c_double), ("n_ngb", C.c_double), ("box", C.c_double * 3),
                ("periodic", C.c_int32 * 3), ("beta", C.c_double), ("cond_max", C.c_double),
                ("cell", C.c_double), ("scheme", C.c_int32), ("limiter", C.c_int32),
                ("beta_min", C.c_double), ("cond_lo", C.c_double), ("cond_hi", C.c_double)]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no FMA contraction, no fast-math), once
    single-threaded and once with OpenMP over particles."""
    for lib_path, extra in ((LIB, []), (LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(lib_path) or os.path.getmtime(lib_path) < os.path.getmtime(SRC):
            tmp = lib_path + ".tmp%d" % os.getpid()
            subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
                                   "-D_GNU_SOURCE", "-Wno-unknown-pragmas", *extra, "-fPIC", "-shared",
                                   "-o", tmp, SRC, "-lm"])
            os.replace(tmp, lib_path)
    return LIB


_libs = {}
_omp = [False]


@contextlib.contextmanager
def openmp():
    """Within the block the oracle's passes run on its OpenMP build (all the
    threads OpenMP is given); results are bitwise those of the serial build."""
    prev = _omp[0]
    _omp[0] = True
    try:
        yield
    finally:
        _omp[0] = prev


def threads() -> int:
    """Threads the active build uses for a pass."""
    return int(lib().or_threads())


def lib():
    key = _omp[0]
    if key not in _libs:
        build()
        L = C.CDLL(LIB_OMP if key else LIB)
        L.or_kernel_W.restype = C.c_double
        L.or_kernel_W.argtypes = [C.c_double, C.c_double]
        L.or_kernel_dWdH.restype = C.c_double
        L.or_kernel_dWdH.argtypes = [C.c_double, C.c_double]
        L.or_find_neighbours.restype = C.c_int
        L.or_mark_within.restype = C.c_int
        L.or_solve_h.restype = C.c_int
        L.or_gradients.restype = C.c_int
        L.or_fluxes.restype = C.c_int
        L.or_fluxes_levels.restype = C.c_int
        L.or_hllc_star.restype = None
        L.or_face.restype = None
        L.or_mfv_flux.restype = None
        L.or_mfv_flux_moving.restype = None
        L.or_threads.restype = C.c_int
        L.or_pair_limit.restype = C.c_double
        L.or_pair_limit.argtypes = [C.c_double, C.c_double, C.c_double]
        L.or_limiter_beta.restype = C.c_double
        _libs[key] = L
    return _libs[key]


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(_dp if a.dtype == np.float64 else (_i64p if a.dtype == np.int64 else _u8p))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    pass


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"oracle {what} failed with status {rc}")


@dataclass
class Setup:
    """Physical parameters of one run."""

    gamma: float
    n_ngb: float
    box: tuple
    periodic: tuple
    beta: float = 1.0
    cond_max: float = 1.0e6
    cell: float = 0.0       # 0: brute-force neighbour search
    scheme: str = "mfm"     # "mfm" (zero mass flux) or "mfv" (full HLLC flux, mass changes)
    limiter: int = 0        # 1: pairwise face limiter (R23) and condition-adaptive beta (R24)
    beta_min: float = 1.0   # R24: beta at cond(E) >= cond_hi
    cond_lo: float = 10.0   # R24: beta applies at cond(E) <= cond_lo
    cond_hi: float = 1000.0

    @classmethod
    def of(cls, w, cell=None, **kw):
        if cell is None:
            # a bucket grid of about two mean spacings; 0 (brute force) for tiny sets
            vol = w.box[0] * w.box[1] * w.box[2]
            cell = 0.0 if w.n <= 5000 else 2.0 * (vol / w.n) ** (1.0 / 3.0)
        return cls(gamma=w.gamma, n_ngb=w.n_ngb, box=tuple(w.box), periodic=tuple(w.periodic),
                   cell=cell, **kw)

    def c(self) -> OrParams:
        p = OrParams()
        p.gamma = self.gamma
        p.n_ngb = self.n_ngb
        for a in range(3):
            p.box[a] = self.box[a]
            p.periodic[a] = int(self.periodic[a])
        p.beta = self.beta
        p.cond_max = self.cond_max
        p.cell = self.cell
        p.scheme = {"mfm": 0, "mfv": 1}[self.scheme]
        p.limiter = int(self.limiter)
        p.beta_min = self.beta_min
        p.cond_lo = self.cond_lo
        p.cond_hi = self.cond_hi
        return p


def kernel_W(r, H):
    return lib().or_kernel_W(float(r), float(H))


def kernel_dWdH(r, H):
    return lib().or_kernel_dWdH(float(r), float(H))


def find_neighbours(s: Setup, x, y, z, i, R, cap=100000):
    x, y, z = _f64(x), _f64(y), _f64(z)
    js = np.zeros(cap, dtype=np.int64)
    cnt = C.c_int64(0)
    p = s.c()
    _check(lib().or_find_neighbours(C.byref(p), C.c_int64(x.size), _p(x), _p(y), _p(z),
                                    C.c_int64(i), C.c_double(R), C.c_int64(cap), _p(js),
                                    C.byref(cnt)), "find_neighbours")
    return js[:cnt.value].copy()


def solve_h(s: Setup, x, y, z, H_guess=None, mask=None):
    x, y, z = _f64(x), _f64(y), _f64(z)
    n = x.size
    H = np.zeros(n) if H_guess is None else _f64(H_guess).copy()
    nk = np.zeros(n)
    V = np.zeros(n)
    it = np.zeros(n, dtype=np.int64)
    mk = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    p = s.c()
    _check(lib().or_solve_h(C.byref(p), C.c_int64(n), _p(x), _p(y), _p(z), _p(mk), _p(H),
                            _p(nk), _p(V), _p(it)), "solve_h")
    return H, nk, V, it


def gradients(s: Setup, st: dict, H, nk, V, mask=None):
    n = st["x"].size
    a = {k: _f64(st[k]) for k in ("x", "y", "z", "m", "vx", "vy", "vz", "u")}
    H, nk, V = _f64(H), _f64(nk), _f64(V)
    B = np.zeros(6 * n)
    rho = np.zeros(n)
    P = np.zeros(n)
    grad = np.zeros(15 * n)
    graw = np.zeros(15 * n)
    alpha = np.zeros(5 * n)
    cond = np.zeros(n)
    nill = C.c_int64(0)
    mk = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    p = s.c()
    _check(lib().or_gradients(C.byref(p), C.c_int64(n), _p(a["x"]), _p(a["y"]), _p(a["z"]),
                              _p(a["m"]), _p(a["vx"]), _p(a["vy"]), _p(a["vz"]), _p(a["u"]),
                              _p(H), _p(nk), _p(V), _p(mk), _p(B), _p(rho), _p(P), _p(grad),
                              _p(graw), _p(alpha), _p(cond), C.byref(nill)), "gradients")
    return dict(B=B.reshape(6, n), rho=rho, P=P, grad=grad.reshape(15, n),
                grad_raw=graw.reshape(15, n), alpha=alpha.reshape(5, n), cond=cond,
                n_illcond=int(nill.value))


def fluxes(s: Setup, st: dict, H, V, g: dict, mask=None, hmax=None, bins=None, lmin=0, lev=None):
    """Fluxes of every flux pair (R9-R16); with bins (R25) only the pairs of
    level >= lmin, their per-level sums written into lev (5, nlev, n), in place."""
    n = st["x"].size
    a = {k: _f64(st[k]) for k in ("x", "y", "z", "vx", "vy", "vz")}
    H, V = _f64(H), _f64(V)
    B = _f64(g["B"]).ravel()
    grad = _f64(g["grad"]).ravel()
    rho, P = _f64(g["rho"]), _f64(g["P"])
    dp = np.zeros(3 * n)
    dE = np.zeros(n)
    dm = np.zeros(n)
    vsig = np.zeros(n)
    counts = np.zeros(3, dtype=np.int64)
    mk = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    if hmax is None:
        hmax = float(np.max(H if mask is None else H[H > 0]))
    p = s.c()
    if bins is None:
        _check(lib().or_fluxes(C.byref(p), C.c_int64(n), _p(a["x"]), _p(a["y"]), _p(a["z"]),
                               _p(a["vx"]), _p(a["vy"]), _p(a["vz"]), _p(H), _p(V), _p(B),
                               _p(rho), _p(P), _p(grad), _p(mk), C.c_double(hmax), _p(dp),
                               _p(dE), _p(vsig), _p(counts), _p(dm)), "fluxes")
    else:
        b = np.ascontiguousarray(bins, dtype=np.int64)
        assert lev.dtype == np.float64 and lev.flags.c_contiguous and lev.ndim == 3 and lev.shape[1] == 5
        assert lev.shape[0] >= int(b.max()) + 1 and lev.shape[2] == n
        _check(lib().or_fluxes_levels(C.byref(p), C.c_int64(n), _p(a["x"]), _p(a["y"]), _p(a["z"]),
                                      _p(a["vx"]), _p(a["vy"]), _p(a["vz"]), _p(H), _p(V), _p(B),
                                      _p(rho), _p(P), _p(grad), _p(mk), C.c_double(hmax), _p(dp),
                                      _p(dE), _p(vsig), _p(counts), _p(dm), _p(b), C.c_int64(lmin),
                                      C.c_int64(lev.shape[0]), _p(lev)), "fluxes")
    return dict(dp=dp.reshape(3, n), dE=dE, dm=dm, vsig=vsig, pair_entries=int(counts[0]),
                fallbacks=int(counts[1]), clamps=int(counts[2]))


def hydro_pass(s: Setup, st: dict, H_guess=None, bins=None, lmin=0, lev=None):
    """Full pass on every particle: kernel lengths, gradients, fluxes (with bins,
    the fluxes of the due levels only, R25; see fluxes)."""
    H, nk, V, it = solve_h(s, st["x"], st["y"], st["z"], H_guess)
    g = gradients(s, st, H, nk, V)
    f = fluxes(s, st, H, V, g, bins=bins, lmin=lmin, lev=lev)
    out = dict(H=H, nk=nk, V=V, iters=it)
    out.update(g)
    out.update(f)
    out["pairs"] = f["pair_entries"] // 2
    return out


def hllc_star(gamma, left, right):
    """(S*, P*) of the HLLC solver with Davis speeds for 1D states (rho, u, P)."""
    Ss, Ps = C.c_double(0), C.c_double(0)
    lib().or_hllc_star(C.c_double(gamma), C.c_double(left[0]), C.c_double(left[1]),
                       C.c_double(left[2]), C.c_double(right[0]), C.c_double(right[1]),
                       C.c_double(right[2]), C.byref(Ss), C.byref(Ps))
    return Ss.value, Ps.value


def mfv_flux(gamma, left, right):
    """MFV flux (mass, momentum, energy per unit area, lab frame) between 1D
    states (rho, u, P) along +x through a face moving with (u_L + u_R)/2."""
    F = np.zeros(3)
    lib().or_mfv_flux(C.c_double(gamma), C.c_double(left[0]), C.c_double(left[1]),
                      C.c_double(left[2]), C.c_double(right[0]), C.c_double(right[1]),
                      C.c_double(right[2]), _p(F))
    return F


def mfv_flux_moving(gamma, v_particles, left, right):
    """MFV flux between 1D face states (rho, u, P) along +x when the two
    particles move with v_particles = (vL, vR), so the face moves with their
    mean; the face states come from the reconstruction."""
    F = np.zeros(3)
    lib().or_mfv_flux_moving(C.c_double(gamma), C.c_double(v_particles[0]), C.c_double(v_particles[1]),
                             C.c_double(left[0]), C.c_double(left[1]), C.c_double(left[2]),
                             C.c_double(right[0]), C.c_double(right[1]), C.c_double(right[2]), _p(F))
    return F


def pair_limit(f, pk, po):
    """R23 on one face value f extrapolated by side K (centre pk; other side po)."""
    return lib().or_pair_limit(float(f), float(pk), float(po))


def limiter_beta(s: Setup, cond):
    """R24: the per-particle limiter constant at condition number cond."""
    p = s.c()
    return lib().or_limiter_beta(C.byref(p), C.c_double(cond))


def face(Ha, Va, Ba6, Hb, Vb, Bb6, d):
    A = np.zeros(3)
    Ba6, Bb6, d = _f64(Ba6), _f64(Bb6), _f64(d)
    lib().or_face(C.c_double(Ha), C.c_double(Va), _p(Ba6), C.c_double(Hb), C.c_double(Vb),
                  _p(Bb6), _p(d), _p(A))
    return A


# --------------------------------------------------------------------------
# Sampled evaluation: outputs for a few target particles of a large set.
# The flux of i needs gradients on its flux set, which need kernel lengths on
# their gather sets; the closure below walks that dependency outwards.
# --------------------------------------------------------------------------
def _ball_mask(s: Setup, st, seeds, radius: float):
    x, y, z = (_f64(st[k]) for k in ("x", "y", "z"))
    sd = np.ascontiguousarray(seeds, dtype=np.uint8)
    mark = np.zeros(x.size, dtype=np.uint8)
    p = s.c()
    _check(lib().or_mark_within(C.byref(p), C.c_int64(x.size), _p(x), _p(y), _p(z), _p(sd),
                                C.c_double(radius), _p(mark)), "mark_within")
    return mark.astype(bool)


def sampled_pass(s: Setup, st: dict, targets, h_bound: float):
    """Oracle outputs at ``targets`` only.  ``h_bound`` must bound every kernel
    length that can matter (the closure takes kernel lengths within
    2 h_bound of each target, gradients within h_bound)."""
    n = st["x"].size
    tmask = np.zeros(n, dtype=bool)
    tmask[np.asarray(targets)] = True
    gmask = _ball_mask(s, st, tmask, h_bound) | tmask
    hmask = _ball_mask(s, st, gmask, h_bound) | gmask
    H, nk, V, _ = solve_h(s, st["x"], st["y"], st["z"], None, mask=hmask)
    g = gradients(s, st, H, nk, V, mask=gmask)
    f = fluxes(s, st, H, V, g, mask=tmask, hmax=h_bound)
    out = dict(H=H, nk=nk, V=V)
    out.update(g)
    out.update(f)
    out["targets"] = np.flatnonzero(tmask)
    return out


# --------------------------------------------------------------------------
# R17/R18: kick-drift-kick step with a predicted state, one pass per step.
# what an inactive particle keeps between its active boundaries (R26)
FROZEN = ("H", "nk", "V", "B", "grad")


# --------------------------------------------------------------------------
class Stepper:
    """Plain FP64 time integration of the gas (global time step).  scheme "mfm"
    keeps every mass; scheme "mfv" (R21/R22) kicks mass, momentum and total
    energy as conserved quantities with the mass flux of the finite-volume form."""

    def __init__(self, w, cell=None, u_floor=None, scheme="mfm"):
        self.s = Setup.of(w, cell=cell)
        self.s.scheme = scheme
        self.cfl = w.cfl
        self.st = {k: _f64(getattr(w, k)).copy() for k in ("x", "y", "z", "m", "vx", "vy", "vz", "u")}
        self.u_floor = 1e-10 * float(np.mean(self.st["u"])) if u_floor is None else u_floor
        self.H = None
        self.last = None
        self.floors = 0
        self.bins = None
        self.lev = None
        self.frz = None

    def _pass(self, x, y, z, vx, vy, vz, u, m=None, lmin=None):
        st = dict(x=x, y=y, z=z, m=self.st["m"] if m is None else m, vx=vx, vy=vy, vz=vz, u=u)
        if lmin is None:
            out = hydro_pass(self.s, st, self.H)
        else:
            out = hydro_pass(self.s, st, self.H, bins=self.bins, lmin=lmin, lev=self.lev)
        self.H = out["H"]
        self.frz = {k: out[k] for k in FROZEN}
        return out

    def _pass_active(self, x, y, z, vx, vy, vz, u, lmin):
        """R26: the levelled pass of a sub-step boundary on which only the
        particles of bin >= lmin are active.  An active particle's kernel
        length (warm-started from its last one), number density, volume,
        gradient matrix and limited gradients are recomputed at the current
        positions and predicted state; an inactive particle keeps those of its
        last active boundary.  Every particle enters with its current position
        and predicted velocity and energy, its density m n and pressure
        (gamma - 1) rho u taken from its (recomputed or kept) n.  The flux set
        is r_ij < max(H_i, H_j) with these kernel lengths, and only the pairs
        of level >= lmin are evaluated, as in R25."""
        s, m, frz = self.s, self.st["m"], self.frz
        act = self.bins >= lmin
        st = dict(x=x, y=y, z=z, m=m, vx=vx, vy=vy, vz=vz, u=u)
        Hn, nkn, Vn, it = solve_h(s, x, y, z, frz["H"], mask=act)
        H = np.where(act, Hn, frz["H"])
        nk = np.where(act, nkn, frz["nk"])
        V = np.where(act, Vn, frz["V"])
        g = gradients(s, st, H, nk, V, mask=act)
        B = np.where(act, g["B"], frz["B"])
        grad = np.where(act, g["grad"], frz["grad"])
        rho = m * nk
        P = (s.gamma - 1.0) * rho * u
        f = fluxes(s, st, H, V, dict(B=B, grad=grad, rho=rho, P=P), bins=self.bins, lmin=lmin, lev=self.lev)
        out = dict(H=H, nk=nk, V=V, iters=it, B=B, grad=grad, rho=rho, P=P, active=act)
        out.update(f)
        out["pairs"] = f["pair_entries"] // 2
        self.H = H
        self.frz = {k: out[k] for k in FROZEN}
        return out

    # ---------------------------------------------------------------- R25
    def set_bins(self, bins, max_bin=None):
        """Power-of-two time bins (R25): particle i steps by T / 2^bins[i], with
        levels 0 .. max_bin (default the largest bin).  The per-level rates of
        the current state are (re)computed by a levelled pass on it: all
        levels due."""
        self.bins = np.ascontiguousarray(bins, dtype=np.int64)
        nlev = (int(self.bins.max()) if max_bin is None else int(max_bin)) + 1
        assert nlev >= int(self.bins.max()) + 1
        self.lev = np.zeros((nlev, 5, self.bins.size))
        st = self.st
        self.last = self._pass(st["x"], st["y"], st["z"], st["vx"], st["vy"], st["vz"], st["u"], lmin=0)
        return self.last

    def hier_step(self, T, active=False, trace=None):
        """One system step of length T with hierarchical power-of-two steps
        (R25; with active, R26: each sub-step's pass recomputes only the
        particles of the due bins, the others keeping what they had; with a
        list as trace, each sub-step's pass output is appended to it together
        with its boundary k, lmin and the positions and predicted state it
        ran on).  With B the largest bin, time advances in 2^B sub-steps of
        T / 2^B; every particle drifts with its current velocity on each.  A
        pair {i, j} has level l = max(bins) and step T / 2^l; at a sub-step
        boundary the levels whose step divides the time elapsed are due.  At
        each due boundary the pass evaluates the due pairs on the predicted
        state (velocities and energies advanced by the half kicks the due
        levels are about to receive, with their previous rates), then each due
        level's new rates close its pair step with a half kick and, before
        the end of T, open the next with another; both particles of a pair
        receive the same kick with opposite signs.  All levels are due at the
        start and at the end of T.  The MFM form: masses are constant."""
        assert self.s.scheme == "mfm" and self.lev is not None
        st, lev = self.st, self.lev
        m = st["m"]
        nlev = lev.shape[0]
        B = nlev - 1
        K = 1 << B
        delta = T / K
        dts = [T / (1 << l) for l in range(nlev)]
        v = [st[k] for k in ("vx", "vy", "vz")]
        E = m * (st["u"] + 0.5 * (v[0] ** 2 + v[1] ** 2 + v[2] ** 2))

        def kick(v, E, levels):
            for l in levels:
                v = [v[c] + 0.5 * dts[l] * lev[l, c] / m for c in range(3)]
                E = E + 0.5 * dts[l] * lev[l, 3]
            return v, E

        # opening half kicks of every level
        v, E = kick(v, E, range(nlev))
        x = [st["x"], st["y"], st["z"]]
        out = self.last
        for k in range(1, K + 1):
            # drift every particle by one sub-step, wrapped into the box
            st.update(x=x[0], y=x[1], z=x[2])
            x = self._drift(v, delta)
            tz = (k & -k).bit_length() - 1
            lmin = max(0, B - tz)
            due = range(lmin, nlev)
            # predicted state: the due levels' closing kicks with their previous rates
            vp, Ep = kick(v, E, due)
            up = Ep / m - 0.5 * (vp[0] ** 2 + vp[1] ** 2 + vp[2] ** 2)
            up = np.maximum(up, self.u_floor)
            if active and lmin > 0:
                out = self._pass_active(x[0], x[1], x[2], vp[0], vp[1], vp[2], up, lmin)
            else:
                out = self._pass(x[0], x[1], x[2], vp[0], vp[1], vp[2], up, lmin=lmin)
            if trace is not None:
                trace.append(dict(out, k=k, lmin=lmin, x=x[0], y=x[1], z=x[2], vx=vp[0], vy=vp[1], vz=vp[2],
                                  u=up))
            # closing half kicks of the due levels, then the opening ones of their next step
            v, E = kick(v, E, due)
            if k < K:
                v, E = kick(v, E, due)
        u = E / m - 0.5 * (v[0] ** 2 + v[1] ** 2 + v[2] ** 2)
        low = u < self.u_floor
        self.floors += int(np.count_nonzero(low))
        u = np.where(low, self.u_floor, u)
        st.update(x=x[0], y=x[1], z=x[2], vx=v[0], vy=v[1], vz=v[2], u=u)
        self.last = out
        return T

    def cfl_dt(self, out):
        return self.cfl * float(np.min(out["H"] / out["vsig"]))

    def start(self):
        st = self.st
        self.last = self._pass(st["x"], st["y"], st["z"], st["vx"], st["vy"], st["vz"], st["u"])
        return self.last

    def step(self, dt=None):
        if self.last is None:
            self.start()
        st, s, last = self.st, self.s, self.last
        if dt is None or dt <= 0:
            dt = self.cfl_dt(last)
        if self.s.scheme == "mfv":
            self._step_mfv(dt)
            return dt
        m = st["m"]
        # first half kick of momentum and total energy
        E = m * (st["u"] + 0.5 * (st["vx"] ** 2 + st["vy"] ** 2 + st["vz"] ** 2))
        v = [st[k] + 0.5 * dt * last["dp"][c] / m for c, k in enumerate(("vx", "vy", "vz"))]
        E = E + 0.5 * dt * last["dE"]
        # drift with the half-step velocity, wrapped into the box
        x = []
        for c, k in enumerate(("x", "y", "z")):
            xc = st[k] + dt * v[c]
            if s.periodic[c]:
                L = s.box[c]
                xc = xc - L * np.floor(xc / L)
                xc[xc >= L] = 0.0
            x.append(xc)
        # predicted state for the flux pass
        vp = [v[c] + 0.5 * dt * last["dp"][c] / m for c in range(3)]
        Ep = E + 0.5 * dt * last["dE"]
        up = Ep / m - 0.5 * (vp[0] ** 2 + vp[1] ** 2 + vp[2] ** 2)
        up = np.maximum(up, self.u_floor)
        out = self._pass(x[0], x[1], x[2], vp[0], vp[1], vp[2], up)
        # second half kick and recovery of u
        v = [v[c] + 0.5 * dt * out["dp"][c] / m for c in range(3)]
        E = E + 0.5 * dt * out["dE"]
        u = E / m - 0.5 * (v[0] ** 2 + v[1] ** 2 + v[2] ** 2)
        low = u < self.u_floor
        self.floors += int(np.count_nonzero(low))
        u = np.where(low, self.u_floor, u)
        st.update(x=x[0], y=x[1], z=x[2], vx=v[0], vy=v[1], vz=v[2], u=u)
        self.last = out
        return dt

    def _drift(self, v, dt):
        st, s = self.st, self.s
        x = []
        for c, k in enumerate(("x", "y", "z")):
            xc = st[k] + dt * v[c]
            if s.periodic[c]:
                L = s.box[c]
                xc = xc - L * np.floor(xc / L)
                xc[xc >= L] = 0.0
            x.append(xc)
        return x

    def _step_mfv(self, dt):
        """R22: kick-drift-kick of the conserved mass Q_m = m, momentum Q_p = m v
        and total energy Q_E = m (u + |v|^2/2) with the rates (dm, dp, dE) of
        the finite-volume pass; velocities and u are recovered as Q_p/Q_m and
        Q_E/Q_m - |v|^2/2 after each kick."""
        st, last = self.st, self.last
        m = st["m"]
        v = [st[k] for k in ("vx", "vy", "vz")]
        # first half kick of the conserved quantities
        Qm = m + 0.5 * dt * last["dm"]
        Qp = [m * v[c] + 0.5 * dt * last["dp"][c] for c in range(3)]
        QE = m * (st["u"] + 0.5 * (v[0] ** 2 + v[1] ** 2 + v[2] ** 2)) + 0.5 * dt * last["dE"]
        vh = [Qp[c] / Qm for c in range(3)]
        # drift with the half-step velocity, wrapped into the box
        x = self._drift(vh, dt)
        # predicted state for the flux pass, its masses included
        mp = Qm + 0.5 * dt * last["dm"]
        vp = [(Qp[c] + 0.5 * dt * last["dp"][c]) / mp for c in range(3)]
        up = (QE + 0.5 * dt * last["dE"]) / mp - 0.5 * (vp[0] ** 2 + vp[1] ** 2 + vp[2] ** 2)
        up = np.maximum(up, self.u_floor)
        out = self._pass(x[0], x[1], x[2], vp[0], vp[1], vp[2], up, m=mp)
        # second half kick and recovery of v and u
        Qm = Qm + 0.5 * dt * out["dm"]
        Qp = [Qp[c] + 0.5 * dt * out["dp"][c] for c in range(3)]
        QE = QE + 0.5 * dt * out["dE"]
        v = [Qp[c] / Qm for c in range(3)]
        u = QE / Qm - 0.5 * (v[0] ** 2 + v[1] ** 2 + v[2] ** 2)
        low = u < self.u_floor
        self.floors += int(np.count_nonzero(low))
        u = np.where(low, self.u_floor, u)
        st.update(x=x[0], y=x[1], z=x[2], m=Qm, vx=v[0], vy=v[1], vz=v[2], u=u)
        self.last = out
