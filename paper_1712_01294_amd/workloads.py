"""Seeded synthetic particle sets for the MFM hydro pass.

This module only draws random numbers and lays out lattices: it holds none of
the method's arithmetic (no kernel, no density estimate, no flux).  Both the
HIP path and the CPU oracle take their inputs from here, so the two always see
identical arrays.

Every workload is a gas of equal-or-given-mass particles in a box, in the
setting of the release paper's hydrodynamics section (a Lagrangian mesh-free
finite-volume gas whose "mesh" moves with the fluid).  The paper measures only
full-physics cosmological runs on CPU clusters, with no public dataset; these
synthetic sets stand in for the five hydro-pass workloads:

* ``jittered_sine``   16^3 jittered lattice, rho = 1 + 0.1 sin(2 pi x), P ~ 1
* ``shock_tube``      planar Sod-type tube, density ratio 8 by spacing ratio 2, jittered
* ``turbulence``      128^3 jittered lattice, Gaussian k^-4 velocity, Mach 2
* ``clustered``       256^3 particles drawn from a log-normal density field
* ``adjoint_box``     the ``jittered_sine`` recipe at 64^3

Thermal energies are set from the *analytic* target density of each recipe
(not from a kernel estimate), so the generator never needs the method.
Random numbers come from numpy's PCG64 with seed ``SEED_BASE + index``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 171201294

FIELDS = ("x", "y", "z", "m", "vx", "vy", "vz", "u")


@dataclass
class Workload:
    """One synthetic particle set plus the run parameters it is meant for."""

    name: str
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    m: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    u: np.ndarray
    gamma: float
    box: tuple
    periodic: tuple = (1, 1, 1)
    n_ngb: float = 32.0
    cfl: float = 0.25
    dt: float = 0.0          # > 0: fixed step; 0: CFL step
    steps: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def arrays(self) -> dict:
        return {k: getattr(self, k) for k in FIELDS}

    def subset(self, idx) -> "Workload":
        kw = {k: np.ascontiguousarray(getattr(self, k)[idx]) for k in FIELDS}
        return Workload(name=self.name + "[subset]", gamma=self.gamma, box=self.box,
                        periodic=self.periodic, n_ngb=self.n_ngb, cfl=self.cfl,
                        dt=self.dt, steps=self.steps, extra=dict(self.extra), **kw)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def lattice_sites(nx: int, ny: int, nz: int, spacing: float, origin=(0.0, 0.0, 0.0)):
    """Cell-centred lattice sites (i + 1/2) * spacing, C order (x slowest)."""
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    x = origin[0] + (ix.ravel() + 0.5) * spacing
    y = origin[1] + (iy.ravel() + 0.5) * spacing
    z = origin[2] + (iz.ravel() + 0.5) * spacing
    return x.astype(np.float64), y.astype(np.float64), z.astype(np.float64)


def _wrap(a: np.ndarray, L: float) -> np.ndarray:
    a = np.mod(a, L)
    a[a >= L] = 0.0
    return a


def jittered_sine(n_side: int = 16, seed: int = SEED_BASE + 0, jitter: float = 0.2,
                  gamma: float = 5.0 / 3.0, sigma_v: float = 0.1, box: float = 1.0,
                  name: str = "jittered_sine") -> Workload:
    """Periodic box of side ``box`` with an ``n_side``^3 lattice of spacing box/n_side,
    each site moved by U(-jitter, jitter) spacings per axis.  Mass follows the
    target density rho(x) = 1 + 0.1 sin(2 pi x / box) at the particle, u is set so
    that (gamma-1) rho(x) u = 1, and each velocity component is N(0, sigma_v^2)."""
    rng = _rng(seed)
    d = box / n_side
    x, y, z = lattice_sites(n_side, n_side, n_side, d)
    j = rng.uniform(-jitter, jitter, size=(3, x.size)) * d
    x = _wrap(x + j[0], box)
    y = _wrap(y + j[1], box)
    z = _wrap(z + j[2], box)
    rho_t = 1.0 + 0.1 * np.sin(2.0 * np.pi * x / box)
    m = rho_t * d ** 3
    v = rng.normal(0.0, sigma_v, size=(3, x.size))
    u = 1.0 / ((gamma - 1.0) * rho_t)
    return Workload(name=name, x=x, y=y, z=z, m=m, vx=v[0].copy(), vy=v[1].copy(),
                    vz=v[2].copy(), u=u, gamma=gamma, box=(box, box, box),
                    extra={"spacing": d, "jitter": jitter})


def adjoint_box(n_side: int = 64, seed: int = SEED_BASE + 4, steps: int = 10,
                dt: float = 1.0e-3) -> Workload:
    """The ``jittered_sine`` recipe at ``n_side``^3, run for ``steps`` fixed steps."""
    w = jittered_sine(n_side=n_side, seed=seed, name="adjoint_box")
    w.steps = steps
    w.dt = dt
    return w


def shock_tube(n_yz: int = 32, l_yz: float = 0.125, seed: int = SEED_BASE + 1,
               gamma: float = 5.0 / 3.0, steps: int = 50, cfl: float = 0.25,
               jitter: float = 0.2) -> Workload:
    """Planar shock tube in [0,2] x [0,l_yz]^2, periodic on every axis.

    Left half (x < 1): lattice spacing dL = l_yz / n_yz, rho = 1, P = 1.
    Right half: spacing 2 dL, rho = 1/8, P = 0.1.  All particles have mass dL^3,
    so the density ratio comes from the spacing ratio alone.  Each site moves
    by U(-jitter, jitter) of its own block's spacing per axis (no site crosses
    x = 1 for jitter < 1/2); the state follows the block.  v = 0.  With
    jitter = 0 the two lattices are perfect: their planar contact layer is then
    a symmetric state that any asymmetric rounding perturbs, and that
    perturbation grows by about 3x per step in the layer.  The x axis is
    periodic too, so a mirrored interface sits at x = 0 == 2; the profile is
    compared on 0.5 <= x <= 1.5 only."""
    rng = _rng(seed)
    dl = l_yz / n_yz
    nxl = int(round(1.0 / dl))
    xl, yl, zl = lattice_sites(nxl, n_yz, n_yz, dl)
    dr = 2.0 * dl
    nxr = nxl // 2
    xr, yr, zr = lattice_sites(nxr, n_yz // 2, n_yz // 2, dr, origin=(1.0, 0.0, 0.0))
    x = np.concatenate([xl, xr])
    y = np.concatenate([yl, yr])
    z = np.concatenate([zl, zr])
    left = np.arange(x.size) < xl.size
    if jitter > 0.0:
        sp = np.where(left, dl, dr)
        j = rng.uniform(-jitter, jitter, size=(3, x.size)) * sp
        x = _wrap(x + j[0], 2.0)
        y = _wrap(y + j[1], l_yz)
        z = _wrap(z + j[2], l_yz)
    m = np.full(x.size, dl ** 3)
    rho = np.where(left, 1.0, 0.125)
    P = np.where(left, 1.0, 0.1)
    u = P / ((gamma - 1.0) * rho)
    zero = np.zeros(x.size)
    # shuffle the storage order so that neighbour building starts from an unsorted set
    perm = rng.permutation(x.size)
    return Workload(name="shock_tube", x=x[perm], y=y[perm], z=z[perm], m=m[perm],
                    vx=zero.copy(), vy=zero.copy(), vz=zero.copy(), u=u[perm],
                    gamma=gamma, box=(2.0, l_yz, l_yz), cfl=cfl, steps=steps,
                    extra={"spacing_left": dl, "spacing_right": dr, "jitter": jitter,
                           "left": (1.0, 0.0, 1.0), "right": (0.125, 0.0, 0.1)})


def gaussian_field(n: int, power, rng: np.random.Generator, kmin: float, kmax: float) -> np.ndarray:
    """Real Gaussian random field on an n^3 periodic grid whose Fourier amplitudes are
    filtered by sqrt(power(|k|)) for kmin <= |k| <= kmax (|k| in units of the
    fundamental), zero elsewhere.  White noise in real space, filtered in k space."""
    white = rng.standard_normal((n, n, n))
    wk = np.fft.rfftn(white)
    k1 = np.fft.fftfreq(n, d=1.0 / n)
    k3 = np.fft.rfftfreq(n, d=1.0 / n)
    kk = np.sqrt(k1[:, None, None] ** 2 + k1[None, :, None] ** 2 + k3[None, None, :] ** 2)
    filt = np.zeros_like(kk)
    band = (kk >= kmin) & (kk <= kmax)
    filt[band] = np.sqrt(power(kk[band]))
    f = np.fft.irfftn(wk * filt, s=(n, n, n), axes=(0, 1, 2))
    return f


def turbulence(n_side: int = 128, seed: int = SEED_BASE + 2, jitter: float = 0.2,
               gamma: float = 1.001, mach: float = 2.0) -> Workload:
    """Jittered lattice in the unit box, rho = 1 (m = spacing^3), P = 1/gamma so the
    sound speed is 1.  Each velocity component is an independent Gaussian field on
    the n_side^3 grid with |v(k)|^2 ~ k^-4 for 1 <= |k| <= 8, scaled so that the
    rms speed is ``mach``, and sampled at each particle's unjittered lattice node."""
    rng = _rng(seed)
    d = 1.0 / n_side
    x, y, z = lattice_sites(n_side, n_side, n_side, d)
    j = rng.uniform(-jitter, jitter, size=(3, x.size)) * d
    x = _wrap(x + j[0], 1.0)
    y = _wrap(y + j[1], 1.0)
    z = _wrap(z + j[2], 1.0)
    comps = [gaussian_field(n_side, lambda k: k ** -4.0, rng, 1.0, 8.0).ravel() for _ in range(3)]
    rms = np.sqrt(np.mean(comps[0] ** 2 + comps[1] ** 2 + comps[2] ** 2))
    vx, vy, vz = (c * (mach / rms) for c in comps)
    m = np.full(x.size, d ** 3)
    P = 1.0 / gamma
    u = np.full(x.size, P / (gamma - 1.0))
    return Workload(name="turbulence", x=x, y=y, z=z, m=m, vx=vx, vy=vy, vz=vz, u=u,
                    gamma=gamma, box=(1.0, 1.0, 1.0), extra={"spacing": d, "mach": mach})


def clustered(n_side: int = 256, seed: int = SEED_BASE + 3, sigma: float = 2.0,
              gamma: float = 5.0 / 3.0, sigma_v: float = 0.3, grid: int | None = None) -> Workload:
    """n_side^3 particles in the unit box drawn from a log-normal density.

    A Gaussian field delta with P(k) ~ k^-3 on 1 <= |k| <= grid/2 lives on a
    ``grid``^3 mesh (default n_side) and is scaled to standard deviation
    ``sigma``; rho_cell ~ exp(delta), normalised to mean 1.  Exactly N particles
    are spread over the cells by a multinomial draw with weights rho_cell (Poisson
    sampling conditioned on the total), uniformly within each cell.  m = 1/N,
    P = rho_cell^(5/3) through u = rho_cell^(2/3)/(gamma-1), v ~ N(0, sigma_v^2)."""
    rng = _rng(seed)
    g = n_side if grid is None else grid
    n = n_side ** 3
    delta = gaussian_field(g, lambda k: k ** -3.0, rng, 1.0, g / 2.0)
    delta *= sigma / delta.std()
    rho = np.exp(delta)
    rho /= rho.mean()
    p = (rho / rho.sum()).ravel()
    counts = rng.multinomial(n, p)
    cell = np.repeat(np.arange(g ** 3, dtype=np.int64), counts)
    del counts, p
    ci = cell // (g * g)
    cj = (cell // g) % g
    ck = cell % g
    h = 1.0 / g
    off = rng.uniform(0.0, 1.0, size=(3, n))
    x = _wrap((ci + off[0]) * h, 1.0)
    y = _wrap((cj + off[1]) * h, 1.0)
    z = _wrap((ck + off[2]) * h, 1.0)
    del off
    rho_p = rho.ravel()[cell]
    del cell, ci, cj, ck
    u = rho_p ** (2.0 / 3.0) / (gamma - 1.0)
    v = rng.normal(0.0, sigma_v, size=(3, n))
    m = np.full(n, 1.0 / n)
    perm = rng.permutation(n)
    return Workload(name="clustered", x=x[perm], y=y[perm], z=z[perm], m=m,
                    vx=v[0][perm], vy=v[1][perm], vz=v[2][perm], u=u[perm], gamma=gamma,
                    box=(1.0, 1.0, 1.0), extra={"sigma_lnrho": sigma, "grid": g})


def by_name(name: str, **kw) -> Workload:
    table = {
        "jittered_sine": jittered_sine,
        "shock_tube": shock_tube,
        "turbulence": turbulence,
        "clustered": clustered,
        "adjoint_box": adjoint_box,
    }
    return table[name](**kw)
