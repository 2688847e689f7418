"""Slow, differentiable PyTorch FP64 reference of the MFM pass and step.

TEST INFRASTRUCTURE ONLY.  Written independently of the C oracle, as dense
N x N tensor expressions for tiny particle sets, so that torch.autograd can
differentiate the whole multi-step update.  It follows the same readings
R1-R18 (meshless finite-mass pass of the Godunov method the release paper
names in its abstract and "Arbitrary (Moving) Meshes" section):

* neighbour sets are fixed at the detached values (the kernel is C^2 at its
  support edge, so set changes are smooth);
* the kernel length is the detached root of the neighbour-number equation
  followed by one differentiable Newton step with a detached slope, which is
  exactly the implicit-function-theorem derivative dH = -(df/dtheta)/(df/dH);
* limiter, Davis speeds, the P* clamp and the first-order fallback follow the
  active branch, as autograd does.
"""
from __future__ import annotations

import math

import torch

T = torch.float64


def w_spline(q):
    """Cubic spline w(q) with support 1, zero (and flat) for q >= 1."""
    inner = 1.0 - 6.0 * q * q + 6.0 * q * q * q
    t = torch.clamp(1.0 - q, min=0.0)
    outer = 2.0 * t * t * t
    return torch.where(q <= 0.5, inner, outer)


def kernel_W(r, H):
    return 8.0 / (math.pi * H ** 3) * w_spline(r / H)


def displacements(x, box, periodic):
    """d[i, j] = x_j - x_i with the nearest periodic image; x is (N, 3)."""
    d = x[None, :, :] - x[:, None, :]
    for a in range(3):
        if periodic[a]:
            L = box[a]
            da = d[..., a]
            da = torch.where(da > 0.5 * L, da - L, torch.where(da < -0.5 * L, da + L, da))
            d = torch.cat([d[..., :a], da[..., None], d[..., a + 1:]], dim=-1)
    return d


def _dist(d):
    n = d.shape[0]
    eye = torch.eye(n, dtype=torch.bool)
    r2 = (d * d).sum(-1)
    r = torch.sqrt(torch.where(eye, torch.ones_like(r2), r2))
    return torch.where(eye, torch.zeros_like(r), r), eye


def solve_h(r, n_ngb, H_guess):
    """Differentiable kernel length: detached bisection root + one IFT Newton step."""
    rd = r.detach()

    def resid(H):
        return 4.0 * math.pi / 3.0 * H ** 3 * kernel_W(rd, H[:, None]).sum(1) - n_ngb

    with torch.no_grad():
        hi = H_guess.clone()
        lo = torch.zeros_like(hi)
        for _ in range(200):
            bad = resid(hi) < 0
            if not bool(bad.any()):
                break
            lo = torch.where(bad, hi, lo)
            hi = torch.where(bad, hi * 1.5, hi)
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            neg = resid(mid) < 0
            lo = torch.where(neg, mid, lo)
            hi = torch.where(neg, hi, mid)
        H0 = hi
    H0r = H0.clone().requires_grad_(True)
    f0 = 4.0 * math.pi / 3.0 * H0r ** 3 * kernel_W(rd, H0r[:, None]).sum(1)
    (slope,) = torch.autograd.grad(f0.sum(), H0r)
    f = 4.0 * math.pi / 3.0 * H0 ** 3 * kernel_W(r, H0[:, None]).sum(1) - n_ngb
    return H0 - f / slope.detach()


def hydro_pass(st, gamma, n_ngb, box, periodic, beta=1.0, H_guess=None):
    """Dense FP64 pass.  st: dict of (N,) tensors x, y, z, m, vx, vy, vz, u.
    Returns H, nk, V, B (N,3,3), rho, P, grad (N,5,3), dp (N,3), dE, vsig, pairs."""
    X = torch.stack([st["x"], st["y"], st["z"]], 1)
    vel = torch.stack([st["vx"], st["vy"], st["vz"]], 1)
    n = X.shape[0]
    d = displacements(X, box, periodic)
    r, eye = _dist(d)
    if H_guess is None:
        vol = box[0] * box[1] * box[2]
        H_guess = torch.full((n,), (3 * n_ngb * vol / (4 * math.pi * n)) ** (1 / 3), dtype=T)
    H = solve_h(r, n_ngb, H_guess.detach())
    Wm = kernel_W(r, H[:, None])                     # W(r_ij, H_i)
    gather = (r.detach() < H.detach()[:, None])      # includes self
    Wm = torch.where(gather, Wm, torch.zeros_like(Wm))
    nk = Wm.sum(1)
    V = 1.0 / nk
    rho = st["m"] * nk
    P = (gamma - 1.0) * rho * st["u"]
    phi = torch.stack([rho, vel[:, 0], vel[:, 1], vel[:, 2], P], 1)   # (N,5)
    psi = Wm * V[:, None]
    psi_off = torch.where(eye, torch.zeros_like(psi), psi)
    E = torch.einsum("ij,ija,ijb->iab", psi_off, d, d)
    B = torch.linalg.inv(E)
    dphi = phi[None, :, :] - phi[:, None, :]                            # (i,j,f)
    S = torch.einsum("ij,ijf,ija->ifa", psi_off, dphi, d)
    graw = torch.einsum("iab,ifb->ifa", B, S)
    big = torch.finfo(T).max
    gm = gather[:, :, None]
    pmax = torch.where(gm, phi[None, :, :].expand(n, n, 5), torch.full_like(dphi, -big)).amax(1)
    pmin = torch.where(gm, phi[None, :, :].expand(n, n, 5), torch.full_like(dphi, big)).amin(1)
    rmax = torch.where(gather, r, torch.zeros_like(r)).amax(1)
    gn = torch.sqrt((graw * graw).sum(-1))
    safe = torch.where(gn > 0, gn, torch.ones_like(gn))
    up = (pmax - phi) / (safe * 0.5 * rmax[:, None])
    dn = (phi - pmin) / (safe * 0.5 * rmax[:, None])
    alpha = torch.where(gn > 0, torch.clamp(beta * torch.minimum(up, dn), max=1.0), torch.ones_like(gn))
    grad = alpha[:, :, None] * graw

    # unordered pairs a < b with r < max(H_a, H_b)
    Hd = H.detach()
    reach = (r.detach() < torch.maximum(Hd[:, None], Hd[None, :])) & (~eye)
    ia, ib = torch.nonzero(torch.triu(reach, diagonal=1), as_tuple=True)
    dab = d[ia, ib]                                   # x_b - x_a
    rab = r[ia, ib]
    Wa = torch.where(rab.detach() < Hd[ia], kernel_W(rab, H[ia]), torch.zeros_like(rab))
    Wb = torch.where(rab.detach() < Hd[ib], kernel_W(rab, H[ib]), torch.zeros_like(rab))
    A = ((V[ia] ** 2 * Wa)[:, None] * torch.einsum("pab,pb->pa", B[ia], dab)
         + (V[ib] ** 2 * Wb)[:, None] * torch.einsum("pab,pb->pa", B[ib], dab))
    Amag = torch.sqrt((A * A).sum(1))
    nh = A / Amag[:, None]
    qL = phi[ia] + 0.5 * torch.einsum("pfa,pa->pf", grad[ia], dab)
    qR = phi[ib] - 0.5 * torch.einsum("pfa,pa->pf", grad[ib], dab)
    ok = (qL[:, 0] > 0) & (qL[:, 4] > 0) & (qR[:, 0] > 0) & (qR[:, 4] > 0)
    qL = torch.where(ok[:, None], qL, phi[ia])
    qR = torch.where(ok[:, None], qR, phi[ib])
    w = 0.5 * (vel[ia] + vel[ib])
    uL = ((qL[:, 1:4] - w) * nh).sum(1)
    uR = ((qR[:, 1:4] - w) * nh).sum(1)
    rL, pL, rR, pR = qL[:, 0], qL[:, 4], qR[:, 0], qR[:, 4]
    cL = torch.sqrt(gamma * pL / rL)
    cR = torch.sqrt(gamma * pR / rR)
    SL = torch.minimum(uL - cL, uR - cR)
    SR = torch.maximum(uL + cL, uR + cR)
    mL = rL * (SL - uL)
    mR = rR * (SR - uR)
    Ss = (pR - pL + mL * uL - mR * uR) / (mL - mR)
    Ps = 0.5 * (pL + pR + mL * (Ss - uL) + mR * (Ss - uR))
    Ps = torch.clamp(Ps, min=0.0)
    Fp = Ps[:, None] * A
    FE = Ps * (Ss + (w * nh).sum(1)) * Amag
    dp = torch.zeros(n, 3, dtype=T).index_add(0, ia, -Fp).index_add(0, ib, Fp)
    dE = torch.zeros(n, dtype=T).index_add(0, ia, -FE).index_add(0, ib, FE)
    c = torch.sqrt(gamma * P / rho)
    proj = ((vel[:, None, :] - vel[None, :, :]) * (-d)).sum(-1) / torch.where(eye, torch.ones_like(r), r)
    sig = c[:, None] + c[None, :] - torch.clamp(proj, max=0.0)
    vsig = torch.where(reach, sig, torch.zeros_like(sig)).amax(1)
    return dict(H=H, nk=nk, V=V, B=B, rho=rho, P=P, grad=grad, grad_raw=graw, alpha=alpha,
                dp=dp, dE=dE, vsig=vsig, pairs=int(ia.numel()))


def run_steps(st0, gamma, n_ngb, box, periodic, dt, steps, u_floor, beta=1.0):
    """Kick-drift-kick with a predicted state, fixed dt, differentiable.
    st0: dict of (N,) tensors; returns the final state dict."""
    st = dict(st0)
    m = st["m"]
    out = hydro_pass(st, gamma, n_ngb, box, periodic, beta)
    H = out["H"].detach()
    for _ in range(steps):
        v = torch.stack([st["vx"], st["vy"], st["vz"]], 1)
        E = m * (st["u"] + 0.5 * (v * v).sum(1))
        v = v + 0.5 * dt * out["dp"] / m[:, None]
        E = E + 0.5 * dt * out["dE"]
        X = torch.stack([st["x"], st["y"], st["z"]], 1) + dt * v
        cols = []
        for a in range(3):
            xa = X[:, a]
            if periodic[a]:
                L = box[a]
                xa = xa - L * torch.floor(xa.detach() / L)
            cols.append(xa)
        vp = v + 0.5 * dt * out["dp"] / m[:, None]
        Ep = E + 0.5 * dt * out["dE"]
        up = torch.clamp(Ep / m - 0.5 * (vp * vp).sum(1), min=u_floor)
        pst = dict(x=cols[0], y=cols[1], z=cols[2], m=m, vx=vp[:, 0], vy=vp[:, 1], vz=vp[:, 2], u=up)
        out = hydro_pass(pst, gamma, n_ngb, box, periodic, beta, H_guess=H)
        H = out["H"].detach()
        v = v + 0.5 * dt * out["dp"] / m[:, None]
        E = E + 0.5 * dt * out["dE"]
        u = torch.clamp(E / m - 0.5 * (v * v).sum(1), min=u_floor)
        st = dict(x=cols[0], y=cols[1], z=cols[2], m=m, vx=v[:, 0], vy=v[:, 1], vz=v[:, 2], u=u)
    return st
