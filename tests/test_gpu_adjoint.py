"""Hand-written adjoint of the pass and of the multi-step update (HIP, through
the C ABI) against autodiff through the dense PyTorch FP64 reference, and
against central finite differences at full size."""
import numpy as np
import pytest

from paper_1712_01294_amd import workloads as W

from .gpu_util import nerr

pytestmark = pytest.mark.gpu

TOL_AD = 1e-10        # adjoint vs autodiff of the FP64 reference, normwise per field


def _torch_state(w, requires=()):
    import torch
    st = {k: torch.tensor(v, dtype=torch.float64) for k, v in w.arrays().items()}
    for k in requires:
        st[k].requires_grad_(True)
    return st


def test_pass_adjoint_matches_torch_autograd():
    import torch

    from oracle import torch_ref as TR
    from paper_1712_01294_amd import mfm
    w = W.jittered_sine(n_side=8, seed=W.SEED_BASE + 140)
    rng = np.random.default_rng(3)
    lp = rng.normal(size=(3, w.n))
    le = rng.normal(size=w.n)
    # reference: gradient of <lp, dp> + <le, dE> through the dense pass
    st = _torch_state(w, requires=("x", "y", "z", "vx", "vy", "vz", "u"))
    out = TR.hydro_pass(st, w.gamma, w.n_ngb, w.box, w.periodic)
    L = (out["dp"] * torch.tensor(lp.T)).sum() + (out["dE"] * torch.tensor(le)).sum()
    L.backward()
    gx = np.stack([st[k].grad.numpy() for k in ("x", "y", "z")])
    gv = np.stack([st[k].grad.numpy() for k in ("vx", "vy", "vz")])
    gu = st["u"].grad.numpy()
    # HIP adjoint, adjoint inputs permuted into the library order
    ctx = mfm.Context(mfm.config_of(w), w.n)
    s = mfm.State.from_arrays(w.arrays())
    ctx.build_neighbours(s)
    ctx.hydro_pass(s)
    ctx.check()
    ids = s.id.cpu().numpy()
    ax, av, au = ctx.pass_adjoint(s, torch.tensor(lp[:, ids], device="cuda"),
                                  torch.tensor(le[ids], device="cuda"))
    hx = np.empty((3, w.n))
    hv = np.empty((3, w.n))
    hu = np.empty(w.n)
    hx[:, ids] = ax.cpu().numpy()
    hv[:, ids] = av.cpu().numpy()
    hu[ids] = au.cpu().numpy()
    errs = {"x": nerr(hx, gx), "v": nerr(hv, gv), "u": nerr(hu, gu)}
    print("pass adjoint vs autograd", errs, flush=True)
    for k, e in errs.items():
        assert e <= TOL_AD, (k, e)


def _loss_grads_torch(w, steps, dt, u_floor):
    import torch

    from oracle import torch_ref as TR
    st = _torch_state(w, requires=("vx", "vy", "vz", "u"))
    out = TR.run_steps(st, w.gamma, w.n_ngb, w.box, w.periodic, dt, steps, u_floor)
    L = (st["m"] * (out["vx"] ** 2 + out["vy"] ** 2 + out["vz"] ** 2)).sum()
    L.backward()
    gv = np.stack([st[k].grad.numpy() for k in ("vx", "vy", "vz")])
    return float(L.detach()), gv, st["u"].grad.numpy()


def _loss_grads_gpu(w, steps, dt, u_floor):
    import torch

    from paper_1712_01294_amd import autodiff, mfm
    evo = autodiff.Evolution(w, steps, dt, mfm.config_of(w, u_floor=u_floor))
    v0 = torch.tensor(np.stack([w.vx, w.vy, w.vz]), device="cuda", requires_grad=True)
    u0 = torch.tensor(w.u, device="cuda", requires_grad=True)
    vk, uk = autodiff.MFMSteps.apply(v0, u0, evo)
    m = torch.tensor(w.m, device="cuda")
    L = (m * (vk * vk).sum(0)).sum()
    L.backward()
    return float(L.detach()), v0.grad.cpu().numpy(), u0.grad.cpu().numpy()


def test_two_step_adjoint_matches_torch_autograd():
    """8^3 jittered box, two fixed-dt steps, L = sum m |v|^2 at the end:
    gradients w.r.t. the initial v and u against autodiff of the reference."""
    w = W.jittered_sine(n_side=8, seed=W.SEED_BASE + 141)
    u_floor = 1e-10 * float(np.mean(w.u))
    Lt, gvt, gut = _loss_grads_torch(w, 2, 1e-3, u_floor)
    Lg, gvg, gug = _loss_grads_gpu(w, 2, 1e-3, u_floor)
    print("L", Lg, Lt, "errs v", nerr(gvg, gvt), "u", nerr(gug, gut), flush=True)
    assert abs(Lg - Lt) <= 1e-13 * abs(Lt)
    assert nerr(gvg, gvt) <= TOL_AD
    assert nerr(gug, gut) <= TOL_AD


@pytest.fixture(scope="module")
def adjoint_box_grad():
    """64^3 jittered box, 10 fixed steps of dt = 1e-3, L = sum m |v|^2: the adjoint
    gradient w.r.t. (v0, u0), and a function giving L(+) - L(-) for a direction."""
    import torch

    from paper_1712_01294_amd import autodiff
    w = W.adjoint_box()
    evo = autodiff.Evolution(w, w.steps, w.dt)
    m = torch.tensor(w.m, device="cuda")
    v0 = torch.tensor(np.stack([w.vx, w.vy, w.vz]), device="cuda")
    u0 = torch.tensor(w.u, device="cuda")

    def final_v(v, u):
        st, _ = evo.run(v, u, keep=False)
        out = torch.empty(3, w.n, dtype=torch.float64, device="cuda")
        out[:, st.id] = torch.stack([st.vx, st.vy, st.vz])
        return out

    def central(d, eps):
        # L(+) - L(-) accumulated particle by particle: the difference of the two
        # sums would be quantised at the FP64 resolution of L itself
        dv = torch.tensor(d[: 3 * w.n].reshape(3, w.n), device="cuda")
        du = torch.tensor(d[3 * w.n:], device="cuda")
        vp = final_v(v0 + eps * dv, u0 + eps * du)
        vm = final_v(v0 - eps * dv, u0 - eps * du)
        return float((m * ((vp - vm) * (vp + vm)).sum(0)).sum()) / (2 * eps)

    vr = v0.clone().requires_grad_(True)
    ur = u0.clone().requires_grad_(True)
    vk, uk = autodiff.MFMSteps.apply(vr, ur, evo)
    L = (m * (vk * vk).sum(0)).sum()
    L.backward()
    g = np.concatenate([vr.grad.cpu().numpy().ravel(), ur.grad.cpu().numpy()])
    return w, g, central


def test_adjoint_box_finite_differences_unit_directions(adjoint_box_grad):
    """16 seeded random unit directions in (v0, u0) (4N = 1,048,576 components),
    central differences at eps = 1e-6, retried at 1e-7 when they miss (a neighbour
    crossing the support edge moves the limiter's extrema: a jump, not an adjoint
    error).  With unit directions the difference L(+) - L(-) is ~1e-13 of L and the
    rounding of the forward pass bounds the agreement at about 1e-5 (the error
    scales as 1/eps below eps = 1e-5); asserted at 2e-4, the values are reported."""
    w, g, central = adjoint_box_grad
    rng = np.random.default_rng(W.SEED_BASE + 4)
    rels = []
    for k in range(16):
        d = rng.normal(size=4 * w.n)
        d /= np.linalg.norm(d)
        ad = float(g @ d)
        best = None
        for eps in (1e-6, 1e-7):
            fd = central(d, eps)
            rel = abs(fd - ad) / abs(ad)
            best = rel if best is None else min(best, rel)
            if rel <= 1e-6:
                break
        print(f"unit direction {k}: adjoint {ad:.12e} fd {fd:.12e} rel {best:.2e}", flush=True)
        rels.append(best)
    print("median", float(np.median(rels)), "max", max(rels), flush=True)
    assert max(rels) <= 2e-4


def test_adjoint_box_finite_differences_local_directions(adjoint_box_grad):
    """16 random unit directions supported on the (v, u) of 64 random particles,
    eps = 1e-5 (retried at 2e-6): the larger per-particle signal takes most
    directions to <= 1e-6 (9 of 16 when measured); the rest sit at the same
    FP64 evaluation floor as the unit directions.  Median <= 1e-5, max <= 2e-4."""
    w, g, central = adjoint_box_grad
    rng = np.random.default_rng(W.SEED_BASE + 44)
    rels = []
    for k in range(16):
        d = np.zeros(4 * w.n)
        sel = rng.choice(w.n, 64, replace=False)
        for c in range(4):
            d[c * w.n + sel] = rng.normal(size=64)
        d /= np.linalg.norm(d)
        ad = float(g @ d)
        best = None
        for eps in (1e-5, 2e-6):
            fd = central(d, eps)
            rel = abs(fd - ad) / abs(ad)
            best = rel if best is None else min(best, rel)
            if rel <= 1e-6:
                break
        print(f"local direction {k}: adjoint {ad:.12e} fd {fd:.12e} rel {best:.2e}", flush=True)
        rels.append(best)
    print("median", float(np.median(rels)), "max", max(rels), flush=True)
    assert float(np.median(rels)) <= 1e-5
    assert max(rels) <= 2e-4
