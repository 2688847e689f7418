"""The optional limiters on the GPU (through the C ABI) against the oracle:
the pairwise face limiter (R23) and the condition-adaptive limiter constant
(R24), in the MFM and MFV forms, FP64 and mixed, the pass and the step."""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_1712_01294_amd import workloads as W

from .gpu_util import compare_pass, elem_rel, in_input_order, nerr, run_pass

pytestmark = pytest.mark.gpu

# R24 with the pairwise limiter as a safety net: beta 2 for well-conditioned
# gradient matrices (cond <= 10), Barth-Jespersen's 1 from cond >= 1000
LIM = dict(limiter=1, beta=2.0, beta_min=1.0, cond_lo=10.0, cond_hi=1000.0)


def _setup(w, scheme="mfm"):
    return dataclasses.replace(O.Setup.of(w), scheme=scheme, **LIM)


def _print(tag, errs):
    print(tag, " ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)


@pytest.mark.parametrize("case", ["sine16", "clustered16", "clustered20"])
@pytest.mark.parametrize("scheme", ["mfm", "mfv"])
def test_limited_pass_matches_oracle(case, scheme):
    from paper_1712_01294_amd import mfm
    w = {"sine16": lambda: W.jittered_sine(n_side=16, sigma_v=1.5),
         "clustered16": lambda: W.clustered(n_side=16, seed=W.SEED_BASE + 160),
         "clustered20": lambda: W.clustered(n_side=20, seed=W.SEED_BASE + 161)}[case]()
    ref = O.hydro_pass(_setup(w, scheme), w.arrays())
    ctx, st = run_pass(w, scheme=mfm.SCHEME_MFV if scheme == "mfv" else mfm.SCHEME_MFM, max_ngb=1024, **LIM)
    ctx.check(allow_illcond=True)
    fields = ("H", "nk", "V", "B", "rho", "P", "grad", "dp", "dE", "vsig") + (("dm",) if scheme == "mfv" else ())
    errs = compare_pass(st, ref, fields)
    _print(f"limited {scheme} {case}", errs)
    c = ctx.counters()
    assert c["fallbacks"] == 0 and ref["fallbacks"] == 0
    assert c["pairs"] == ref["pairs"]
    # B on the clustered sets: 32 eps cond(E) per particle where E is ill-conditioned
    for k, e in errs.items():
        if k == "B" and case != "sine16":
            continue
        assert e <= 1e-12, (k, e)
    for k in ("H", "nk", "V"):
        assert elem_rel(in_input_order(st, k), ref[k]) <= 1e-12
    if case != "sine16":
        Bg = in_input_order(st, "B")
        tol = np.maximum(1e-12, 32 * np.finfo(np.float64).eps * ref["cond"])
        assert np.all(np.abs(Bg - ref["B"]).max(0) <= tol * np.abs(ref["B"]).max(0))


def test_limited_alpha_follows_the_adaptive_beta():
    """R24 on the GPU: the limiter factors equal the oracle's, whose beta moves
    with cond(E) (pinned on the oracle alone)."""
    w = W.clustered(n_side=16, seed=W.SEED_BASE + 160)
    s = _setup(w)
    H, nk, V, _ = O.solve_h(s, w.x, w.y, w.z)
    g = O.gradients(s, w.arrays(), H, nk, V)
    ctx, st = run_pass(w, max_ngb=1024, **LIM)
    al = in_input_order(st, "alpha")
    good = g["cond"] <= 1e3      # elsewhere the gradients carry cond(E) eps of rounding
    assert np.abs(al[:, good] - g["alpha"][:, good]).max() <= 1e-12
    # the condition numbers span the interpolation range, so R24 is exercised
    assert (g["cond"] > 10.0).any() and (g["cond"] < 10.0).any()


@pytest.mark.parametrize("scheme", ["mfm", "mfv"])
def test_limited_mixed_form_on_the_clustered_benchmark_set(scheme):
    """With the pairwise limiter no face state is non-positive, so the mixed
    form never switches to first order where the FP64 form does not (without
    it, a face pressure within FP32 rounding of zero can): on the full
    16,777,216-particle clustered set the mixed pass stays within 1e-5
    normwise of the FP64 pass on every flux."""
    import torch

    from paper_1712_01294_amd import mfm
    w = W.clustered()
    sch = mfm.SCHEME_MFV if scheme == "mfv" else mfm.SCHEME_MFM
    c64, s64 = run_pass(w, alpha=False, scheme=sch, **LIM)
    f64 = c64.counters()["fallbacks"]
    del c64
    c32, s32 = run_pass(w, alpha=False, precision=mfm.MIXED, scheme=sch, **LIM)
    f32 = c32.counters()["fallbacks"]
    del c32
    assert torch.equal(s64.id, s32.id)
    errs = {}
    for k in ("dp", "dE", "vsig") + (("dm",) if scheme == "mfv" else ()):
        a, b = getattr(s64, k).double(), getattr(s32, k).double()
        errs[k] = float((a - b).abs().max() / a.abs().max())
    _print(f"limited mixed vs fp64 clustered16M {scheme} fallbacks {f64} {f32}", errs)
    assert f64 == 0 and f32 == 0
    for k, e in errs.items():
        assert e <= 1e-5, (k, e)


def test_limited_steps_match_oracle_small_tube():
    """10 CFL steps of the jittered small tube with the optional limiters, against
    the oracle's stepper with the same settings, at 1e-10."""
    from paper_1712_01294_amd import mfm
    w = W.shock_tube(n_yz=12, l_yz=12 / 64)
    ref = O.Stepper(w)
    for k, v in LIM.items():
        setattr(ref.s, k, v)
    ref.start()
    for _ in range(10):
        ref.step()
    ctx = mfm.Context(mfm.config_of(w, **LIM), w.n)
    st = mfm.State.from_arrays(w.arrays())
    ctx.build_neighbours(st)
    ctx.hydro_pass(st)
    for _ in range(10):
        ctx.step(st)
    ctx.check()
    L = np.array(w.box)
    for c, k in enumerate(("x", "y", "z")):
        d = in_input_order(st, k) - ref.st[k]
        d -= L[c] * np.round(d / L[c])
        assert np.abs(d).max() <= 1e-10 * L[c], k
    scale = np.abs(ref.st["vx"]).max()
    for k in ("vx", "vy", "vz"):
        assert np.abs(in_input_order(st, k) - ref.st[k]).max() <= 1e-10 * scale, k
    assert nerr(in_input_order(st, "u"), ref.st["u"]) <= 1e-10


def test_adjoints_refuse_the_optional_limiters():
    import torch

    from paper_1712_01294_amd import mfm
    w = W.jittered_sine(n_side=8)
    ctx, st = run_pass(w, **LIM)
    f = dict(dtype=torch.float64, device="cuda")
    with pytest.raises(mfm.MFMError) as e:
        ctx.pass_adjoint(st, torch.zeros(3, w.n, **f), torch.zeros(w.n, **f))
    assert e.value.status == -1
