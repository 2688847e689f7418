"""mfm_unpermute (through the C ABI): the particles back in the order they were
given in, every array moved bit for bit, ids checked on the device."""
import numpy as np
import pytest

from paper_1712_01294_amd import workloads as W

from .gpu_util import in_input_order, nerr, run_pass

pytestmark = pytest.mark.gpu

FIELDS_IN = ("x", "y", "z", "m", "vx", "vy", "vz", "u")
FIELDS_OUT = ("H", "nk", "V", "B", "rho", "P", "grad", "alpha", "dp", "dE", "vsig")


@pytest.fixture(scope="module")
def sine16():
    return W.jittered_sine(n_side=16, seed=W.SEED_BASE + 180)


@pytest.mark.parametrize("scheme", [0, 1])
def test_unpermute_restores_the_input_order_bitwise(sine16, scheme):
    """After a pass (MFM, and MFV with its mass rates) every array, all rows of
    B, grad, alpha and dp included, equals the Morton-ordered result scattered
    back by the carried ids on the host, bit for bit; the inputs equal the
    caller's arrays and id is 0 .. n-1."""
    w = sine16
    ctx, st = run_pass(w, scheme=scheme)
    fields = FIELDS_OUT + (("dm",) if scheme == 1 else ())
    want = {k: in_input_order(st, k) for k in fields}
    ctx.unpermute(st)
    assert np.array_equal(st.id.cpu().numpy(), np.arange(w.n))
    arrays = w.arrays()
    for k in FIELDS_IN:
        assert np.array_equal(getattr(st, k).cpu().numpy(), arrays[k]), k
    for k in fields:
        assert np.array_equal(getattr(st, k).cpu().numpy(), want[k]), k


def test_pass_after_unpermute_needs_a_build_and_repeats_the_first(sine16):
    """The context's lists belong to the old order: a pass returns MFM_E_STATE
    until the neighbours are rebuilt.  Rebuilt from a cold start, the pass
    repeats the first one bit for bit (the stable key sort from the caller's
    order again)."""
    import torch

    from paper_1712_01294_amd import mfm
    w = sine16
    ctx, st = run_pass(w)
    first = {k: in_input_order(st, k) for k in FIELDS_OUT}
    ctx.unpermute(st)
    with pytest.raises(mfm.MFMError) as e:
        ctx.hydro_pass(st)
    assert e.value.status == -8
    st.H.zero_()
    ctx.build_neighbours(st)
    ctx.hydro_pass(st)
    torch.cuda.synchronize()
    ctx.check()
    for k in FIELDS_OUT:
        assert np.array_equal(in_input_order(st, k), first[k]), k


def test_unpermute_rejects_ids_that_are_not_a_permutation(sine16):
    """A repeated id, an id out of range and a missing id array each return
    MFM_E_INVALID with nothing moved."""
    import torch

    from paper_1712_01294_amd import mfm
    w = sine16
    ctx, st = run_pass(w)
    before = {k: getattr(st, k).clone() for k in FIELDS_IN + ("H", "dp")}
    ids = st.id.clone()
    for bad in ("repeat", "range"):
        st.id.copy_(ids)
        if bad == "repeat":
            st.id[5] = st.id[7]
        else:
            st.id[3] = w.n
        with pytest.raises(mfm.MFMError) as e:
            ctx.unpermute(st)
        assert e.value.status == -1, bad
        for k, v in before.items():
            assert torch.equal(getattr(st, k), v), (bad, k)
    st.id.copy_(ids)
    keep = st.id
    st.id = None
    with pytest.raises(mfm.MFMError) as e:
        ctx.unpermute(st)
    assert e.value.status == -1
    st.id = keep
    ctx.unpermute(st)
    assert np.array_equal(st.id.cpu().numpy(), np.arange(w.n))


def test_hierarchical_step_after_unpermute():
    """A hierarchical system step, the particles (and, by the caller, their bins)
    put back in the input order, then a second system step with a rebin: the
    same state as two steps without the unpermute, to rounding (the second
    step re-solves the kernel lengths from the kept ones, where the other
    reuses them)."""
    import dataclasses

    import torch

    from paper_1712_01294_amd import mfm
    w0 = W.jittered_sine(n_side=16, seed=W.SEED_BASE + 181)
    tp = 2.0 * np.pi
    w = dataclasses.replace(w0, vx=0.5 * np.sin(tp * w0.y), vy=0.5 * np.sin(tp * w0.z),
                            vz=0.5 * np.sin(tp * w0.x))
    bins = np.minimum((w.x * 3).astype(np.int64), 2)
    T = 0.004
    out = []
    for undo in (False, True):
        ctx = mfm.Context(mfm.config_of(w, u_floor=0.0), w.n)
        st = mfm.State.from_arrays(w.arrays())
        ctx.build_neighbours(st)
        ctx.hydro_pass(st)
        b = torch.as_tensor(bins[st.id.cpu().numpy()], device="cuda")
        ctx.step_hier(st, b, 2, T, rebin=True, active=True)
        if undo:
            ids = st.id.clone()
            ctx.unpermute(st)
            nb = torch.empty_like(b)
            nb[ids] = b
            b = nb
            assert np.array_equal(b.cpu().numpy(), bins)
        ctx.step_hier(st, b, 2, T, rebin=True, active=True)
        ctx.check()
        out.append({k: in_input_order(st, k) for k in FIELDS_IN + ("dp", "dE", "vsig")})
    L = np.array(w.box)
    for c, k in enumerate(("x", "y", "z")):
        d = out[1][k] - out[0][k]
        d -= L[c] * np.round(d / L[c])
        assert np.abs(d).max() <= 1e-12 * L[c], k
    for k in ("vx", "vy", "vz", "u", "dp", "dE", "vsig"):
        assert nerr(out[1][k], out[0][k]) <= 1e-12, k
