"""The no-allocation whole pass (mfm_hydro_pass_noalloc, through the C ABI)
against the context path it replaces (mfm_build_neighbours + mfm_hydro_pass):
two calls in a row on one GPU, the second with a smaller set, each held to the
FP64 bar (1e-12 normwise per field; H, n, V element by element)."""
import numpy as np
import pytest

from paper_1712_01294_amd import workloads as W

from .gpu_util import elem_rel, in_input_order, nerr

pytestmark = pytest.mark.gpu

FIELDS = ("H", "nk", "V", "B", "rho", "P", "grad", "dp", "dE", "vsig")


def _context_pass(w, scheme):
    from paper_1712_01294_amd import mfm
    ctx = mfm.Context(mfm.config_of(w, scheme=scheme), w.n)
    st = mfm.State.from_arrays(w.arrays(), dm=scheme == mfm.SCHEME_MFV)
    ctx.build_neighbours(st)
    ctx.hydro_pass(st)
    ctx.check()
    return st, ctx.counters()


@pytest.mark.parametrize("scheme", [0, 1], ids=["mfm", "mfv"])
def test_noalloc_pass_matches_the_context_pass_twice_in_a_row(scheme):
    import torch

    from paper_1712_01294_amd import mfm
    fields = FIELDS + (("dm",) if scheme == mfm.SCHEME_MFV else ())
    for n_side, seed in ((16, W.SEED_BASE + 130), (12, W.SEED_BASE + 131)):
        w = W.jittered_sine(n_side=n_side, seed=seed)
        ref, rc = _context_pass(w, scheme)
        st = mfm.State.from_arrays(w.arrays(), dm=scheme == mfm.SCHEME_MFV)
        c = mfm.hydro_pass_noalloc(mfm.config_of(w, scheme=scheme), st)
        torch.cuda.synchronize()
        print(f"n={w.n} pairs noalloc={c['pairs']} context={rc['pairs']}", flush=True)
        assert c["pairs"] == rc["pairs"]
        assert c["gather_entries"] == rc["gather_entries"]
        for k in fields:
            a, b = in_input_order(st, k), in_input_order(ref, k)
            assert nerr(a, b) <= 1e-12, (n_side, k)
        for k in ("H", "nk", "V"):
            assert elem_rel(in_input_order(st, k), in_input_order(ref, k)) <= 1e-12


def test_noalloc_pass_without_counters_queues_only_and_rejects_large_sets():
    import torch

    from paper_1712_01294_amd import mfm
    w = W.jittered_sine(n_side=10, seed=W.SEED_BASE + 132)
    ref, _ = _context_pass(w, 0)
    st = mfm.State.from_arrays(w.arrays())
    assert mfm.hydro_pass_noalloc(mfm.config_of(w), st, counters=False) is None
    torch.cuda.synchronize()
    for k in ("H", "dp", "dE"):
        assert nerr(in_input_order(st, k), in_input_order(ref, k)) <= 1e-12, k
    big = W.jittered_sine(n_side=21, seed=W.SEED_BASE + 133)   # 9261 > 8192 particles
    assert big.n > mfm.NOALLOC_MAX_N
    sb = mfm.State.from_arrays(big.arrays())
    with pytest.raises(mfm.MFMError) as e:
        mfm.hydro_pass_noalloc(mfm.config_of(big), sb)
    assert e.value.status == -6
    with pytest.raises(mfm.MFMError) as e:
        mfm.hydro_pass_noalloc(mfm.config_of(w, max_ngb=512), st)
    assert e.value.status == -1
