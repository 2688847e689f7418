"""Helpers shared by the GPU tests: run the HIP path, map its reordered outputs
back to the input order, and compare with the oracle."""
import numpy as np


def run_pass(w, precision=0, alpha=True, **cfg_kw):
    import torch

    from paper_1712_01294_amd import mfm
    cfg = mfm.config_of(w, precision=precision, **cfg_kw)
    ctx = mfm.Context(cfg, w.n)
    st = mfm.State.from_arrays(w.arrays(), alpha=alpha, dm=cfg.scheme == mfm.SCHEME_MFV)
    ctx.build_neighbours(st)
    ctx.hydro_pass(st)
    torch.cuda.synchronize()
    return ctx, st


def in_input_order(st, name):
    """Array `name` of a GPU state, permuted back to the input order via the carried ids."""
    arr = getattr(st, name).detach().cpu().numpy()
    ids = st.id.cpu().numpy()
    out = np.empty_like(arr)
    out[..., ids] = arr
    return out


def nerr(a, b):
    """Normwise error max|a - b| / max|b| (per field)."""
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def elem_rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b) / np.abs(b)))


PASS_FIELDS = ("H", "nk", "V", "B", "rho", "P", "grad", "dp", "dE", "vsig")


def compare_pass(st, ref, fields=PASS_FIELDS):
    """dict field -> normwise error of the GPU pass against oracle outputs `ref`."""
    return {f: nerr(in_input_order(st, f), ref[f]) for f in fields}


class ClosureUnsettled(AssertionError):
    pass


def oracle_sample(w, targets, pad: float = 1.5, doublings: int = 5, setup=None):
    """Oracle outputs at ``targets`` of workload ``w``, from oracle inputs only.
    The closure bound starts at ``pad`` times the largest oracle kernel length
    of the targets and is doubled (at most ``doublings`` times) until no kernel
    length the oracle solved inside the closure exceeds it."""
    from oracle import oracle as O
    s = setup or O.Setup.of(w)
    mask = np.zeros(w.n, dtype=bool)
    mask[np.asarray(targets)] = True
    H, _, _, _ = O.solve_h(s, w.x, w.y, w.z, None, mask=mask)
    h = pad * float(H[mask].max())
    for _ in range(doublings + 1):
        out = O.sampled_pass(s, w.arrays(), targets, h_bound=h)
        if float(out["H"].max()) <= h:
            return out
        h *= 2.0
    raise ClosureUnsettled("oracle closure bound did not settle")
