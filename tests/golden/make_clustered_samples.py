"""Writes clustered_16M_samples.json: oracle outputs of the full hydro pass at a
few particles of the 16,777,216-particle clustered log-normal set (the
benchmark's own set), for the MFM and the MFV form.

Every value comes from the FP64 oracle (oracle/): each target's dependency
closure is sized from the oracle's own kernel lengths and verified against
every kernel length solved inside it.  Targets are drawn with a fixed seed:
eight from the middle eighth of the density ranks, sampled in two groups
of four (the generator sets u from the cell density, so u ranks density).
A group takes the oracle minutes on one core, which is why the values are
stored; groups at the 75th percentile of density and above took it more
than five minutes each, so this set stays in the middle band.

    python tests/golden/make_clustered_samples.py [mfm|mfv|both]
"""
import dataclasses
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O                       # noqa: E402
from paper_1712_01294_amd import workloads as W      # noqa: E402
from tests.gpu_util import oracle_sample             # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "clustered_16M_samples.json")
FIELDS = ("H", "nk", "V", "rho", "P", "B", "grad", "dp", "dE", "vsig", "dm", "cond")


def targets(w):
    rng = np.random.default_rng(20171204)
    order = np.argsort(w.u, kind="stable")
    n = w.n
    mid = order[n // 2 - n // 16: n // 2 + n // 16]
    return rng.choice(mid, 8, replace=False)


def sample(w, tg, scheme):
    """Oracle outputs at the targets, each density group sampled on its own:
    a closure is sized from the largest kernel length of its targets, so a
    shared closure would give the dense targets the median-density radius."""
    s = dataclasses.replace(O.Setup.of(w), scheme=scheme)
    out = {k: [] for k in FIELDS}
    for group in (tg[:4], tg[4:]):
        ref = oracle_sample(w, group, setup=s)
        for k in FIELDS:
            v = np.asarray(ref[k])
            out[k].append(v[..., group] if v.ndim > 1 else v[group])
    return {k: np.concatenate(v, axis=-1).tolist() for k, v in out.items()}


def main():
    which = sys.argv[1] if len(sys.argv) > 1 else "both"
    w = W.clustered()
    tg = targets(w)
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    data.update({"workload": "clustered", "n": int(w.n), "targets": tg.tolist(),
                 "note": "oracle outputs (FP64) at the targets, per scheme; arrays of shape (k, targets)"})
    for scheme in (("mfm", "mfv") if which == "both" else (which,)):
        data[scheme] = sample(w, tg, scheme)
        print(scheme, "done", flush=True)
    with open(OUT, "w") as f:
        json.dump(data, f, indent=1)


if __name__ == "__main__":
    main()
