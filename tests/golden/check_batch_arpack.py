"""The stored runs of the 64-pencil batched workload (cfg2_oracle.json) against
shift-invert ARPACK on every pencil (about ten minutes on eight cores):

    python -m tests.golden.check_batch_arpack

For each pencil: the eigenvalues ARPACK finds in the region, the clusters, and every
eigenvalue farther than two last-level square widths from all cluster centres, with
the fate of its squares in the stored run (the level at which its square was
rejected, and its position in that square in units of the width; or "admitted" when
the square reached the last level and only the cluster's centre is far).  It reads
the stored runs and calls no part of the library or of the oracle.
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

from tests import arpack_ref
from workloads import make_batch

HERE = os.path.dirname(os.path.abspath(__file__))


def fate(run, prm, z):
    x0, y0 = prm["x0"], prm["y0"]
    w1 = (prm["x1"] - x0) / prm["n1"]
    for L in run["levels"]:
        w = w1 / 2 ** (L["level"] - 1)
        ix, iy = int(np.floor((z.real - x0) / w)), int(np.floor((z.imag - y0) / w))
        keys = list(zip(L["ix"], L["iy"]))
        if (ix, iy) not in keys:
            return f"not tested at level {L['level']}"
        r = keys.index((ix, iy))
        if L["decision"][r] == 0:
            return (f"rejected at level {L['level']}, at ({(z.real - x0) / w - ix:.3f}, "
                    f"{(z.imag - y0) / w - iy:.3f}) of its square")
    return "admitted"


def main() -> int:
    with open(os.path.join(HERE, "cfg2_oracle.json")) as fh:
        gold = json.load(fh)
    batch = make_batch("cfg2")
    total = far = rejected = 0
    for i in sorted(range(len(batch)), key=lambda q: batch[q][0].n):
        pen, _, prm = batch[i]
        run = gold["runs"][i]
        ncl = len(run["clusters"])
        try:
            eigs = arpack_ref.eigenvalues_in_region(pen, prm["x0"], prm["x1"], prm["y0"], prm["y1"], nx=2, ny=2,
                                                    k=min(pen.n - 2, max(40, int(0.8 * ncl) + 20)))
        except AssertionError:
            eigs = arpack_ref.eigenvalues_in_region(pen, prm["x0"], prm["x1"], prm["y0"], prm["y1"], nx=3, ny=3,
                                                    k=min(pen.n - 2, max(40, int(0.5 * ncl) + 20)))
        w = (prm["x1"] - prm["x0"]) / prm["n1"] / 2 ** (run["K"] - 1)
        lam = np.array([complex(*c["lam"]) for c in run["clusters"]])
        out = [e for e in eigs if float(np.min(np.abs(lam - e))) > 2 * w]
        total += len(eigs)
        far += len(out)
        print(f"pencil {i}: n = {pen.n}, {ncl} clusters, {len(eigs)} eigenvalues in R, {len(out)} far", flush=True)
        for e in out:
            f = fate(run, prm, e)
            rejected += f.startswith("rejected")
            print(f"    {e.real:+.6f}{e.imag:+.6f}i: {f}", flush=True)
    print(f"{total} eigenvalues, {far} far from every cluster centre, {rejected} of them in a rejected square")
    return 0


if __name__ == "__main__":
    sys.exit(main())
