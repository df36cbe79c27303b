"""Writes the stored expected results of full SIM-M runs.  Calls only the CPU
oracle (oracle/simm.py) on the seeded workloads; nothing here comes from the
HIP library.  Usage: python tests/golden/make_golden.py cfg0 [cfg1 ...]"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle.simm as O  # noqa: E402
from workloads import make_workload  # noqa: E402


def cplx(z):
    return [float(np.real(z)), float(np.imag(z))]


def main(names):
    for name in names:
        pen, f, params = make_workload(name)
        t0 = time.time()
        res = O.simm(pen, f, params)
        out = {
            "workload": name,
            "generated_by": "oracle/simm.py via tests/golden/make_golden.py",
            "oracle_seconds": round(time.time() - t0, 1),
            "K": res.K,
            "shifts": [{"sigma": cplx(s.sigma), "beta": s.beta, "m_eff": s.m_eff, "h_last": s.h_last,
                        "H_diag": [cplx(v) for v in np.diag(s.Hm)],
                        "H_sub": [float(np.real(v)) for v in np.diag(s.H, -1)]} for s in res.shifts],
            "levels": [{"level": L.level,
                        "ix": [int(v) for v in L.keys[:, 0]], "iy": [int(v) for v in L.keys[:, 1]],
                        "shift": [int(v) for v in L.shift], "decision": [int(v) for v in L.decision],
                        "indicator": [float(v) for v in L.indicator], "rho_max": [float(v) for v in L.rho_max],
                        "margin": [float(v) for v in L.margin]} for L in res.levels],
            "clusters": [{"lam": cplx(c.lam), "lam_ritz": cplx(c.lam_ritz), "shift": c.shift,
                          "unresolved": c.unresolved, "members": c.members} for c in res.clusters],
        }
        path = os.path.join(HERE, f"{name}_oracle.json")
        with open(path, "w") as fh:
            json.dump(out, fh, separators=(",", ":"))
        print(name, "->", path, f"{out['oracle_seconds']} s, {len(res.shifts)} shifts, {len(res.clusters)} clusters")


if __name__ == "__main__":
    main(sys.argv[1:] or ["cfg0"])
