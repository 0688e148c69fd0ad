"""Write the oracle's values for the accuracy-versus-cost curve on the water box
(tests/golden/curve_water26k.json).

Calls only the FP64 oracle (oracle/) on the seeded water box of 26,268 charges
(paper_1911_01377_amd.synth, which holds no u-series arithmetic).  One entry
per series construction, each with the parameters of its table row (typed
from paper_values.json, which cites the tables), sigma = r_c / r0 (Sec. III.C,
eq. 23) and the smallest N whose eq. 33 bound is at most 1e-8:

  C1_b2     Table 2, C1 row (the default series)
  C2_b2     Table 2, C2 row (eq. 28, with s0)
  T1_row1   Table 1, first C2 point of the C1 construction (b = 1.63)
  T1_row2   Table 1, second (b = 1.32)
  T1_row3   Table 1, third (b = 1.22)

plus "coulomb": Table 1 row 3 with N at an eq. 33 bound of 1e-12.  Its
series differs from 1/r by at most about M_b = 3.9e-11 (eq. 14), so it
stands for the exact periodic Coulomb energy and forces (the oracle agrees
with a converged Ewald sum to 1e-9 with these parameters).

Stored per entry: the parameters, the energy parts, the RMS force and the
forces on the same 512 seeded charges as oracle_water26k.json.

    python tests/golden/make_curve.py [entry ...]
"""
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1911_01377_amd import synth  # noqa: E402

OUT = os.path.join(HERE, "curve_water26k.json")
RC = 9.0


def table_rows():
    pv = json.load(open(os.path.join(HERE, "paper_values.json")))
    t2 = pv["table2_b2"]
    rows = {
        "C1_b2": (2.0, t2["C1"]),
        "C2_b2": (2.0, t2["C2"]),
    }
    for k, r in enumerate(pv["table1_c2_points_of_c1_construction"]["rows"]):
        rows["T1_row%d" % (k + 1)] = (float(r["b"]), dict(r, s0="1.0"))
    out = {}
    for name, (b, r) in rows.items():
        out[name] = dict(b=b, r0=float(r["r0"]), w0=float(r["w0"]), s0=float(r["s0"]))
    out["coulomb"] = dict(out["T1_row3"], tol=1e-12)
    return out


def params(row, L):
    sigma = RC / row["r0"]
    tol = row.get("tol", 1e-8)
    n = 1
    while oracle.eq33_bound(n, row["b"], sigma, L) > tol:
        n += 1
    return oracle.Params(b=row["b"], sigma=sigma, w0=row["w0"], s0=row["s0"], rc=RC, nterms=n)


def main(names):
    xyz, q, box = synth.WORKLOADS["water26k"]()
    x64, q64 = xyz.astype(np.float64), q.astype(np.float64)
    idx = np.sort(np.random.default_rng(2024).choice(len(q), 512, replace=False))
    data = json.load(open(OUT)) if os.path.exists(OUT) else {
        "_what": "FP64 oracle values per series construction for the water box of 26,268 "
                 "charges (written by tests/golden/make_curve.py)",
        "sample_idx": idx.tolist(), "entries": {}}
    rows = table_rows()
    for name in names or list(rows):
        p = params(rows[name], max(box))
        t = time.time()
        parts, f = oracle.eval_full(x64, q64, box, p)
        dt = time.time() - t
        data["entries"][name] = {
            "params": {"b": p.b, "sigma": p.sigma, "w0": p.w0, "s0": p.s0, "rc": p.rc,
                       "nterms": p.nterms, "eq33_tol": rows[name].get("tol", 1e-8)},
            "parts": {k: float(v) for k, v in parts.items()},
            "force_rms": float(math.sqrt(np.mean(np.sum(f * f, axis=1)))),
            "sample_forces": f[idx].tolist(),
            "oracle_seconds": dt, "oracle_threads": oracle.num_threads(),
        }
        with open(OUT, "w") as fh:
            json.dump(data, fh)
        print("%s: N=%d E=%.12f (%.0f s on %d threads)"
              % (name, p.nterms, parts["total"], dt, oracle.num_threads()), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
