"""Write tests/golden/poisson256_oracle.json: reference values of the CPU
oracle for the 256^3 Poisson workload (b = A x_true, x_true ~ U[0,1) seed 0,
rtol 1e-6), used by the full-size GPU parity test. Calls only oracle/ and the
seeded input generators. Takes about two minutes on one core.

    python tests/golden/make_poisson256.py
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2406_19754_amd import problems as P  # noqa: E402

N_SIDE = 256
SAMPLES = 2048


def main():
    n = N_SIDE
    N = n ** 3
    t0 = time.time()
    rp, col, val = P.poisson7(n)
    xt = P.x_true(N, 0)
    b = P.rhs_from_solution(rp, col, val, xt)
    h = oracle.Hierarchy(rp, col, val)
    levels = []
    for l in range(h.nlevels):
        L = h.level(l)
        entry = {"rows": L["n"], "nnz": L["nnz"]}
        if L["agg"] is not None:
            entry["agg_sha256"] = hashlib.sha256(L["agg"].astype("<i4").tobytes()).hexdigest()
        entry["val_sha256"] = hashlib.sha256(L["val"].astype("<f8").tobytes()).hexdigest()
        levels.append(entry)
    idx = np.sort(np.random.default_rng(123).choice(N, SAMPLES, replace=False))
    r7 = P.rhs_uniform(N, 7)
    z7 = h.vcycle(r7)
    res = h.pcg(b, rtol=1e-6, maxit=500)
    out = {
        "workload": f"3D Poisson 7-point {n}^3, b = A x_true, x_true = default_rng(0).random(N), x0 = 0, rtol 1e-6",
        "levels": levels,
        "operator_complexity": h.operator_complexity(),
        "vcycle_rhs": "rhs_uniform(N, 7)",
        "vcycle_norm": float(np.linalg.norm(z7)),
        "pcg_iters": res["iters"],
        "pcg_relres": res["relres"],
        "x_norm": float(np.linalg.norm(res["x"])),
        "sample_idx": idx.tolist(),
        "vcycle_sample": z7[idx].tolist(),
        "x_sample": res["x"][idx].tolist(),
        "seconds": time.time() - t0,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "poisson256_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"wrote {path}: {res['iters']} iterations, relres {res['relres']:.3e}, {out['seconds']:.0f}s")


if __name__ == "__main__":
    main()
