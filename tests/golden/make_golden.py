"""Write the full-size reference files of the CPU oracle used by the GPU
parity tests (tests/test_gpu_full.py). Calls only oracle/ and the seeded
input generators of paper_2406_19754_amd/problems.py.

Workloads (b = A x_true, x_true = default_rng(0).random(N), x0 = 0):
  poisson256    3D Poisson 7-point 256^3, FP64 PCG
  diffusion256  lognormal diffusion 256^3 (log k ~ N(0, 1.5^2) seed 0,
                a_z = 1), FP64 PCG and FCG(1) with the FP32 V-cycle
  poisson384    3D Poisson 7-point 384^3, FP64 PCG

For each solve the file holds the iteration count o at rtol 1e-6 and, for
the iterates after o-1, o and o+1 iterations, 2048 sampled entries, the norm
and PROJ projections onto the +-1 vectors of problems.projection_signs, so a
solve that stops one iteration earlier or later is compared at equal count.
Also the hash of every level's aggregate map and values, and a sampled
V-cycle. Run with the oracle built (about five minutes on 8 threads):

    python tests/golden/make_golden.py [poisson256 diffusion256 poisson384]
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

SAMPLES = 2048
PROJ = 8
HERE = os.path.dirname(os.path.abspath(__file__))


def problem(name):
    if name.startswith("poisson"):
        n = int(name[len("poisson"):])
        rp, col, val = P.poisson7(n)
        desc = f"3D Poisson 7-point {n}^3"
    else:
        n = int(name[len("diffusion"):])
        rp, col, val = P.diffusion7(n, seed=0, sigma=1.5, az=1.0)
        desc = f"3D lognormal diffusion {n}^3, log k ~ N(0, 1.5^2) seed 0, a_z = 1"
    return n, rp, col, val, desc


def summary(x, idx, W):
    return {"sample": x[idx].tolist(), "norm": float(np.linalg.norm(x)), "proj": [float(w @ x) for w in W]}


def solve_family(run, idx, W):
    """run(rtol, maxit) -> oracle result; the iterates after o-1, o, o+1 steps."""
    base = run(1e-6, 500)
    o = base["iters"]
    out = {"iters": o, "relres": base["relres"], "at": {}}
    for k in (o - 1, o, o + 1):
        if k < 1:
            continue
        x = base["x"] if k == o else run(1e-30, k)["x"]
        out["at"][str(k)] = summary(x, idx, W)
    return out


def make(name):
    t0 = time.time()
    n, rp, col, val, desc = problem(name)
    N = n ** 3
    b = P.rhs_from_solution(rp, col, val, P.x_true(N, 0))
    h = oracle.Hierarchy(rp, col, val)
    levels = []
    for l in range(h.nlevels):
        L = h.level(l)
        e = {"rows": L["n"], "nnz": L["nnz"]}
        if L["agg"] is not None:
            e["agg_sha256"] = hashlib.sha256(L["agg"].astype("<i4").tobytes()).hexdigest()
        e["val_sha256"] = hashlib.sha256(L["val"].astype("<f8").tobytes()).hexdigest()
        levels.append(e)
    idx = np.sort(np.random.default_rng(123).choice(N, SAMPLES, replace=False))
    W = [P.projection_signs(N, j) for j in range(PROJ)]
    z7 = h.vcycle(P.rhs_uniform(N, 7))
    out = {"workload": desc + ", b = A x_true, x_true = default_rng(0).random(N), x0 = 0, rtol 1e-6",
           "n": n, "levels": levels, "operator_complexity": h.operator_complexity(),
           "sample_idx": idx.tolist(), "proj_count": PROJ,
           "vcycle_rhs": "rhs_uniform(N, 7)", "vcycle_norm": float(np.linalg.norm(z7)),
           "vcycle_sample": z7[idx].tolist()}
    out["pcg"] = solve_family(lambda rtol, maxit: h.pcg(b, rtol=rtol, maxit=maxit), idx, W)
    if name.startswith("diffusion"):
        out["fcg32"] = solve_family(lambda rtol, maxit: h.fcg(b, rtol=rtol, maxit=maxit, form=1), idx, W)
    out["seconds"] = time.time() - t0
    path = os.path.join(HERE, f"{name}_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"wrote {path}: PCG {out['pcg']['iters']} its"
          + (f", FP32-V-cycle FCG {out['fcg32']['iters']} its" if "fcg32" in out else "")
          + f", {out['seconds']:.0f}s", flush=True)


if __name__ == "__main__":
    for name in sys.argv[1:] or ["poisson256", "diffusion256", "poisson384"]:
        make(name)
