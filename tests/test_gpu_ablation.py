"""What the trained network gains: the learned form's schedule (FCG(1), the
alternate step on iterations 1, 3, 5, ..., V-cycle fallback and switch-off
rules) run with four choices of the alternate step, on 3D Poisson with
held-out right-hand sides U[-1,1] (seeds 1001, 1002; training used 1-64 and
101-132):

  vcycle     no alternate step: FCG(1) with the V-cycle on every iteration
  trained    the shipped network trained on 128^3 pairs
             (paper_2406_19754_amd/weights/net_poisson128.ckpt)
  untrained  the same architecture at its seeded initialisation
  l1jacobi   one l1-Jacobi sweep from zero, z = M_0^-1 r

Reported per grid and arm: iterations, scheduled steps that fell back to the
V-cycle, and the solve time. At 32^3 every arm is also run by the CPU oracle
and must agree (iterations within one, fallbacks equal). The gains are
printed, not asserted: the test records them, whatever their sign.
"""
import os
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle
from paper_2406_19754_amd import problems as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CKPT = os.path.join(ROOT, "paper_2406_19754_amd", "weights", "net_poisson128.ckpt")
SEEDS = [1001, 1002]


@pytest.fixture(scope="module")
def psc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_19754_amd import psc as m
    return m


def _trained_params():
    blob = open(CKPT, "rb").read()
    return np.frombuffer(blob[40:40 + 4 * 7809], dtype="<f4").astype(np.float64)


@pytest.mark.parametrize("n", [32, 48, 64])
def test_alternate_step_ablation(psc, n):
    rp, c, v = P.poisson7(n)
    N = n ** 3
    h = psc.Hierarchy(rp, c, v)
    arms = {"vcycle": None, "trained": psc.Net.load(CKPT), "untrained": psc.Net(P.net_init(5).astype(np.float32)),
            "l1jacobi": psc.Net.l1jacobi(h)}
    for name in ("trained", "untrained"):
        arms[name].set_grid((n, n, n))
    o = oracle.Hierarchy(rp, c, v) if n == 32 else None
    rows = []
    for seed in SEEDS:
        b = torch.from_numpy(P.rhs_uniform(N, seed)).cuda()
        x = torch.zeros(N, dtype=torch.float64, device="cuda")
        res = {}
        for name, net in arms.items():
            x.zero_()
            h.fcg(b, x, net=net)                  # warm-up (graph capture)
            x.zero_()
            torch.cuda.synchronize()
            t = time.perf_counter()
            g = h.fcg(b, x, net=net)
            torch.cuda.synchronize()
            g["ms"] = (time.perf_counter() - t) * 1e3
            assert g["status"] == psc.OK and g["relres"] <= 1e-6, (n, seed, name, g)
            res[name] = g
            if o is not None:
                bh = b.cpu().numpy()
                if name == "vcycle":
                    r = o.fcg(bh)
                elif name == "l1jacobi":
                    r = o.fcg(bh, alt_jacobi=True)
                else:
                    p = _trained_params() if name == "trained" else P.net_init(5).astype(np.float32).astype(np.float64)
                    r = o.fcg(bh, params=p, dims=(n, n, n))
                assert abs(g["iters"] - r["iters"]) <= 1, (name, g["iters"], r["iters"])
                assert g["fallbacks"] == r["fallbacks"] or abs(g["iters"] - r["iters"]) == 1, (name, g, r)
        rows.append((seed, res))
    print(f"\n[ablation] Poisson {n}^3, FCG(1) to rtol 1e-6, held-out U[-1,1] right-hand sides")
    print("[ablation] seed  arm        iters  fallbacks   ms    gain vs V-cycle only (iterations, time)")
    for seed, res in rows:
        base = res["vcycle"]
        for name, g in res.items():
            print(f"[ablation] {seed}  {name:10s} {g['iters']:5d}  {g['fallbacks']:9d}  {g['ms']:6.2f}   "
                  f"{base['iters'] - g['iters']:+d} its, x{base['ms'] / g['ms']:.2f}", flush=True)
