"""GPU parity of the AINV / INVK smoothers (Section "GPU enabled smoothers")
against the CPU oracle, through the C ABI.

The factors are built on the host bit-identical to the oracle's; the device
applies each sweep x <- x + Z (D^-1 Z^T (b - A x)) with hacked-ELL products.
Tolerances as for the l1-Jacobi V-cycle: 1e-12 relative (FP64; summation
order and FMA only), 1e-5 relative to the oracle's FP32 V-cycle, solves
within +-1 iteration and 1e-8 at equal iteration count.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle
from paper_2406_19754_amd import problems as P


@pytest.fixture(scope="module")
def psc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_19754_amd import psc as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


CASES = {
    "poisson24": lambda: P.poisson7(24),
    "diffusion20": lambda: P.diffusion7(20, seed=0),
    "poisson13": lambda: P.poisson7(13),
    "diffusion20_az100": lambda: P.diffusion7(20, seed=0, az=100.0),
    "random_long_rows": lambda: P.random_spd_csr(700, 5, density=0.01, maxrow=90),
}

CONFIGS = {
    # name: (library options, oracle options)
    "ainv": (dict(smoother=1), dict(smoother=1)),
    "invk": (dict(smoother=2), dict(smoother=2)),
    "invk_11": (dict(smoother=2, invk_fill=1, invk_inv_fill=1), dict(smoother=2, invk_fill=1, invk_inv_fill=1)),
    "invk_00": (dict(smoother=2, invk_inv_fill=0), dict(smoother=2, invk_inv_fill=0)),
    "ainv_tau003_nu2": (dict(smoother=1, ainv_tau=0.03, smoother_sweeps=2), dict(smoother=1, ainv_tau=0.03, nu=2)),
    "ainv_smoothed": (dict(smoother=1, smoothed_prol=True, sweeps=3, smoother_sweeps=2),
                      dict(smoother=1, prol=1, sweeps=3, nu=2)),
    "invk_variable": (dict(smoother=2, sweeps=3, vcycle_double=True), dict(smoother=2, sweeps=3, nu_double=True)),
}


def _pair(psc, case, cfg):
    rp, c, v = CASES[case]()
    cm = 40 if case == "random_long_rows" else 200
    lo, oo = CONFIGS[cfg]
    h = psc.Hierarchy(rp, c, v, coarse_max=cm, build_fp32=True, **lo)
    o = oracle.Hierarchy(rp, c, v, coarse_max=cm, **oo)
    return rp, c, v, h, o


@pytest.mark.parametrize("cfg", list(CONFIGS))
@pytest.mark.parametrize("case", list(CASES))
def test_fai_vcycle_matches_oracle(psc, case, cfg):
    rp, c, v, h, o = _pair(psc, case, cfg)
    inf = h.info()
    assert inf["rows"] == o.sizes() and inf["levels"] >= 2
    assert all(inf["smoother_nnz"][l] >= inf["rows"][l] for l in range(inf["levels"] - 1))
    n = len(rp) - 1
    for seed in (5, 6):
        x = np.random.default_rng(seed).standard_normal(n)
        y = torch.empty(n, dtype=torch.float64, device="cuda")
        h.vcycle(dev(x), y)
        ref = o.vcycle(x)
        assert np.linalg.norm(y.cpu().numpy() - ref) <= 1e-12 * np.linalg.norm(ref)
        h.vcycle(dev(x), y, prec=psc.FP32)
        ref32 = o.vcycle32(x)
        assert np.linalg.norm(y.cpu().numpy() - ref32) <= 1e-5 * np.linalg.norm(ref32)


@pytest.mark.parametrize("case,cfg", [(c, f) for c in ["poisson24", "diffusion20", "random_long_rows"]
                                      for f in ["ainv", "invk", "ainv_tau003_nu2", "ainv_smoothed"]]
                         + [("diffusion20_az100", "ainv")])
def test_fai_solves_match_oracle(psc, case, cfg):
    rp, c, v, h, o = _pair(psc, case, cfg)
    n = len(rp) - 1
    b = P.rhs_from_solution(rp, c, v, P.x_true(n, 1))
    r = o.pcg(b)
    assert r["status"] == oracle.OK
    xg = torch.zeros(n, dtype=torch.float64, device="cuda")
    for fused in (1, 0):
        h.tune(psc.TUNE_FUSED_PCG, fused)
        xg.zero_()
        g = h.pcg(dev(b), xg)
        assert g["status"] == psc.OK and abs(g["iters"] - r["iters"]) <= 1 and g["relres"] <= 1e-6
    k = min(g["iters"], r["iters"])
    xg.zero_()
    h.pcg(dev(b), xg, rtol=1e-30, maxit=k)
    refk = o.pcg(b, rtol=1e-30, maxit=k)["x"]
    assert np.linalg.norm(xg.cpu().numpy() - refk) <= 1e-8 * np.linalg.norm(refk)
    for fused in (1, 0):
        h.tune(psc.TUNE_FUSED_PCG, fused)
        for form, prec in ((0, psc.FP64), (1, psc.FP32)):
            rf = o.fcg(b, form=form)
            xg.zero_()
            g = h.fcg(dev(b), xg, prec=prec)
            assert g["status"] == psc.OK and abs(g["iters"] - rf["iters"]) <= 1 and g["relres"] <= 1e-6


def test_fai_smoother_reduces_iterations(psc):
    rp, c, v = P.poisson7(32)
    n = len(rp) - 1
    b = P.rhs_uniform(n, 2)
    its = {}
    for name, kw in [("l1", {}), ("ainv", dict(smoother=1)), ("invk", dict(smoother=2))]:
        h = psc.Hierarchy(rp, c, v, **kw)
        x = torch.zeros(n, dtype=torch.float64, device="cuda")
        g = h.pcg(dev(b), x)
        assert g["status"] == psc.OK and g["relres"] <= 1e-6
        its[name] = g["iters"]
    assert its["ainv"] <= 0.75 * its["l1"] and its["invk"] <= 0.75 * its["l1"]


def test_fai_with_jacobi_coarsest_and_single_level(psc):
    # coarsening stalls above 2000 rows: the coarsest keeps its l1-Jacobi
    # sweeps, the levels above use AINV
    rp, c, v = P.diffusion7(48, seed=0)
    h = psc.Hierarchy(rp, c, v, build_fp32=True, smoother=1)
    o = oracle.Hierarchy(rp, c, v, smoother=1)
    assert h.info()["coarse_sweeps"] == 30 == o.coarse_sweeps
    n = len(rp) - 1
    x = np.random.default_rng(8).standard_normal(n)
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    h.vcycle(dev(x), y)
    ref = o.vcycle(x)
    assert np.linalg.norm(y.cpu().numpy() - ref) <= 1e-12 * np.linalg.norm(ref)
    h.vcycle(dev(x), y, prec=psc.FP32)
    ref32 = o.vcycle32(x)
    assert np.linalg.norm(y.cpu().numpy() - ref32) <= 1e-5 * np.linalg.norm(ref32)
    # one level only: the coarsest solve is the whole preconditioner
    rp, c, v = P.poisson7(5)
    h = psc.Hierarchy(rp, c, v, smoother=2)
    assert h.info()["levels"] == 1
    b = P.rhs_uniform(125, 1)
    xg = torch.zeros(125, dtype=torch.float64, device="cuda")
    g = h.pcg(dev(b), xg)
    assert g["status"] == psc.OK and g["iters"] == 1


def test_invk_breakdown_under_strong_anisotropy_is_reported(psc):
    # a_z = 100: the level-limited inverse of the incomplete factor overshoots
    # (the largest eigenvalue of G A on level 0 is about 15), the V-cycle is
    # no longer positive definite and CG breaks down at once -- in the oracle
    # and in the library alike, reported as a breakdown, not as a result
    rp, c, v = CASES["diffusion20_az100"]()
    n = len(rp) - 1
    b = P.rhs_from_solution(rp, c, v, P.x_true(n, 1))
    r = oracle.Hierarchy(rp, c, v, smoother=2).pcg(b)
    assert r["status"] == oracle.ERR_NOT_SPD
    h = psc.Hierarchy(rp, c, v, smoother=2)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(psc.PscError) as e:
        h.pcg(dev(b), x)
    assert e.value.status == psc.ERR_NOT_SPD
