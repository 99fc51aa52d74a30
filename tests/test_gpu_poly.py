"""GPU parity of the polynomial (fourth-kind Chebyshev) smoother against the
CPU oracle, through the C ABI. Tolerances as for the l1-Jacobi V-cycle:
1e-12 relative (FP64), 1e-5 relative to the oracle's FP32 V-cycle, solves
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
    "poisson13": lambda: P.poisson7(13),
    "diffusion20_az100": lambda: P.diffusion7(20, seed=0, az=100.0),
    "random_long_rows": lambda: P.random_spd_csr(700, 5, density=0.01, maxrow=90),
    "diffusion48_lognormal": lambda: P.diffusion7(48, seed=0),      # stalled: Jacobi coarsest
}

CONFIGS = {
    # name: (library options, oracle options)
    "deg1": (dict(smoother=3), dict(smoother=3)),
    "deg2": (dict(smoother=3, smoother_sweeps=2), dict(smoother=3, nu=2)),
    "deg3": (dict(smoother=3, smoother_sweeps=3), dict(smoother=3, nu=3)),
    "deg2_variable": (dict(smoother=3, smoother_sweeps=2, sweeps=3, vcycle_double=True),
                      dict(smoother=3, nu=2, sweeps=3, nu_double=True)),
    "deg2_smoothed": (dict(smoother=3, smoother_sweeps=2, sweeps=3, smoothed_prol=True),
                      dict(smoother=3, nu=2, sweeps=3, prol=1)),
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
def test_poly_vcycle_matches_oracle(psc, case, cfg):
    if case == "diffusion48_lognormal" and cfg not in ("deg1", "deg2"):
        pytest.skip("the stalled case is covered by the plain degrees")
    rp, c, v, h, o = _pair(psc, case, cfg)
    inf = h.info()
    assert inf["rows"] == o.sizes() and inf["smoother"] == 3
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


@pytest.mark.parametrize("cfg", ["deg1", "deg2", "deg3", "deg2_smoothed"])
@pytest.mark.parametrize("case", ["poisson24", "diffusion20_az100", "random_long_rows"])
def test_poly_solves_match_oracle(psc, case, cfg):
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


def test_poly_smoother_beats_l1_sweeps_of_the_same_count(psc):
    rp, c, v = P.poisson7(32)
    n = len(rp) - 1
    b = P.rhs_uniform(n, 2)
    its = {}
    for name, kw in [("l1_2", dict(smoother_sweeps=2)), ("cheb_2", dict(smoother=3, smoother_sweeps=2))]:
        h = psc.Hierarchy(rp, c, v, **kw)
        x = torch.zeros(n, dtype=torch.float64, device="cuda")
        g = h.pcg(dev(b), x)
        assert g["status"] == psc.OK and g["relres"] <= 1e-6
        its[name] = g["iters"]
    assert its["cheb_2"] < its["l1_2"]


@pytest.mark.parametrize("knob", ["split_off", "tail_4096", "dia_off"])
def test_degree_one_runs_on_the_l1_path_with_every_variant(psc, knob):
    # degree 1 is l1-Jacobi weighted 4/3: the weight sits in M^-1, A M^-1 and
    # (I - M^-1 A) P, so every kernel variant of the l1 path applies
    rp, c, v = P.poisson7(13)
    h = psc.Hierarchy(rp, c, v, build_fp32=True, smoother=3)
    o = oracle.Hierarchy(rp, c, v, smoother=3)
    if knob == "split_off":
        h.tune(psc.TUNE_SPLIT, 0)
    elif knob == "tail_4096":
        h.tune(psc.TUNE_TAIL, 4096)
    else:
        h.tune(psc.TUNE_DIA, 0)
    n = len(rp) - 1
    x = np.random.default_rng(3).standard_normal(n)
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    h.vcycle(dev(x), y)
    ref = o.vcycle(x)
    assert np.linalg.norm(y.cpu().numpy() - ref) <= 1e-12 * np.linalg.norm(ref)
    h.vcycle(dev(x), y, prec=psc.FP32)
    ref32 = o.vcycle32(x)
    assert np.linalg.norm(y.cpu().numpy() - ref32) <= 1e-5 * np.linalg.norm(ref32)
    b = P.rhs_uniform(n, 4)
    xg = torch.zeros(n, dtype=torch.float64, device="cuda")
    g = h.pcg(dev(b), xg)
    r = o.pcg(b)
    assert abs(g["iters"] - r["iters"]) <= 1 and g["relres"] <= 1e-6
