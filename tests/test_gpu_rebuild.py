"""GPU side of the numeric-only rebuild (psc_amg_rebuild): the device copies
are refreshed (V-cycle and solves against the oracle's build of 4A, which
reaches the same aggregates), captured iterations are dropped, solves on new
coefficients converge and agree with a V-cycle written from the exported
levels, and a failed rebuild makes the handle refuse work until a rebuild
succeeds. Tolerances as for the other parity tests."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as sla

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


CONFIGS = {
    "matching": (dict(), dict()),
    "smoothed_nu2": (dict(smoothed_prol=True, sweeps=3, smoother_sweeps=2), dict(prol=1, sweeps=3, nu=2)),
    "smoothed_device_products": (dict(smoothed_prol=True, sweeps=3, smoother_sweeps=2, setup_device_products=True),
                                 dict(prol=1, sweeps=3, nu=2)),
    "ainv": (dict(smoother=1), dict(smoother=1)),
    "cheb2": (dict(smoother=3, smoother_sweeps=2), dict(smoother=3, nu=2)),
}


@pytest.mark.parametrize("cfg", list(CONFIGS))
def test_rebuild_4a_matches_oracle_build_of_4a(psc, cfg):
    rp, c, v = P.poisson7(20)
    n = len(rp) - 1
    lo, oo = CONFIGS[cfg]
    h = psc.Hierarchy(rp, c, v, build_fp32=True, **lo)
    b = P.rhs_uniform(n, 1)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    h.pcg(dev(b), x)                                 # capture iteration graphs on the old buffers
    h.fcg(dev(b), x, prec=psc.FP32)
    h.rebuild(4.0 * v)
    o = oracle.Hierarchy(rp, c, 4.0 * v, **oo)
    r = np.random.default_rng(4).standard_normal(n)
    z = torch.empty(n, dtype=torch.float64, device="cuda")
    h.vcycle(dev(r), z)
    ref = o.vcycle(r)
    assert np.linalg.norm(z.cpu().numpy() - ref) <= 1e-12 * np.linalg.norm(ref)
    h.vcycle(dev(r), z, prec=psc.FP32)
    ref32 = o.vcycle32(r)
    assert np.linalg.norm(z.cpu().numpy() - ref32) <= 1e-5 * np.linalg.norm(ref32)
    b4 = P.rhs_from_solution(rp, c, 4.0 * v, P.x_true(n, 2))
    ro = o.pcg(b4)
    for fused in (1, 0):
        h.tune(psc.TUNE_FUSED_PCG, fused)
        x.zero_()
        g = h.pcg(dev(b4), x)
        assert g["status"] == psc.OK and abs(g["iters"] - ro["iters"]) <= 1 and g["relres"] <= 1e-6


REFRESH_CASES = {
    "poisson21": (lambda: P.poisson7(21), dict()),                       # DIA levels, ragged slices
    "diffusion20_az100": (lambda: P.diffusion7(20, seed=0, az=100.0), dict()),
    "random_long_rows": (lambda: P.random_spd_csr(700, 5, density=0.01, maxrow=90), dict(coarse_max=40)),
    "smoothed_nu2": (lambda: P.poisson7(17), dict(smoothed_prol=True, sweeps=3, smoother_sweeps=2)),
    "poisson20_pairs": (lambda: P.poisson7(20), dict()),                 # pair restriction on levels 0 and 1
    # capped hacked-ELL copies (every level where a cap pays): the stalled
    # lognormal coarse levels, and a random matrix's uneven rows
    "lognormal48_capped": (lambda: P.diffusion7(48, seed=0), dict(capped_min_rows=1)),
    "random_long_rows_capped": (lambda: P.random_spd_csr(700, 5, density=0.01, maxrow=90),
                                dict(coarse_max=40, capped_min_rows=1)),
}


@pytest.mark.parametrize("knob", ["default", "dia_off", "dia_per_slice", "split_off"])
@pytest.mark.parametrize("case", list(REFRESH_CASES))
def test_rebuilt_device_data_equal_a_fresh_build_bitwise(psc, case, knob):
    """The rebuild scatters new values into the build's ELL / DIA slots on the
    device; a fresh build on 4A reaches the same aggregates and exactly 4x
    the values, so every operator it reads must agree bit for bit."""
    gen, kw = REFRESH_CASES[case]
    rp, c, v = gen()
    if knob == "split_off" and kw.get("smoothed_prol"):
        pytest.skip("the unsplit sweep supports the tentative prolongator only")
    n = len(rp) - 1
    h = psc.Hierarchy(rp, c, v, build_fp32=True, **kw)
    h.rebuild(4.0 * v)
    f = psc.Hierarchy(rp, c, 4.0 * v, build_fp32=True, **kw)
    for q in (h, f):
        if knob == "dia_off":
            q.tune(psc.TUNE_DIA, 0)
        elif knob == "dia_per_slice":
            q.tune(psc.TUNE_DIA_UNIFORM, 0)
        elif knob == "split_off":
            q.tune(psc.TUNE_SPLIT, 0)
    assert h.info()["dia_slots"] == f.info()["dia_slots"]
    assert h.info()["capped_cap"] == f.info()["capped_cap"]
    assert h.info()["pair_restrict"] == f.info()["pair_restrict"]
    if case.endswith("_capped"):
        assert any(h.info()["capped_cap"])
    if case == "poisson20_pairs" and knob == "default":
        assert h.info()["pair_restrict"][:2] == [1, 1]
    r = dev(np.random.default_rng(8).standard_normal(n))
    outs = []
    for q in (h, f):
        y = torch.empty(n, dtype=torch.float64, device="cuda")
        z = torch.empty(n, dtype=torch.float64, device="cuda")
        z32 = torch.empty(n, dtype=torch.float64, device="cuda")
        q.spmv(r, y)
        q.vcycle(r, z)
        q.vcycle(r, z32, prec=psc.FP32)
        outs.append((y, z, z32))
    for a, b in zip(*outs):
        assert torch.equal(a, b)


def _vcycle_from_exports(h, r, fai=False):
    """V(1,1) written from the exported levels (scipy): l1-Jacobi, or the
    exported AINV / INVK factors G = Z D^-1 Z^T."""
    inf = h.info()
    L = inf["levels"]
    levs = [h.export_level(l) for l in range(L)]
    mats = [sp.csr_matrix((lv["val"], lv["col"], lv["rowptr"]), shape=(lv["n"], lv["n"])) for lv in levs]
    Ps = []
    for l in range(L - 1):
        prp, pci, pv = h.export_prolongator(l)
        Ps.append(sp.csr_matrix((pv, pci, prp), shape=(levs[l]["n"], levs[l + 1]["n"])))

    Gs = []
    for l in range(L - 1):
        if fai:
            zr, zi, zv, d = h.export_smoother(l)
            Z = sp.csc_matrix((zv, zi, zr), shape=(levs[l]["n"], levs[l]["n"]))
            Gs.append(lambda t, Z=Z, d=d: Z @ ((Z.T @ t) / d))
        else:
            Gs.append(lambda t, m=levs[l]["minv"]: m * t)

    def vc(l, b):
        A = mats[l]
        if l == L - 1:
            return np.linalg.solve(A.toarray(), b)
        x = Gs[l](b)
        xc = vc(l + 1, Ps[l].T @ (b - A @ x))
        x = x + Ps[l] @ xc
        return x + Gs[l](b - A @ x)
    return vc(0, r)


def test_rebuild_with_new_coefficients(psc):
    rp, c, v = P.diffusion7(20, seed=1)
    _, _, v2 = P.diffusion7(20, seed=5, az=20.0)
    n = len(rp) - 1
    h = psc.Hierarchy(rp, c, v, build_fp32=True)
    assert h.info()["coarse_sweeps"] == 0
    h.rebuild(v2)
    r = np.random.default_rng(6).standard_normal(n)
    z = torch.empty(n, dtype=torch.float64, device="cuda")
    h.vcycle(dev(r), z)
    ref = _vcycle_from_exports(h, r)
    assert np.linalg.norm(z.cpu().numpy() - ref) <= 1e-12 * np.linalg.norm(ref)
    b = P.rhs_from_solution(rp, c, v2, P.x_true(n, 3))
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    g = h.pcg(dev(b), x)
    assert g["status"] == psc.OK and g["relres"] <= 1e-6
    A2 = sp.csr_matrix((v2, c, rp))
    assert np.linalg.norm(b - A2 @ x.cpu().numpy()) <= 1.01e-6 * np.linalg.norm(b)
    x.zero_()
    g = h.fcg(dev(b), x, prec=psc.FP32)
    assert g["status"] == psc.OK and g["relres"] <= 1e-6


def test_failed_rebuild_refuses_work_until_a_rebuild_succeeds(psc):
    rp, c, v = P.poisson7(10)
    n = len(rp) - 1
    h = psc.Hierarchy(rp, c, v)
    bad = v.copy()
    bad[rp[7]:rp[8]][c[rp[7]:rp[8]] == 7] = 0.0
    with pytest.raises(psc.PscError) as e:
        h.rebuild(bad)
    assert e.value.status == psc.ERR_NOT_SPD
    b = P.rhs_uniform(n, 2)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(psc.PscError) as e:
        h.pcg(dev(b), x)
    assert e.value.status == psc.ERR_STATE
    with pytest.raises(psc.PscError):
        h.vcycle(dev(b), x)
    h.rebuild(v)
    g = h.pcg(dev(b), x)
    assert g["status"] == psc.OK and g["relres"] <= 1e-6


@pytest.mark.parametrize("smoother", [1, 2])
def test_rebuild_of_factored_smoothers_with_new_coefficients(psc, smoother):
    # AINV's pattern depends on the values (the rebuild may re-upload the
    # factors); INVK's does not (refreshed in place)
    rp, c, v = P.diffusion7(16, seed=2)
    _, _, v2 = P.diffusion7(16, seed=9, az=5.0)
    n = len(rp) - 1
    h = psc.Hierarchy(rp, c, v, build_fp32=True, smoother=smoother)
    b = P.rhs_uniform(n, 5)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    h.pcg(dev(b), x)
    h.rebuild(v2)
    r = np.random.default_rng(7).standard_normal(n)
    z = torch.empty(n, dtype=torch.float64, device="cuda")
    h.vcycle(dev(r), z)
    ref = _vcycle_from_exports(h, r, fai=True)
    assert np.linalg.norm(z.cpu().numpy() - ref) <= 1e-12 * np.linalg.norm(ref)
    b2 = P.rhs_from_solution(rp, c, v2, P.x_true(n, 4))
    x.zero_()
    g = h.pcg(dev(b2), x)
    assert g["status"] == psc.OK and g["relres"] <= 1e-6


def test_rebuild_refreshes_rows_beyond_one_full_grid(psc):
    """260^3 = 17.6 M rows: more rows than one launch of the capped grid
    covers (65536 workgroups of 256), so every refresh kernel must stride;
    the rebuilt handle's operators equal a fresh build on 4A bit for bit."""
    rp, c, v = P.poisson7(260)
    n = len(rp) - 1
    assert n > 65536 * 256
    r = dev(np.random.default_rng(9).standard_normal(n))
    f = psc.Hierarchy(rp, c, 4.0 * v)
    zf = torch.empty(n, dtype=torch.float64, device="cuda")
    yf = torch.empty(n, dtype=torch.float64, device="cuda")
    f.vcycle(r, zf)
    f.spmv(r, yf)
    f.close()
    h = psc.Hierarchy(rp, c, v)
    h.rebuild(4.0 * v)
    z = torch.empty(n, dtype=torch.float64, device="cuda")
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    h.vcycle(r, z)
    h.spmv(r, y)
    assert torch.equal(y, yf) and torch.equal(z, zf)


def test_staging_memory_is_released_after_build_rebuild_and_free(psc):
    """The device staging of CSR rows and values (here about 140 MB) lives
    only while a build or a rebuild fills the level data: the memory a handle
    holds is the same after its build and after a rebuild, and freeing the
    handle returns everything."""
    rp, c, v = P.poisson7(128)
    stage = 4 * len(rp) + 8 * len(v) + 8 * (len(rp) - 1)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    h = psc.Hierarchy(rp, c, v, build_fp32=True)
    free1, _ = torch.cuda.mem_get_info()
    h.rebuild(2.0 * v)
    free2, _ = torch.cuda.mem_get_info()
    assert abs(free1 - free2) < stage / 4
    h.close()
    free3, _ = torch.cuda.mem_get_info()
    assert abs(free0 - free3) < 16 << 20
