"""Host setup of the library (locally-dominant matching, canonical Galerkin
sums) against the oracle (sorted-greedy matching): the hierarchies must be
bit-identical. Runs on the CPU through the C ABI with host_only=1."""
import numpy as np
import pytest

import oracle
from paper_2406_19754_amd import problems as P
from paper_2406_19754_amd import psc

def _block_diag(*mats):
    rps, cs, vs, off, nnz = [np.zeros(1, np.int32)], [], [], 0, 0
    for rp, c, v in mats:
        rps.append((rp[1:] + nnz).astype(np.int32))
        cs.append((c + off).astype(np.int32))
        vs.append(v)
        off += len(rp) - 1
        nnz += rp[-1]
    return np.concatenate(rps), np.concatenate(cs), np.concatenate(vs)


CASES = {
    "poisson32": (lambda: P.poisson7(32), 200, 2),
    "poisson9": (lambda: P.poisson7(9), 200, 2),
    "poisson24_aggr8": (lambda: P.poisson7(24), 200, 3),
    "diffusion16_lognormal_az100": (lambda: P.diffusion7(16, seed=0, az=100.0), 200, 2),
    "diffusion14_lognormal_az0.01": (lambda: P.diffusion7(14, seed=2, az=0.01), 100, 2),
    "random_spd": (lambda: P.random_spd_csr(500, 3, density=0.02, maxrow=50), 40, 2),
    "diffusion48_lognormal_stalls": (lambda: P.diffusion7(48, seed=0), 200, 2),
    # degenerate: one row; a diagonal matrix (nothing to match, stalls at once);
    # two disconnected Poisson blocks of different sizes
    "one_by_one": (lambda: (np.array([0, 1], np.int32), np.array([0], np.int32), np.array([4.0])), 200, 2),
    "diagonal_3000": (lambda: (np.arange(3001, dtype=np.int32), np.arange(3000, dtype=np.int32),
                               1.0 + np.random.default_rng(4).random(3000)), 200, 2),
    "two_components": (lambda: _block_diag(P.poisson7(10), P.poisson7(9)), 200, 2),
}

# smoothed prolongator (general Galerkin product); aggregates <= 8 is the
# paper's SMATCH setting
SMOOTHED = {
    "poisson24_smatch": (lambda: P.poisson7(24), 200, 3),
    "poisson9_smoothed": (lambda: P.poisson7(9), 40, 2),
    "diffusion12_az100_smoothed": (lambda: P.diffusion7(12, seed=0, az=100.0), 100, 3),
    "random_spd_smoothed": (lambda: P.random_spd_csr(400, 3, density=0.02, maxrow=40), 40, 2),
}


@pytest.mark.parametrize("case", list(CASES))
def test_host_hierarchy_bit_identical_to_oracle(case):
    mk, cm, sweeps = CASES[case]
    rp, c, v = mk()
    h = psc.Hierarchy(rp, c, v, host_only=True, coarse_max=cm, sweeps=sweeps)
    o = oracle.Hierarchy(rp, c, v, coarse_max=cm, sweeps=sweeps)
    inf = h.info()
    assert inf["rows"] == o.sizes()
    assert inf["nnz"] == o.nnzs()
    assert abs(inf["operator_complexity"] - o.operator_complexity()) < 1e-15
    assert inf["coarse_sweeps"] == o.coarse_sweeps
    for l in range(inf["levels"]):
        a, b = h.export_level(l), o.level(l)
        for key in ["rowptr", "col", "val", "minv"]:
            assert np.array_equal(a[key], b[key]), (l, key)
        if l < inf["levels"] - 1:
            assert np.array_equal(a["agg"], b["agg"]) and np.array_equal(a["p"], b["p"]), l


def test_host_only_handle_refuses_solves():
    rp, c, v = P.poisson7(8)
    h = psc.Hierarchy(rp, c, v, host_only=True)
    with pytest.raises(psc.PscError) as e:
        h.pcg(0, 0)
    assert e.value.status == psc.ERR_STATE


def test_malformed_csr_is_rejected():
    rp, c, v = P.poisson7(6)
    bad = c.copy()
    bad[5] = 10 ** 6                                   # column out of range
    with pytest.raises(psc.PscError) as e:
        psc.Hierarchy(rp, bad, v, host_only=True)
    assert e.value.status == psc.ERR_ARG
    rp2 = rp.copy()
    rp2[3] = rp2[4] + 1                                # decreasing row pointer
    with pytest.raises(psc.PscError) as e:
        psc.Hierarchy(rp2, c, v, host_only=True)
    assert e.value.status == psc.ERR_ARG
    v2 = v.copy()
    v2[0] = 0.0                                        # zero diagonal
    with pytest.raises(psc.PscError) as e:
        psc.Hierarchy(rp, c, v2, host_only=True)
    assert e.value.status == psc.ERR_NOT_SPD


def test_stall_above_dense_limit_uses_jacobi_or_fails_without_sweeps():
    rp, c, v = P.diffusion7(48, seed=0)
    h = psc.Hierarchy(rp, c, v, host_only=True, coarse_sweeps=7)
    inf = h.info()
    assert inf["coarse_sweeps"] == 7 and inf["rows"][-1] > 2000
    assert inf["rows"][-1] > 0.9 * inf["rows"][-2]
    with pytest.raises(psc.PscError) as e:
        psc.Hierarchy(rp, c, v, host_only=True, coarse_sweeps=0)
    assert e.value.status == psc.ERR_COARSEN
    with pytest.raises(psc.PscError) as e:
        psc.Hierarchy(rp, c, v, host_only=True, coarse_sweeps=-1)
    assert e.value.status == psc.ERR_ARG


@pytest.mark.parametrize("case", list(SMOOTHED))
def test_smoothed_hierarchy_bit_identical_to_oracle(case):
    mk, cm, sweeps = SMOOTHED[case]
    rp, c, v = mk()
    h = psc.Hierarchy(rp, c, v, host_only=True, coarse_max=cm, sweeps=sweeps, smoothed_prol=True,
                      smoother_sweeps=4)
    o = oracle.Hierarchy(rp, c, v, coarse_max=cm, sweeps=sweeps, prol=1, nu=4)
    inf = h.info()
    assert inf["smoothed_prol"] == 1 and inf["smoother_sweeps"] == 4
    assert inf["rows"] == o.sizes() and inf["nnz"] == o.nnzs()
    for l in range(inf["levels"]):
        a, b = h.export_level(l), o.level(l)
        for key in ["rowptr", "col", "val", "minv"]:
            assert np.array_equal(a[key], b[key]), (l, key)
        if l < inf["levels"] - 1:
            assert np.array_equal(a["agg"], b["agg"]) and np.array_equal(a["p"], b["p"]), l
            prp, pci, pv = h.export_prolongator(l)
            orp, oci, ov, om = o.prolongator(l)
            assert np.array_equal(prp, orp) and np.array_equal(pci, oci) and np.array_equal(pv, ov), l
            assert inf["omega"][l] == om and inf["p_nnz"][l] == len(ov)


VBM = {
    "poisson20_vbm_smoothed": (lambda: P.poisson7(20), 1, 0.01),
    "poisson9_vbm_tentative": (lambda: P.poisson7(9), 0, 0.01),
    "diffusion12_az100_vbm": (lambda: P.diffusion7(12, seed=0, az=100.0), 1, 0.08),
    "random_spd_vbm": (lambda: P.random_spd_csr(400, 3, density=0.02, maxrow=40), 1, 0.05),
}


@pytest.mark.parametrize("case", list(VBM))
def test_vbm_hierarchy_bit_identical_to_oracle(case):
    mk, prol, theta = VBM[case]
    rp, c, v = mk()
    h = psc.Hierarchy(rp, c, v, host_only=True, coarse_max=40, smoothed_prol=bool(prol), smoother_sweeps=4,
                      aggregation=psc.AGGR_VBM, vbm_theta=theta)
    o = oracle.Hierarchy(rp, c, v, coarse_max=40, prol=prol, nu=4, aggr=1, theta=theta)
    inf = h.info()
    assert inf["aggregation"] == psc.AGGR_VBM
    assert inf["rows"] == o.sizes() and inf["nnz"] == o.nnzs()
    for l in range(inf["levels"]):
        a, b = h.export_level(l), o.level(l)
        for key in ["rowptr", "col", "val", "minv"]:
            assert np.array_equal(a[key], b[key]), (l, key)
        if l < inf["levels"] - 1:
            assert np.array_equal(a["agg"], b["agg"]) and np.array_equal(a["p"], b["p"]), l
            prp, pci, pv = h.export_prolongator(l)
            orp, oci, ov, om = o.prolongator(l)
            assert np.array_equal(prp, orp) and np.array_equal(pci, oci) and np.array_equal(pv, ov), l


def test_vmatch_options_reported():
    rp, c, v = P.poisson7(16)
    h = psc.Hierarchy(rp, c, v, host_only=True, sweeps=3, smoother_sweeps=2, vcycle_double=True)
    inf = h.info()
    assert inf["vcycle_double"] == 1 and inf["smoother_sweeps"] == 2
    assert inf["rows"] == oracle.Hierarchy(rp, c, v, sweeps=3, nu=2, nu_double=True).sizes()


def test_tentative_prolongator_export_is_the_aggregate_map():
    rp, c, v = P.poisson7(10)
    h = psc.Hierarchy(rp, c, v, host_only=True)
    L0 = h.export_level(0)
    prp, pci, pv = h.export_prolongator(0)
    assert np.array_equal(prp, np.arange(1001)) and np.array_equal(pci, L0["agg"]) and np.array_equal(pv, L0["p"])
    assert h.info()["omega"][0] == 0.0
    with pytest.raises(psc.PscError):
        psc.Hierarchy(rp, c, v, host_only=True, smoother_sweeps=0)


FAI = {
    # name: (matrix, library options, oracle options)
    "ainv_poisson12": (lambda: P.poisson7(12), dict(smoother=psc.SMOOTH_AINV), dict(smoother=oracle.SMOOTH_AINV)),
    "ainv_tau003_diffusion10": (lambda: P.diffusion7(10, seed=1, az=100.0),
                                dict(smoother=psc.SMOOTH_AINV, ainv_tau=0.03),
                                dict(smoother=oracle.SMOOTH_AINV, ainv_tau=0.03)),
    "invk_poisson12": (lambda: P.poisson7(12), dict(smoother=psc.SMOOTH_INVK), dict(smoother=oracle.SMOOTH_INVK)),
    "invk12_random": (lambda: P.random_spd_csr(400, 4, density=0.01, maxrow=30),
                      dict(smoother=psc.SMOOTH_INVK, invk_fill=1, invk_inv_fill=2, coarse_max=40),
                      dict(smoother=oracle.SMOOTH_INVK, invk_fill=1, invk_inv_fill=2, coarse_max=40)),
    "ainv_smoothed_prol": (lambda: P.poisson7(12), dict(smoother=psc.SMOOTH_AINV, smoothed_prol=True, sweeps=3),
                           dict(smoother=oracle.SMOOTH_AINV, prol=1, sweeps=3)),
}


@pytest.mark.parametrize("case", list(FAI))
def test_fai_factors_bit_identical_to_oracle(case):
    mk, lo, oo = FAI[case]
    rp, c, v = mk()
    h = psc.Hierarchy(rp, c, v, host_only=True, **lo)
    o = oracle.Hierarchy(rp, c, v, **oo)
    inf = h.info()
    assert inf["rows"] == o.sizes() and inf["smoother"] == lo["smoother"]
    assert inf["levels"] >= 2
    for l in range(inf["levels"] - 1):
        zr, zi, zv, d = h.export_smoother(l)
        ozr, ozi, ozv, od = o.fai(l)
        assert np.array_equal(zr, ozr) and np.array_equal(zi, ozi)
        assert np.array_equal(zv, ozv) and np.array_equal(d, od)
        assert inf["smoother_nnz"][l] == len(zi)
    with pytest.raises(psc.PscError):
        h.export_smoother(inf["levels"] - 1)          # the coarsest level has no smoother


def test_fai_options_validated():
    rp, c, v = P.poisson7(6)
    for kw in [dict(smoother=4), dict(smoother=psc.SMOOTH_AINV, ainv_tau=-0.5),
               dict(smoother=psc.SMOOTH_INVK, invk_fill=65), dict(smoother=psc.SMOOTH_INVK, invk_inv_fill=-1)]:
        with pytest.raises(psc.PscError) as e:
            psc.Hierarchy(rp, c, v, host_only=True, **kw)
        assert e.value.status == psc.ERR_ARG
    h = psc.Hierarchy(rp, c, v, host_only=True)
    with pytest.raises(psc.PscError):
        h.export_smoother(0)                          # l1-Jacobi hierarchy: no factors
