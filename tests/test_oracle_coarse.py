"""Pins of the oracle's inexact coarsest solver: at most k iterations of CG
preconditioned by l1-Jacobi from x = 0, stopped at ||r|| <= rtol ||b|| (the
paper's coarsest solver in its tests caps CG at 40 iterations). Checked on a
one-level hierarchy, where the V-cycle is that solve, against SciPy's
independent preconditioned CG (same stopping rule), against the exact
solution when the cap exceeds the size, and inside FCG on a multilevel
hierarchy."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as sla

import oracle
from paper_2406_19754_amd import problems as P


def _l1(A):
    A = A.toarray()
    return 1.0 / (np.diag(A) + np.abs(A).sum(axis=1) - np.abs(np.diag(A)))


@pytest.mark.parametrize("case", ["random60", "poisson5", "diffusion5"])
@pytest.mark.parametrize("k,rtol", [(3, 0.0), (10, 0.0), (40, 1e-4), (40, 1e-9)])
def test_coarse_pcg_matches_scipy_cg(case, k, rtol):
    rp, c, v = {"random60": lambda: P.random_spd_csr(60, 7, density=0.1), "poisson5": lambda: P.poisson7(5),
                "diffusion5": lambda: P.diffusion7(5, seed=4, az=50.0)}[case]()
    n = len(rp) - 1
    h = oracle.Hierarchy(rp, c, v, coarse_max=n, coarse_pcg=k, coarse_rtol=rtol)
    assert h.nlevels == 1
    A = sp.csr_matrix((v, c, rp), shape=(n, n))
    m = _l1(A)
    b = np.random.default_rng(3).standard_normal(n)
    x = h.vcycle(b)
    its = [0]
    ref, info = sla.cg(A, b, x0=np.zeros(n), rtol=rtol, atol=0.0, maxiter=k,
                       M=sla.LinearOperator((n, n), matvec=lambda t: m * t),
                       callback=lambda _: its.__setitem__(0, its[0] + 1))
    np.testing.assert_allclose(x, ref, rtol=0, atol=1e-10 * np.linalg.norm(ref))
    if rtol > 0 and info == 0:
        assert np.linalg.norm(b - A @ x) <= rtol * np.linalg.norm(b)


def test_coarse_pcg_with_cap_above_size_is_exact():
    rp, c, v = P.random_spd_csr(30, 2, density=0.2)
    n = 30
    h = oracle.Hierarchy(rp, c, v, coarse_max=n, coarse_pcg=200, coarse_rtol=0.0)
    A = sp.csr_matrix((v, c, rp), shape=(n, n)).toarray()
    b = np.random.default_rng(1).standard_normal(n)
    np.testing.assert_allclose(h.vcycle(b), np.linalg.solve(A, b), rtol=1e-8, atol=1e-10)


def test_inexact_coarsest_inside_fcg():
    rp, c, v = P.poisson7(20)
    b = np.random.default_rng(2).standard_normal(len(rp) - 1)
    exact = oracle.Hierarchy(rp, c, v, sweeps=3, coarse_max=200)
    inexact = oracle.Hierarchy(rp, c, v, sweeps=3, coarse_max=200, coarse_pcg=40, coarse_rtol=1e-4)
    assert exact.sizes() == inexact.sizes() and inexact.coarse_sweeps == 0
    re, ri = exact.fcg(b), inexact.fcg(b)
    assert re["status"] == ri["status"] == oracle.OK
    assert ri["relres"] <= 1e-6 and abs(ri["iters"] - re["iters"]) <= 2
    # a single PCG iteration on the coarsest level still converges, more slowly
    crude = oracle.Hierarchy(rp, c, v, sweeps=3, coarse_max=200, coarse_pcg=1, coarse_rtol=0.0)
    rc = crude.fcg(b)
    assert rc["status"] == oracle.OK and rc["iters"] > re["iters"]
