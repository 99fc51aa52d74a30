"""Pins of the oracle's polynomial smoother.

The paper names polynomial smoothers as GPU-friendly future work without
fixing one; the smoother taken is the fourth-kind Chebyshev smoother on the
l1-Jacobi preconditioned operator M^-1 A with the bound rho = 1 (A <= M for
the l1 diagonal). Its error propagation after nu steps is the polynomial
W_nu(1 - 2 lambda) / (2 nu + 1) in lambda = M^-1 A, where W_nu is the Chebyshev
polynomial of the fourth kind, W_nu(cos t) = sin((nu + 1/2) t) / sin(t / 2).
The oracle runs the three-term recurrence; these tests hold it to that closed
form through an eigendecomposition, and check its use in the V-cycle.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_2406_19754_amd import problems as P

CHEB4 = oracle.SMOOTH_CHEB4


def dense(rp, c, v):
    n = len(rp) - 1
    return sp.csr_matrix((v, c, rp), shape=(n, n)).toarray()


def l1_diag(A):
    return np.diag(A) + (np.abs(A).sum(axis=1) - np.abs(np.diag(A)))


def w4(nu, t):
    th = np.arccos(np.clip(t, -1.0, 1.0))
    out = np.empty_like(th)
    small = np.abs(th) < 1e-8
    out[~small] = np.sin((nu + 0.5) * th[~small]) / np.sin(th[~small] / 2)
    out[small] = 2 * nu + 1
    return out


def _cases():
    return {"random40": P.random_spd_csr(40, 3, density=0.15), "poisson4": P.poisson7(4),
            "diffusion4": P.diffusion7(4, seed=2, az=100.0)}


@pytest.mark.parametrize("case", ["random40", "poisson4", "diffusion4"])
@pytest.mark.parametrize("nu", [1, 2, 3, 5])
def test_error_propagation_is_the_fourth_kind_polynomial(case, nu):
    rp, c, v = _cases()[case]
    A = dense(rp, c, v)
    n = A.shape[0]
    m = l1_diag(A)
    # G_nu from the smoother applied to the basis vectors: x = G b from x = 0
    G = np.stack([oracle.cheb4_apply(rp, c, v, nu, np.eye(n)[:, j]) for j in range(n)], axis=1)
    E = np.eye(n) - G @ A
    # closed form: M^-1/2 U p(L) U^T M^1/2 with M^-1/2 A M^-1/2 = U L U^T
    s = 1 / np.sqrt(m)
    lam, U = np.linalg.eigh(s[:, None] * A * s[None, :])
    assert lam.max() <= 1 + 1e-12 and lam.min() > 0          # A <= M: rho = 1 is a bound
    p = w4(nu, 1 - 2 * lam) / (2 * nu + 1)
    Ec = (s[:, None] * U) @ np.diag(p) @ (U.T / s[None, :])
    np.testing.assert_allclose(E, Ec, atol=1e-12)
    # |p| < 1 on the spectrum: every eigencomponent is damped
    assert np.abs(p).max() < 1


def test_degree_one_is_l1_jacobi_weighted_four_thirds():
    rp, c, v = P.random_spd_csr(30, 4, density=0.2)
    A = dense(rp, c, v)
    b = np.random.default_rng(0).standard_normal(30)
    x = oracle.cheb4_apply(rp, c, v, 1, b)
    np.testing.assert_allclose(x, (4.0 / 3.0) * b / l1_diag(A), rtol=1e-15)


@pytest.mark.parametrize("nu,double", [(1, False), (3, False), (2, True)])
def test_vcycle_with_polynomial_smoother_two_level_formula(nu, double):
    # eq. (amg) with S = p(M^-1 A) before and after the coarse correction
    rp, c, v = P.poisson7(6)
    h = oracle.Hierarchy(rp, c, v, coarse_max=60, smoother=CHEB4, nu=nu, nu_double=double)
    assert h.nlevels == 2
    L0, L1 = h.level(0), h.level(1)
    A = dense(L0["rowptr"], L0["col"], L0["val"])
    Ac = dense(L1["rowptr"], L1["col"], L1["val"])
    m = 1 / L0["minv"]
    s = 1 / np.sqrt(m)
    lam, U = np.linalg.eigh(s[:, None] * A * s[None, :])
    S = (s[:, None] * U) @ np.diag(w4(nu, 1 - 2 * lam) / (2 * nu + 1)) @ (U.T / s[None, :])
    prp, pci, pv, _ = h.prolongator(0)
    Pm = sp.csr_matrix((pv, pci, prp), shape=(L0["n"], L0["nc"])).toarray()
    I = np.eye(L0["n"])
    E = S @ (I - Pm @ np.linalg.inv(Ac) @ Pm.T @ A) @ S
    B = (I - E) @ np.linalg.inv(A)
    V = np.stack([h.vcycle(np.eye(L0["n"])[:, j]) for j in range(0, L0["n"], 5)], axis=1)
    np.testing.assert_allclose(V, B[:, ::5], rtol=0, atol=1e-12)
    np.testing.assert_allclose(B, B.T, atol=1e-12)
    assert np.linalg.eigvalsh((B + B.T) / 2).min() > 0


def test_polynomial_smoother_in_pcg():
    rp, c, v = P.poisson7(16)
    b = np.random.default_rng(1).standard_normal(len(rp) - 1)
    its = {}
    for name, kw in [("l1_nu2", dict(nu=2)), ("cheb_nu2", dict(nu=2, smoother=CHEB4)),
                     ("l1_nu1", {}), ("cheb_nu1", dict(smoother=CHEB4))]:
        r = oracle.Hierarchy(rp, c, v, **kw).pcg(b)
        assert r["status"] == oracle.OK and r["relres"] < 1e-6
        its[name] = r["iters"]
    # the polynomial of the same degree damps more than repeated l1-Jacobi sweeps
    assert its["cheb_nu2"] < its["l1_nu2"] and its["cheb_nu1"] < its["l1_nu1"]
    h = oracle.Hierarchy(rp, c, v, smoother=CHEB4, nu=3)
    r = np.random.default_rng(2).standard_normal(len(b))
    z64, z32 = h.vcycle(r), h.vcycle32(r)
    assert np.linalg.norm(z32 - z64) < 1e-5 * np.linalg.norm(z64)
