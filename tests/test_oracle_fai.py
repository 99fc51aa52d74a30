"""Pins of the oracle's factored approximate inverse smoothers (AINV, INVK).

Section "GPU enabled smoothers" of the paper: both smoothers approximate
A_l^-1 by sparse triangular factors, G = Z D^-1 Z^T, applied through sparse
products only. The pins below fix the oracle against what the mathematics
fixes: exact inverses when nothing is dropped, the identity when everything
is dropped, the defining property of an incomplete factorisation on its
pattern, an independent symbolic level-of-fill computation, the truncated
triangular solve on its pattern, an independent dense right-looking form of
the biconjugation, and the V-cycle error propagation with the smoother.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_2406_19754_amd import problems as P

AINV, INVK = oracle.SMOOTH_AINV, oracle.SMOOTH_INVK


def dense(rp, c, v):
    n = len(rp) - 1
    return sp.csr_matrix((v, c, rp), shape=(n, n)).toarray()


def zmat(f):
    zr, zi, zv, d = f
    n = len(zr) - 1
    return sp.csc_matrix((zv, zi, zr), shape=(n, n)).toarray(), d


def _cases():
    return {
        "random40": P.random_spd_csr(40, 3, density=0.15),
        "random64": P.random_spd_csr(64, 11, density=0.08),
        "poisson4": P.poisson7(4),
        "diffusion4": P.diffusion7(4, seed=2, az=100.0),
    }


@pytest.mark.parametrize("case", ["random40", "random64", "poisson4", "diffusion4"])
def test_ainv_without_dropping_is_the_exact_inverse(case):
    rp, c, v = _cases()[case]
    A = dense(rp, c, v)
    Z, d = zmat(oracle.fai_factor(rp, c, v, AINV, tau=0.0))
    n = len(d)
    assert np.all(np.tril(Z, -1) == 0) and np.all(np.diag(Z) == 1.0)
    assert np.all(d > 0)
    # complete A-biconjugation: Z^T A Z = D, so A^-1 = Z D^-1 Z^T
    np.testing.assert_allclose(Z.T @ A @ Z, np.diag(d), atol=1e-11 * np.abs(A).max())
    np.testing.assert_allclose((Z / d) @ Z.T @ A, np.eye(n), atol=1e-10)


@pytest.mark.parametrize("case", ["random40", "poisson4"])
def test_invk_with_full_fill_is_the_exact_inverse(case):
    rp, c, v = _cases()[case]
    A = dense(rp, c, v)
    n = A.shape[0]
    Z, d = zmat(oracle.fai_factor(rp, c, v, INVK, fill1=n, fill2=n))
    assert np.all(np.tril(Z, -1) == 0) and np.all(np.diag(Z) == 1.0)
    np.testing.assert_allclose((Z / d) @ Z.T @ A, np.eye(n), atol=1e-10)
    # the complete factor is the LDL^T factor of the Cholesky decomposition
    Lc = np.linalg.cholesky(A)
    np.testing.assert_allclose(d, np.diag(Lc) ** 2, rtol=1e-12)


@pytest.mark.parametrize("kind", [AINV, INVK])
def test_everything_dropped_gives_jacobi(kind):
    # AINV with a tolerance above every entry, INVK(0) with no inverse fill
    # on a diagonal matrix: Z = I and D = diag(A) (plain Jacobi)
    rp, c, v = P.random_spd_csr(30, 5, density=0.2)
    A = dense(rp, c, v)
    if kind == AINV:
        Z, d = zmat(oracle.fai_factor(rp, c, v, AINV, tau=1e30))
        np.testing.assert_array_equal(Z, np.eye(30))
        np.testing.assert_array_equal(d, np.diag(A))
    else:
        D = sp.diags(np.diag(A)).tocsr()
        Z, d = zmat(oracle.fai_factor(D.indptr, D.indices, D.data, INVK, fill1=0, fill2=0))
        np.testing.assert_array_equal(Z, np.eye(30))
        np.testing.assert_array_equal(d, np.diag(A))


def _levels_symbolic(A, k):
    """Independent symbolic IC(k) by the textbook level rule on a dense level
    table: lev_ij = 0 on the pattern of A, fill through pivot m gets
    lev_im + lev_mj + 1, kept when <= k (lower triangle)."""
    n = A.shape[0]
    INF = 10 ** 9
    lev = np.where(A != 0, 0, INF)
    for i in range(n):
        for m in range(i):
            if lev[i, m] > k:
                continue
            for j in range(m + 1, i + 1):
                if lev[j, m] <= k:
                    lev[i, j] = min(lev[i, j], lev[i, m] + lev[j, m] + 1)
            # symmetric pattern: row i, column j of the upper factor is (j, m)
    return np.tril(lev <= k, -1)


@pytest.mark.parametrize("case,k1", [("poisson4", 0), ("poisson4", 1), ("random40", 1), ("diffusion4", 2)])
def test_incomplete_factor_pattern_and_exactness_on_pattern(case, k1):
    rp, c, v = _cases()[case]
    A = dense(rp, c, v)
    n = A.shape[0]
    # with a complete inverse (fill2 = n), Z = L^-T for the incomplete factor L
    Z, d = zmat(oracle.fai_factor(rp, c, v, INVK, fill1=k1, fill2=n))
    L = np.linalg.inv(Z).T
    np.testing.assert_allclose(np.diag(L), 1.0, atol=1e-12)
    L[np.abs(L) < 1e-13] = 0.0
    pat = _levels_symbolic(A, k1)
    # the factor's strictly lower pattern is the symbolic level-k1 pattern
    assert np.array_equal(np.tril(L, -1) != 0, pat)
    # an incomplete factorisation reproduces A on its own pattern (and the diagonal)
    R = L @ np.diag(d) @ L.T - A
    on = pat | pat.T | np.eye(n, dtype=bool)
    assert np.abs(R[on]).max() < 1e-11 * np.abs(A).max()
    if k1 == 0 and case == "poisson4":
        # IC(0) of a 7-point stencil drops fill, so it is not exact off the pattern
        assert np.abs(R[~on]).max() > 1e-3


@pytest.mark.parametrize("k1,k2", [(0, 0), (0, 1), (1, 1), (0, 2)])
def test_invk_inverse_is_a_truncated_triangular_solve(k1, k2):
    rp, c, v = P.poisson7(4)
    A = dense(rp, c, v)
    n = A.shape[0]
    Zfull, _ = zmat(oracle.fai_factor(rp, c, v, INVK, fill1=k1, fill2=n))
    L = np.linalg.inv(Zfull).T
    L[np.abs(L) < 1e-13] = 0.0
    Z, _ = zmat(oracle.fai_factor(rp, c, v, INVK, fill1=k1, fill2=k2))
    pz = Z != 0
    # pattern: entries reachable from the diagonal by at most k2 + 1 steps
    # along the strictly upper pattern of L^T
    U = (np.triu(L.T, 1) != 0).astype(int)
    reach = np.eye(n, dtype=int)
    tot = np.eye(n, dtype=bool)
    for _ in range(k2 + 1):
        reach = (U @ reach > 0).astype(int)
        tot |= reach > 0
    assert np.array_equal(pz, tot)
    # on that pattern the solve L^T z = e_k holds exactly
    R = L.T @ Z - np.eye(n)
    assert np.abs(R[pz]).max() < 1e-12


def _ainv_dense_right_looking(A, tau):
    """Independent dense form: for i = 0..n-1, v = A z_i, d_i = v.z_i, and
    for j > i with p = v.z_j != 0: z_j -= (p/d_i) z_i, then drop entries
    r != j with |z_rj| sqrt(a_rr/a_jj) < tau."""
    n = A.shape[0]
    Z = np.eye(n)
    d = np.zeros(n)
    dg = np.diag(A)
    for i in range(n):
        vv = A @ Z[:, i]
        d[i] = vv @ Z[:, i]
        for j in range(i + 1, n):
            p = vv @ Z[:, j]
            if p != 0.0:
                Z[:, j] -= (p / d[i]) * Z[:, i]
                small = np.abs(Z[:, j]) * np.sqrt(dg / dg[j]) < tau
                small[j] = False
                Z[small, j] = 0.0
    return Z, d


@pytest.mark.parametrize("case,tau", [("random40", 0.05), ("random64", 0.1), ("poisson4", 0.1),
                                      ("poisson4", 0.02), ("diffusion4", 0.1)])
def test_ainv_matches_dense_right_looking_biconjugation(case, tau):
    rp, c, v = _cases()[case]
    A = dense(rp, c, v)
    Zr, dr = _ainv_dense_right_looking(A, tau)
    Z, d = zmat(oracle.fai_factor(rp, c, v, AINV, tau=tau))
    assert np.array_equal(Z != 0, Zr != 0)
    np.testing.assert_allclose(Z, Zr, atol=1e-12)
    np.testing.assert_allclose(d, dr, rtol=1e-12)
    assert (Z != 0).sum() < 0.5 * n_upper(A.shape[0])


def n_upper(n):
    return n * (n + 1) // 2


def test_ainv_drop_tolerance_is_scale_invariant():
    # dropping acts on the matrix scaled to unit diagonal: a symmetric
    # diagonal scaling S A S gives the factor S^-1 Z S and pivots S^2 D
    rp, c, v = P.random_spd_csr(40, 3, density=0.15)
    A = dense(rp, c, v)
    s = 2.0 ** np.random.default_rng(0).integers(-3, 4, size=40)   # exact scalings
    As = sp.csr_matrix(s[:, None] * A * s[None, :])
    Z, d = zmat(oracle.fai_factor(rp, c, v, AINV, tau=0.1))
    Zs, ds = zmat(oracle.fai_factor(As.indptr, As.indices, As.data, AINV, tau=0.1))
    np.testing.assert_allclose(Zs, Z * (1 / s)[:, None] * s[None, :], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(ds, d * s * s, rtol=1e-12)


@pytest.mark.parametrize("smoother,nu", [(AINV, 1), (AINV, 2), (INVK, 1)])
def test_vcycle_with_fai_smoother_two_level_formula(smoother, nu):
    # eq. (amg) with the smoother G = Z D^-1 Z^T in place of M^-1:
    # B = (I - E) A^-1, E = S^nu (I - P A_c^-1 P^T A) S^nu, S = I - G A
    rp, c, v = P.poisson7(6)
    h = oracle.Hierarchy(rp, c, v, coarse_max=60, smoother=smoother, nu=nu)
    assert h.nlevels == 2
    L0, L1 = h.level(0), h.level(1)
    A = dense(L0["rowptr"], L0["col"], L0["val"])
    Ac = dense(L1["rowptr"], L1["col"], L1["val"])
    Z, d = zmat(h.fai(0))
    assert h.fai(1) is None
    G = (Z / d) @ Z.T
    prp, pci, pv, _ = h.prolongator(0)
    Pm = sp.csr_matrix((pv, pci, prp), shape=(L0["n"], L0["nc"])).toarray()
    I = np.eye(L0["n"])
    S = np.linalg.matrix_power(I - G @ A, nu)
    E = S @ (I - Pm @ np.linalg.inv(Ac) @ Pm.T @ A) @ S
    B = (I - E) @ np.linalg.inv(A)
    V = np.stack([h.vcycle(np.eye(L0["n"])[:, j]) for j in range(0, L0["n"], 5)], axis=1)
    np.testing.assert_allclose(V, B[:, ::5], rtol=0, atol=1e-12)
    # symmetric: the V-cycle is a valid CG preconditioner
    np.testing.assert_allclose(B, B.T, atol=1e-12)


@pytest.mark.parametrize("smoother", [AINV, INVK])
def test_fai_smoothers_take_fewer_pcg_iterations(smoother):
    rp, c, v = P.poisson7(16)
    b = np.random.default_rng(1).standard_normal(len(rp) - 1)
    base = oracle.Hierarchy(rp, c, v)
    h = oracle.Hierarchy(rp, c, v, smoother=smoother)
    o0, o1 = base.pcg(b), h.pcg(b)
    assert o0["status"] == 0 and o1["status"] == 0
    assert o0["relres"] < 1e-6 and o1["relres"] < 1e-6
    assert o1["iters"] <= 0.75 * o0["iters"]
    # the FP32 V-cycle with the same smoother stays close to the FP64 one
    r = np.random.default_rng(2).standard_normal(len(b))
    z64, z32 = h.vcycle(r), h.vcycle32(r)
    assert np.linalg.norm(z32 - z64) < 1e-5 * np.linalg.norm(z64)


def test_fai_options_rejected():
    rp, c, v = P.poisson7(4)
    for kw in [dict(smoother=4), dict(smoother=AINV, ainv_tau=-1.0), dict(smoother=INVK, invk_fill=-1)]:
        with pytest.raises(RuntimeError):
            oracle.Hierarchy(rp, c, v, **kw)
