"""Pins for the seeded problem generators (closed forms of the 7-point operator)."""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_2406_19754_amd import problems as P


def dense(rp, c, v):
    n = len(rp) - 1
    return sp.csr_matrix((v, c, rp), shape=(n, n)).toarray()


@pytest.mark.parametrize("n", [1, 2, 3, 7, 16])
def test_poisson_nnz_and_sorted(n):
    rp, c, v = P.poisson7(n)
    assert rp[-1] == P.poisson_nnz(n) == 7 * n ** 3 - 6 * n ** 2
    for i in range(n ** 3):
        row = c[rp[i]:rp[i + 1]]
        assert np.all(np.diff(row) > 0)
        assert i in row


@pytest.mark.parametrize("n", [4, 5, 6])
def test_poisson_closed_form_eigenvalues(n):
    rp, c, v = P.poisson7(n)
    lam = np.linalg.eigvalsh(dense(rp, c, v))
    t = 2.0 - 2.0 * np.cos(np.arange(1, n + 1) * np.pi / (n + 1))
    ref = np.sort((t[:, None, None] + t[None, :, None] + t[None, None, :]).ravel())
    np.testing.assert_allclose(lam, ref, rtol=0, atol=1e-12)


def test_poisson_sine_eigenvectors_n32():
    n = 32
    rp, c, v = P.poisson7(n)
    A = sp.csr_matrix((v, c, rp), shape=(n ** 3, n ** 3))
    g = np.arange(1, n + 1)
    for (p, q, r) in [(1, 1, 1), (3, 7, 2), (32, 1, 17)]:
        sx = np.sin(p * g * np.pi / (n + 1))
        sy = np.sin(q * g * np.pi / (n + 1))
        sz = np.sin(r * g * np.pi / (n + 1))
        vec = (sz[:, None, None] * sy[None, :, None] * sx[None, None, :]).ravel()
        lam = 6 - 2 * np.cos(p * np.pi / (n + 1)) - 2 * np.cos(q * np.pi / (n + 1)) - 2 * np.cos(r * np.pi / (n + 1))
        np.testing.assert_allclose(A @ vec, lam * vec, rtol=0, atol=1e-12)


def test_diffusion_unit_k_is_poisson_bitwise():
    n = 9
    rp, c, v = P.poisson7(n)
    rp2, c2, v2 = P.diffusion7(n, k=np.ones(n ** 3))
    assert np.array_equal(rp, rp2) and np.array_equal(c, c2)
    assert np.array_equal(v, v2)


def test_diffusion_bitwise_symmetric_and_lognormal():
    n = 20
    rp, c, v = P.diffusion7(n, seed=3, sigma=1.5, az=100.0)
    A = sp.csr_matrix((v, c, rp), shape=(n ** 3, n ** 3))
    assert (A != A.T).nnz == 0
    # diagonal = sum |offdiag| + boundary faces > 0; off-diagonals negative
    d = A.diagonal()
    off = A - sp.diags(d)
    assert off.max() <= 0.0
    rowsum = np.asarray(abs(off).sum(axis=1)).ravel()
    assert np.all(d >= rowsum * (1 - 1e-15))
    g = np.random.default_rng(3).standard_normal(n ** 3)
    k = np.exp(1.5 * g)
    assert abs(np.log(k).mean()) < 0.05 and abs(np.log(k).std() - 1.5) < 0.05


@pytest.mark.parametrize("az", [100.0, 0.01])
def test_anisotropic_unit_k_closed_form(az):
    n = 5
    rp, c, v = P.diffusion7(n, k=np.ones(n ** 3), az=az)
    lam = np.linalg.eigvalsh(dense(rp, c, v))
    t = 2.0 - 2.0 * np.cos(np.arange(1, n + 1) * np.pi / (n + 1))
    ref = np.sort((az * t[:, None, None] + t[None, :, None] + t[None, None, :]).ravel())
    np.testing.assert_allclose(lam, ref, rtol=1e-12, atol=1e-12)


def test_rhs_generators_seeded():
    assert np.array_equal(P.x_true(100, 5), P.x_true(100, 5))
    u = P.rhs_uniform(10000, 1)
    assert u.min() >= -1 and u.max() < 1
    b = P.rhs_bumps(16, 101)
    assert b.shape == (16 ** 3,) and np.all(np.isfinite(b))
    w = P.net_init(0)
    assert w.dtype == np.float32 and w.size == P.net_param_count() == 7809
