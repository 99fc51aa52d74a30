"""Pins for the CPU oracle's AMG hierarchy, V-cycle and Krylov loops.

Each check ties the oracle to something other than itself: closed forms of
the 7-point operator, dense linear algebra (numpy), brute-force matchings,
scipy's CG, the V-cycle's error-propagation formula (eq. amg) and an
operator complexity printed in the paper.
"""
import itertools
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from paper_2406_19754_amd import problems as P

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dense(rp, c, v):
    n = len(rp) - 1
    return sp.csr_matrix((v, c, rp), shape=(n, n)).toarray()


def prolongator(lev):
    n, nc = lev["n"], lev["nc"]
    return sp.csr_matrix((lev["p"], (np.arange(n), lev["agg"])), shape=(n, nc)).toarray()


# --------------------------------------------------------------------------
# SpMV
# --------------------------------------------------------------------------

def test_spmv_matches_dense_product():
    rp, c, v = P.poisson7(6)
    x = np.random.default_rng(0).standard_normal(216)
    np.testing.assert_allclose(oracle.spmv(rp, c, v, x), dense(rp, c, v) @ x, rtol=0, atol=1e-13)
    rp, c, v = P.random_spd_csr(150, 1, density=0.03, maxrow=60)
    x = np.random.default_rng(1).standard_normal(150)
    np.testing.assert_allclose(oracle.spmv(rp, c, v, x), dense(rp, c, v) @ x, rtol=1e-14, atol=1e-13)


# --------------------------------------------------------------------------
# Matching
# --------------------------------------------------------------------------

def _edges(rp, c, S):
    n = len(rp) - 1
    d = np.zeros(n)
    for i in range(n):
        for k in range(rp[i], rp[i + 1]):
            if c[k] == i:
                d[i] = S[k]
    E = {}
    for i in range(n):
        for k in range(rp[i], rp[i + 1]):
            j = c[k]
            j = int(j)
            if j > i:
                cij = 1.0 - 2.0 * S[k] / (d[i] + d[j])
                q = int(round(cij * 2 ** 30))  # values here are never exact halves
                if q > 0:
                    E[(i, j)] = q
    return E


def _brute_max_weight(n, E):
    adj = {i: [] for i in range(n)}
    for (i, j), q in E.items():
        adj[int(i)].append((int(j), q))
        adj[int(j)].append((int(i), q))
    memo = {}

    def f(mask):
        if mask == 0:
            return 0
        if mask in memo:
            return memo[mask]
        i = (mask & -mask).bit_length() - 1
        best = f(mask & ~(1 << i))
        for j, q in adj[i]:
            if mask >> j & 1:
                best = max(best, q + f(mask & ~(1 << i) & ~(1 << j)))
        memo[mask] = best
        return best

    return f((1 << n) - 1)


def _locally_dominant(n, E):
    """Independent matching: repeatedly match mutually-heaviest free pairs."""
    key = {e: (-q, e[0], e[1]) for e, q in E.items()}
    mate = [-1] * n
    nbrs = {i: [] for i in range(n)}
    for (i, j) in E:
        nbrs[i].append(j)
        nbrs[j].append(i)
    changed = True
    while changed:
        changed = False
        cand = [-1] * n
        for i in range(n):
            if mate[i] >= 0:
                continue
            best = None
            for j in nbrs[i]:
                if mate[j] >= 0:
                    continue
                e = (min(i, j), max(i, j))
                if best is None or key[e] < key[best]:
                    best = e
            if best is not None:
                cand[i] = best[0] if best[1] == i else best[1]
        for i in range(n):
            j = cand[i]
            if j > i and cand[j] == i:
                mate[i], mate[j] = j, i
                changed = True
    return np.array(mate)


def _random_graph(n, seed, levels=None):
    rng = np.random.default_rng(seed)
    A = np.zeros((n, n))
    for i in range(n):
        for j in range(i + 1, n):
            if rng.random() < 0.45:
                val = -rng.integers(1, levels + 1) if levels else -rng.uniform(0.05, 2.0)
                A[i, j] = A[j, i] = val
    A[np.arange(n), np.arange(n)] = np.abs(A).sum(1) + (rng.integers(1, 4, n) if levels else rng.uniform(0.1, 2, n))
    rp = np.zeros(n + 1, np.int32)
    cols, vals = [], []
    for i in range(n):
        nz = np.nonzero(A[i])[0]
        cols += list(nz)
        vals += list(A[i, nz])
        rp[i + 1] = len(cols)
    return rp, np.array(cols, np.int32), np.array(vals)


@pytest.mark.parametrize("seed", range(12))
def test_matching_half_approx_and_locally_dominant(seed):
    n = 6 + seed % 7                     # 6..12 vertices
    rp, c, S = _random_graph(n, seed, levels=2 if seed % 2 else None)  # even seeds: ties
    mate = oracle.match(rp, c, S)
    E = _edges(rp, c, S)
    # a valid matching on eligible edges
    for i in range(n):
        if mate[i] >= 0:
            assert mate[mate[i]] == i and (min(i, mate[i]), max(i, mate[i])) in E
    # maximal: no eligible edge with both ends free
    for (i, j) in E:
        assert mate[i] >= 0 or mate[j] >= 0
    w = sum(q for (i, j), q in E.items() if mate[i] == j)
    assert 2 * w >= _brute_max_weight(n, E)
    assert np.array_equal(mate, _locally_dominant(n, E))


def test_matching_ignores_nonpositive_weights():
    # a_01 = +4 with a_00 = a_11 = 4 -> c = 1 - 2*4/8 = 0 -> not eligible
    rp = np.array([0, 2, 4], np.int32)
    c = np.array([0, 1, 0, 1], np.int32)
    S = np.array([4.0, 4.0, 4.0, 4.0])
    assert list(oracle.match(rp, c, S)) == [-1, -1]
    S = np.array([4.0, -1.0, -1.0, 4.0])
    assert list(oracle.match(rp, c, S)) == [1, 0]
    assert oracle.edge_key(-1.0, 6.0, 6.0) == round(7.0 / 6.0 * 2 ** 30)


def test_poisson_first_sweep_is_x_pairs():
    n = 8
    rp, c, v = P.poisson7(n)
    mate = oracle.match(rp, c, v)
    assert np.array_equal(mate, np.arange(n ** 3) ^ 1)


@pytest.mark.parametrize("n", [8, 16])
def test_poisson_aggregates_are_2x2x1_blocks(n):
    rp, c, v = P.poisson7(n)
    h = oracle.Hierarchy(rp, c, v)
    agg = h.level(0)["agg"]
    idx = np.arange(n ** 3)
    i, j, k = idx % n, (idx // n) % n, idx // (n * n)
    m = n // 2
    assert np.array_equal(agg, (i // 2) + m * ((j // 2) + m * k))


# --------------------------------------------------------------------------
# Hierarchy
# --------------------------------------------------------------------------

def test_poisson_level1_closed_form():
    n = 8
    rp, c, v = P.poisson7(n)
    h = oracle.Hierarchy(rp, c, v)
    L1 = h.level(1)
    A1 = dense(L1["rowptr"], L1["col"], L1["val"])
    m = n // 2
    N1 = m * m * n
    ref = np.zeros((N1, N1))
    for I in range(N1):
        a, b, k = I % m, (I // m) % m, I // (m * m)
        ref[I, I] = 4.0
        if a > 0: ref[I, I - 1] = -0.5
        if a < m - 1: ref[I, I + 1] = -0.5
        if b > 0: ref[I, I - m] = -0.5
        if b < m - 1: ref[I, I + m] = -0.5
        if k > 0: ref[I, I - m * m] = -1.0
        if k < n - 1: ref[I, I + m * m] = -1.0
    np.testing.assert_allclose(A1, ref, rtol=0, atol=1e-15)
    # the closed form reaches every nonzero and no more
    assert L1["nnz"] == np.count_nonzero(ref)


@pytest.mark.parametrize("n,sizes", [(32, [32768, 8192, 2048, 512, 128]),
                                     (64, [262144, 65536, 16384, 4096, 1024, 256, 64])])
def test_poisson_level_sizes_and_complexity(n, sizes):
    rp, c, v = P.poisson7(n)
    h = oracle.Hierarchy(rp, c, v)
    assert h.sizes() == sizes
    # tentative aggregates of 4: complexity -> 4/3 from below
    oc = h.operator_complexity()
    assert 1.30 < oc < 4.0 / 3.0


def _check_invariants(h, tol=1e-13):
    for l in range(h.nlevels - 1):
        L = h.level(l)
        C = h.level(l + 1)
        agg = L["agg"]
        n, nc = L["n"], L["nc"]
        assert nc == C["n"]
        assert agg.min() == 0 and agg.max() == nc - 1          # every aggregate non-empty
        counts = np.bincount(agg, minlength=nc)
        assert counts.max() <= 4 and counts.min() >= 1         # each row in one aggregate, size <= 4
        # numbering by ascending smallest member
        first = np.full(nc, n)
        np.minimum.at(first, agg, np.arange(n))
        assert np.all(np.diff(first) > 0)
        Pm = prolongator(L)
        np.testing.assert_allclose(Pm.T @ Pm, np.eye(nc), rtol=0, atol=tol)
        w = L["w"]
        np.testing.assert_allclose(Pm @ (Pm.T @ w), w, rtol=0, atol=tol * np.abs(w).max())
        np.testing.assert_allclose(C["w"], Pm.T @ w, rtol=1e-14, atol=0)
        A = dense(L["rowptr"], L["col"], L["val"])
        Ac = dense(C["rowptr"], C["col"], C["val"])
        scale = np.abs(A).max()
        np.testing.assert_allclose(Ac, Pm.T @ A @ Pm, rtol=0, atol=tol * scale)
        assert np.abs(Ac - Ac.T).max() <= 1e-14 * np.abs(Ac).max()
        vc = np.random.default_rng(l).standard_normal(nc)
        e1 = vc @ Ac @ vc
        e2 = (Pm @ vc) @ A @ (Pm @ vc)
        assert abs(e1 - e2) <= 1e-12 * abs(e2)
        if nc <= 1500:
            assert np.linalg.eigvalsh(Ac).min() > 0


@pytest.mark.parametrize("case", ["poisson12", "poisson9odd", "diffusion10", "random"])
def test_hierarchy_invariants(case):
    if case == "poisson12":
        rp, c, v = P.poisson7(12)
    elif case == "poisson9odd":
        rp, c, v = P.poisson7(9)
    elif case == "diffusion10":
        rp, c, v = P.diffusion7(10, seed=1, az=100.0)
    else:
        rp, c, v = P.random_spd_csr(400, 7, density=0.02, maxrow=40)
    h = oracle.Hierarchy(rp, c, v, coarse_max=40)
    assert h.nlevels >= 2
    _check_invariants(h)


def test_coarse_cholesky_factor():
    rp, c, v = P.poisson7(8)
    h = oracle.Hierarchy(rp, c, v)
    Lc = h.level(h.nlevels - 1)
    A = dense(Lc["rowptr"], Lc["col"], Lc["val"])
    Lf = h.coarse_factor()
    assert np.allclose(np.triu(Lf, 1), 0)
    np.testing.assert_allclose(Lf @ Lf.T, A, rtol=0, atol=1e-13)


def test_l1_jacobi_closed_form_and_convergence():
    n = 6
    rp, c, v = P.poisson7(n)
    h = oracle.Hierarchy(rp, c, v, coarse_max=20)
    L0 = h.level(0)
    idx = np.arange(n ** 3)
    i, j, k = idx % n, (idx // n) % n, idx // (n * n)
    nb = sum(((a > 0).astype(int) + (a < n - 1).astype(int)) for a in (i, j, k))
    np.testing.assert_allclose(L0["minv"], 1.0 / (6.0 + nb), rtol=0, atol=1e-16)
    assert set(np.unique(1.0 / L0["minv"])) == {9.0, 10.0, 11.0, 12.0}
    for l in range(h.nlevels):
        L = h.level(l)
        A = dense(L["rowptr"], L["col"], L["val"])
        d = np.sqrt(L["minv"])
        ev = np.linalg.eigvalsh(d[:, None] * A * d[None, :])   # spectrum of M^-1 A
        assert ev.min() > 0 and ev.max() <= 1.0 + 1e-14


# --------------------------------------------------------------------------
# V-cycle
# --------------------------------------------------------------------------

def test_vcycle_two_level_matches_error_propagation_formula():
    n = 8
    rp, c, v = P.poisson7(n)
    h = oracle.Hierarchy(rp, c, v)
    assert h.sizes() == [512, 128]
    L0, L1 = h.level(0), h.level(1)
    A = dense(rp, c, v)
    Ac = dense(L1["rowptr"], L1["col"], L1["val"])
    Pm = prolongator(L0)
    Mi = np.diag(L0["minv"])
    I = np.eye(512)
    E = (I - Mi @ A) @ (I - Pm @ np.linalg.solve(Ac, Pm.T @ A)) @ (I - Mi @ A)
    Bref = (I - E) @ np.linalg.inv(A)
    B = np.stack([h.vcycle(I[:, j]) for j in range(512)], axis=1)
    np.testing.assert_allclose(B, Bref, rtol=0, atol=1e-12)
    assert np.abs(B - B.T).max() < 1e-13
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0


def _stall_matrix(n, chain, seed):
    """SPD matrix that is diagonal except for a 1-D chain on its first rows,
    so one coarsening step removes at most 3/4 of the chain rows and stalls."""
    rng = np.random.default_rng(seed)
    d = 2.5 + rng.random(n)
    off = np.zeros(n - 1)
    off[:chain - 1] = -(0.2 + 0.8 * rng.random(chain - 1))
    A = sp.diags(d) + sp.diags(off, 1, shape=(n, n)) + sp.diags(off, -1, shape=(n, n))
    A = sp.csr_matrix(A)
    A.eliminate_zeros()
    A = sp.csr_matrix(A)
    A.sort_indices()
    return A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.copy()


@pytest.mark.parametrize("K", [1, 5, 30])
def test_stalled_coarsest_jacobi_matches_spectral_closed_form(K):
    # Coarsening stalls (about 2060 rows after 2200) above the dense-factor limit, so
    # the coarsest level is solved by K l1-Jacobi sweeps from zero. With
    # S = M^-1/2 A_c M^-1/2 = U diag(lam) U^T, K sweeps apply
    # B_c = M^-1/2 U diag((1 - (1 - lam)^K) / lam) U^T M^-1/2 (Richardson
    # polynomial); the two-level V-cycle is then (I - E) A^-1 with E of eq. (amg).
    rp, c, v = _stall_matrix(2200, 200, seed=3)
    h = oracle.Hierarchy(rp, c, v, coarse_sweeps=K)
    s = h.sizes()
    assert len(s) == 2 and 2000 < s[1] and s[1] > 0.9 * s[0] and h.coarse_sweeps == K
    L0, L1 = h.level(0), h.level(1)
    A = dense(rp, c, v)
    Ac = dense(L1["rowptr"], L1["col"], L1["val"])
    ms = np.sqrt(L1["minv"])
    lam, U = np.linalg.eigh(ms[:, None] * Ac * ms[None, :])
    assert lam.min() > 0 and lam.max() <= 1 + 1e-14
    Bc = ms[:, None] * (U * ((1 - (1 - lam) ** K) / lam)) @ U.T * ms[None, :]
    Pm = prolongator(L0)
    Mi = L0["minv"]
    n = s[0]
    I = np.eye(n)
    S0 = I - Mi[:, None] * A
    E = S0 @ (I - Pm @ (Bc @ (Pm.T @ A))) @ S0
    rng = np.random.default_rng(K)
    for _ in range(4):
        b = rng.standard_normal(n)
        ref = (I - E) @ np.linalg.solve(A, b)
        np.testing.assert_allclose(h.vcycle(b), ref, rtol=0, atol=1e-11 * np.abs(ref).max())


def test_stall_below_dense_limit_is_factored_and_above_without_sweeps_fails():
    rp, c, v = _stall_matrix(1800, 200, seed=4)      # stalls below 2000 rows: dense factor
    h = oracle.Hierarchy(rp, c, v)
    s = h.sizes()
    assert len(s) == 2 and s[1] > 0.9 * s[0] and s[1] <= 2000 and h.coarse_sweeps == 0
    Lf = h.coarse_factor()
    Ac = dense(*(h.level(1)[k] for k in ("rowptr", "col", "val")))
    np.testing.assert_allclose(Lf @ Lf.T, Ac, rtol=0, atol=1e-13)
    rp, c, v = _stall_matrix(2200, 200, seed=4)
    with pytest.raises(RuntimeError):
        oracle.Hierarchy(rp, c, v, coarse_sweeps=0)


def test_lognormal_diffusion_stalls_and_pcg_converges():
    rp, c, v = P.diffusion7(48, seed=0)
    h = oracle.Hierarchy(rp, c, v)
    s = h.sizes()
    assert s[-1] > 2000 and s[-1] > 0.9 * s[-2] and h.coarse_sweeps == 30
    rng = np.random.default_rng(0)
    u, w = rng.standard_normal(s[0]), rng.standard_normal(s[0])
    assert abs(u @ h.vcycle(w) - w @ h.vcycle(u)) <= 1e-12 * abs(u @ h.vcycle(w))
    b = P.rhs_from_solution(rp, c, v, P.x_true(s[0], 0))
    r = h.pcg(b)
    assert r["status"] == oracle.OK and r["relres"] <= 1e-6


def _laplace1d(n):
    A = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1], format="csr")
    A.sort_indices()
    return A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.copy()


def test_smoothed_prolongator_1d_closed_form():
    # 1-D Laplacian (2, -1): all matching weights tie, so one sweep pairs
    # (0,1), (2,3), ...; P^ = 1/sqrt(2) on each pair; ||D^-1 A||_inf = 2 gives
    # omega = 1/2 and P = (I - A/4) P^: the classic smoothed-aggregation
    # columns (1/4, 3/4, 3/4, 1/4) / sqrt(2).
    n = 16
    rp, c, v = _laplace1d(n)
    h = oracle.Hierarchy(rp, c, v, sweeps=1, coarse_max=4, prol=1)
    L0 = h.level(0)
    assert np.array_equal(L0["agg"], np.arange(n) // 2)
    prp, pci, pv, omega = h.prolongator(0)
    assert omega == 0.5
    Pm = sp.csr_matrix((pv, pci, prp), shape=(n, n // 2)).toarray()
    ref = np.zeros((n, n // 2))
    for J in range(n // 2):
        ref[2 * J, J] = ref[2 * J + 1, J] = 0.75
        if 2 * J - 1 >= 0:
            ref[2 * J - 1, J] = 0.25
        if 2 * J + 2 < n:
            ref[2 * J + 2, J] = 0.25
    np.testing.assert_allclose(Pm, ref / np.sqrt(2), rtol=0, atol=1e-15)


@pytest.mark.parametrize("case", ["poisson10_aggr8", "poisson9odd", "diffusion10", "random"])
def test_smoothed_hierarchy_galerkin_matches_dense(case):
    if case == "poisson10_aggr8":
        rp, c, v = P.poisson7(10)
        sweeps = 3
    elif case == "poisson9odd":
        rp, c, v = P.poisson7(9)
        sweeps = 2
    elif case == "diffusion10":
        rp, c, v = P.diffusion7(10, seed=1, az=100.0)
        sweeps = 2
    else:
        rp, c, v = P.random_spd_csr(300, 7, density=0.02, maxrow=30)
        sweeps = 2
    h = oracle.Hierarchy(rp, c, v, sweeps=sweeps, coarse_max=40, prol=1)
    assert h.nlevels >= 2
    for l in range(h.nlevels - 1):
        L, C = h.level(l), h.level(l + 1)
        A = dense(L["rowptr"], L["col"], L["val"])
        prp, pci, pv, omega = h.prolongator(l)
        Pm = sp.csr_matrix((pv, pci, prp), shape=(L["n"], L["nc"])).toarray()
        # omega from its definition, P = (I - omega D^-1 A) P^ densely
        d = np.diag(A)
        assert omega == pytest.approx(1.0 / (np.abs(A).sum(axis=1) / d).max(), rel=1e-15)
        Ph = prolongator(L)
        np.testing.assert_allclose(Pm, Ph - omega * (A / d[:, None]) @ Ph, rtol=0, atol=1e-14)
        Ac = dense(C["rowptr"], C["col"], C["val"])
        scale = np.abs(A).max()
        np.testing.assert_allclose(Ac, Pm.T @ A @ Pm, rtol=0, atol=1e-13 * scale)
        assert np.abs(Ac - Ac.T).max() <= 1e-13 * np.abs(Ac).max()
        if L["nc"] <= 1500:
            assert np.linalg.eigvalsh(Ac).min() > 0
        counts = np.bincount(L["agg"], minlength=L["nc"])
        assert counts.max() <= 2 ** sweeps and counts.min() >= 1


@pytest.mark.parametrize("prol,nu", [(0, 2), (1, 1), (1, 3)])
def test_vcycle_nu_sweeps_two_level_formula(prol, nu):
    # eq. (amg) with nu smoothing sweeps: E = S^nu (I - P A_c^-1 P^T A) S^nu,
    # S = I - M^-1 A, and B = (I - E) A^-1.
    n = 8
    rp, c, v = P.poisson7(n)
    h = oracle.Hierarchy(rp, c, v, prol=prol, nu=nu)
    assert h.nlevels == 2
    L0, L1 = h.level(0), h.level(1)
    A = dense(rp, c, v)
    Ac = dense(L1["rowptr"], L1["col"], L1["val"])
    prp, pci, pv, _ = h.prolongator(0)
    Pm = sp.csr_matrix((pv, pci, prp), shape=(512, L0["nc"])).toarray()
    I = np.eye(512)
    S = I - L0["minv"][:, None] * A
    Snu = np.linalg.matrix_power(S, nu)
    E = Snu @ (I - Pm @ np.linalg.solve(Ac, Pm.T @ A)) @ Snu
    Bref = (I - E) @ np.linalg.inv(A)
    B = np.stack([h.vcycle(I[:, j]) for j in range(512)], axis=1)
    np.testing.assert_allclose(B, Bref, rtol=0, atol=1e-12)
    assert np.abs(B - B.T).max() < 1e-13
    B32 = np.stack([h.vcycle32(I[:, j]) for j in range(0, 512, 37)], axis=1)
    assert np.abs(B32 - Bref[:, ::37]).max() <= 1e-5 * np.abs(Bref).max()


def test_variable_vcycle_three_levels_recursive_formula():
    # variable V-cycle (nu_l = nu 2^l): eq. (amg) applied recursively,
    # B_l = (I - E_l) A_l^-1 with E_l = S_l^nu_l (I - P_l B_{l+1} P_l^T A_l) S_l^nu_l
    # and B_L = A_L^-1 on the coarsest level.
    rp, c, v = P.poisson7(8)
    h = oracle.Hierarchy(rp, c, v, sweeps=3, coarse_max=10, nu=2, nu_double=True)
    assert h.sizes() == [512, 64, 8]
    B = None
    for l in range(h.nlevels - 1, -1, -1):
        L = h.level(l)
        A = dense(L["rowptr"], L["col"], L["val"])
        if l == h.nlevels - 1:
            B = np.linalg.inv(A)
            continue
        prp, pci, pv, _ = h.prolongator(l)
        Pm = sp.csr_matrix((pv, pci, prp), shape=(L["n"], L["nc"])).toarray()
        I = np.eye(L["n"])
        Snu = np.linalg.matrix_power(I - L["minv"][:, None] * A, 2 * 2 ** l)
        E = Snu @ (I - Pm @ B @ Pm.T @ A) @ Snu
        B = (I - E) @ np.linalg.inv(A)
    V = np.stack([h.vcycle(np.eye(512)[:, j]) for j in range(0, 512, 7)], axis=1)
    np.testing.assert_allclose(V, B[:, ::7], rtol=0, atol=1e-12)


def test_vbm_aggregates_1d_closed_form():
    # 1-D Laplacian: every off-diagonal is strong (|a_ij| / sqrt(a_ii a_jj) =
    # 1/2 >= theta). Step 1 in ascending order takes {0,1}, then the
    # neighbourhoods {2,3,4}, {5,6,7}, ... of every third node, and {14,15}.
    n = 16
    rp, c, v = _laplace1d(n)
    h = oracle.Hierarchy(rp, c, v, aggr=1, theta=0.01, coarse_max=4)
    agg = h.level(0)["agg"]
    assert list(agg) == [0, 0, 1, 1, 1, 2, 2, 2, 3, 3, 3, 4, 4, 4, 5, 5]
    # P^_{i,agg_i} = w_i = 1 (no normalisation) and the smoothed P keeps P^ 1 = 1
    assert np.all(h.level(0)["p"] == 1.0)


def test_vbm_threshold_and_invariants():
    # theta above every coupling ratio (1/6 for the 7-point stencil): no strong
    # neighbours, every node is its own aggregate
    rp, c, v = P.poisson7(6)
    h = oracle.Hierarchy(rp, c, v, aggr=1, theta=0.5, coarse_max=100)
    assert np.array_equal(h.level(0)["agg"], np.arange(216))
    for case in ["poisson12", "diffusion10", "random"]:
        if case == "poisson12":
            rp, c, v = P.poisson7(12)
        elif case == "diffusion10":
            rp, c, v = P.diffusion7(10, seed=2, az=100.0)
        else:
            rp, c, v = P.random_spd_csr(300, 7, density=0.02, maxrow=30)
        h = oracle.Hierarchy(rp, c, v, aggr=1, theta=0.05, coarse_max=40, prol=1)
        for l in range(h.nlevels - 1):
            L = h.level(l)
            A = dense(L["rowptr"], L["col"], L["val"])
            agg = L["agg"]
            assert agg.min() == 0 and agg.max() == L["nc"] - 1
            d = np.diag(A)
            strong = (np.abs(A) >= 0.05 * np.sqrt(np.outer(d, d))) & ~np.eye(L["n"], dtype=bool)
            # every aggregate is connected in the strength graph, or a singleton
            for J in range(L["nc"]):
                mem = np.flatnonzero(agg == J)
                if len(mem) == 1:
                    continue
                seen, todo = {mem[0]}, [mem[0]]
                while todo:
                    i = todo.pop()
                    for j in mem[strong[i, mem]]:
                        if j not in seen:
                            seen.add(j)
                            todo.append(j)
                assert len(seen) == len(mem), (case, l, J)
            prp, pci, pv, omega = h.prolongator(l)
            Pm = sp.csr_matrix((pv, pci, prp), shape=(L["n"], L["nc"])).toarray()
            Ph = prolongator(L)
            np.testing.assert_allclose(Pm, Ph - omega * (A / d[:, None]) @ Ph, rtol=0, atol=1e-14)
            C = h.level(l + 1)
            Ac = dense(C["rowptr"], C["col"], C["val"])
            np.testing.assert_allclose(Ac, Pm.T @ A @ Pm, rtol=0, atol=1e-13 * np.abs(A).max())


def test_smatch_beats_tentative_in_iterations():
    # SMATCH-style (aggregates <= 8, smoothed prolongator, 4 sweeps) against
    # the tentative V(1,1) of the main path on the same problem
    rp, c, v = P.poisson7(32)
    b = P.rhs_from_solution(rp, c, v, P.x_true(32 ** 3, 0))
    sm = oracle.Hierarchy(rp, c, v, sweeps=3, prol=1, nu=4).pcg(b)
    vm = oracle.Hierarchy(rp, c, v).pcg(b)
    assert sm["status"] == vm["status"] == oracle.OK
    assert sm["iters"] < vm["iters"] and sm["relres"] <= 1e-6


def test_vcycle_multilevel_symmetric_positive():
    rp, c, v = P.poisson7(16)
    h = oracle.Hierarchy(rp, c, v, coarse_max=30)
    assert h.nlevels >= 3
    rng = np.random.default_rng(0)
    u, w = rng.standard_normal(16 ** 3), rng.standard_normal(16 ** 3)
    assert abs(u @ h.vcycle(w) - w @ h.vcycle(u)) <= 1e-12 * abs(u @ h.vcycle(w)) + 1e-14
    for _ in range(3):
        z = rng.standard_normal(16 ** 3)
        assert z @ h.vcycle(z) > 0


def test_vcycle32_close_to_vcycle64():
    rp, c, v = P.poisson7(24)
    h = oracle.Hierarchy(rp, c, v)
    r = np.random.default_rng(2).standard_normal(24 ** 3)
    z64, z32 = h.vcycle(r), h.vcycle32(r)
    err = np.linalg.norm(z32 - z64) / np.linalg.norm(z64)
    assert 0 < err <= 1e-5


# --------------------------------------------------------------------------
# Krylov
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_single_level_pcg_is_exact_in_one_iteration(n):
    rp, c, v = P.poisson7(n)
    h = oracle.Hierarchy(rp, c, v)
    assert h.nlevels == 1
    b = P.rhs_uniform(n ** 3, 9)
    r = h.pcg(b, rtol=1e-10)
    assert r["status"] == oracle.OK and r["iters"] == 1
    ref = np.linalg.solve(dense(rp, c, v), b)
    np.testing.assert_allclose(r["x"], ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_jacobi_pcg_iterates_match_scipy_cg():
    n = 10
    rp, c, v = P.diffusion7(n, seed=4)
    A = sp.csr_matrix((v, c, rp), shape=(n ** 3, n ** 3))
    b = P.rhs_uniform(n ** 3, 4)
    h = oracle.Hierarchy(rp, c, v)
    dinv = 1.0 / A.diagonal()
    M = spla.LinearOperator(A.shape, matvec=lambda x: dinv * x)
    for k in [1, 2, 5, 9]:
        xs, _ = spla.cg(A, b, rtol=1e-30, atol=0.0, maxiter=k, M=M)
        r = h.pcg(b, rtol=1e-30, maxit=k, prec=oracle.PREC_JACOBI)
        assert r["iters"] == k
        np.testing.assert_allclose(r["x"], xs, rtol=0, atol=1e-11 * np.abs(xs).max())


def test_unpreconditioned_cg_lanczos_recovers_lambda_max():
    n = 10
    rp, c, v = P.poisson7(n)
    h = oracle.Hierarchy(rp, c, v)
    b = P.rhs_uniform(n ** 3, 3)
    r = h.pcg(b, rtol=1e-13, maxit=400, prec=oracle.PREC_NONE, history=True)
    al, be = r["alpha"], r["beta"]
    m = len(al) - 1
    T = np.zeros((m, m))
    for j in range(m):
        T[j, j] = 1.0 / al[j] + (be[j - 1] / al[j - 1] if j > 0 else 0.0)
        if j + 1 < m:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(be[j]) / al[j]
    lam = np.linalg.eigvalsh(T)
    assert abs(lam.max() - (6 + 6 * np.cos(np.pi / (n + 1)))) < 1e-8
    assert abs(lam.min() - (6 - 6 * np.cos(np.pi / (n + 1)))) < 1e-8


def test_manufactured_solution_within_condition_bound():
    n = 32
    rp, c, v = P.poisson7(n)
    h = oracle.Hierarchy(rp, c, v)
    xt = P.x_true(n ** 3, 0)
    b = P.rhs_from_solution(rp, c, v, xt)
    r = h.pcg(b, rtol=1e-6)
    assert r["status"] == oracle.OK and r["relres"] <= 1e-6
    kappa = (6 + 6 * np.cos(np.pi / (n + 1))) / (6 - 6 * np.cos(np.pi / (n + 1)))
    assert np.linalg.norm(r["x"] - xt) / np.linalg.norm(xt) <= kappa * 1e-6
    assert r["iters"] == 16        # calibration: matches an independent scipy replica


def test_fcg_with_fixed_preconditioner_equals_pcg():
    n = 16
    rp, c, v = P.poisson7(n)
    h = oracle.Hierarchy(rp, c, v)
    b = P.rhs_uniform(n ** 3, 11)
    for k in [1, 3, 6]:
        a = h.pcg(b, rtol=1e-30, maxit=k)
        f = h.fcg(b, rtol=1e-30, maxit=k, form=0)
        np.testing.assert_allclose(f["x"], a["x"], rtol=0, atol=1e-10 * np.abs(a["x"]).max())
    a = h.pcg(b, rtol=1e-6)
    f = h.fcg(b, rtol=1e-6, form=0)
    assert abs(a["iters"] - f["iters"]) <= 1


def test_mixed_fcg_reaches_true_residual():
    n = 24
    rp, c, v = P.diffusion7(n, seed=0)
    h = oracle.Hierarchy(rp, c, v)
    b = P.rhs_from_solution(rp, c, v, P.x_true(n ** 3, 0))
    f = h.fcg(b, rtol=1e-6, form=1)
    d = h.pcg(b, rtol=1e-6)
    assert f["status"] == oracle.OK and f["relres"] <= 1e-6
    assert abs(f["iters"] - d["iters"]) <= 2


def test_failure_paths():
    rp, c, v = P.poisson7(6)
    h = oracle.Hierarchy(rp, c, v, coarse_max=20)
    b = P.rhs_uniform(216, 0)
    r = h.pcg(np.zeros(216))
    assert r["status"] == oracle.OK and r["iters"] == 0 and not r["x"].any()
    r = h.pcg(b, maxit=1, rtol=1e-12)
    assert r["status"] == oracle.NOCONV and r["iters"] == 1 and 0 < r["relres"] < 1
    bn = b.copy(); bn[5] = np.nan
    assert h.pcg(bn)["status"] == oracle.ERR_NAN
    v2 = v.copy()
    v2[rp[3] + list(c[rp[3]:rp[4]]).index(3)] = -6.0
    with pytest.raises(RuntimeError):
        oracle.Hierarchy(rp, c, v2)


# --------------------------------------------------------------------------
# The paper's printed operator complexity (golden fixture)
# --------------------------------------------------------------------------

@pytest.mark.slow
def test_vmatch_operator_complexity_matches_paper():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "paper_operator_complexity.txt"))
            if l.strip() and not l.startswith("#")]
    ref = float([r for r in rows if r[0] == "VMATCH" and r[1] == "1"][0][2])
    rp, c, v = P.poisson7(200)                 # 8e6 unknowns, one GPU's share
    h = oracle.Hierarchy(rp, c, v, sweeps=3)   # aggregates <= 8, tentative prolongator
    assert abs(h.operator_complexity() - ref) <= 0.01


@pytest.mark.slow
def test_vbm_operator_complexity_near_paper():
    # The paper does not state its VBM strength threshold; for the 7-point
    # stencil every coupling ratio is 1/6, so any theta < 1/6 gives the same
    # aggregates. The oracle's 1.592 at 200^3 is within 0.02 of the printed
    # 1.575; the remaining gap comes from unpublished details of the toolkit's
    # aggregation (boundary treatment, order of the passes), so the bound is
    # loose but still separates VBM from the tentative (1.22) or matching-based
    # (1.14 / 2.2) hierarchies.
    rows = [l.split() for l in open(os.path.join(GOLDEN, "paper_operator_complexity.txt"))
            if l.strip() and not l.startswith("#")]
    ref = float([r for r in rows if r[0] == "VBM" and r[1] == "1"][0][2])
    rp, c, v = P.poisson7(200)
    h = oracle.Hierarchy(rp, c, v, aggr=1, theta=0.01, prol=1, nu=4)
    assert abs(h.operator_complexity() - ref) <= 0.02


def _indefinite_shifted_poisson(n, sigma):
    # Poisson - sigma I with lambda_min(A) < sigma < lambda_min(A_coarse):
    # the build succeeds (positive diagonals, SPD coarsest level) but A has a
    # negative eigenvalue, so CG meets p.Ap <= 0 after a few iterations
    rp, c, v = P.poisson7(n)
    v = v.copy()
    rows = np.repeat(np.arange(n ** 3), np.diff(rp))
    v[rows == c] -= sigma
    return rp, c, v


@pytest.mark.parametrize("kind", ["pcg", "fcg64", "fcg32"])
def test_breakdown_returns_last_valid_iterate(kind):
    n, sigma = 8, 0.40
    lam_min = 6.0 - 6.0 * np.cos(np.pi / (n + 1))          # closed form, 0.3618
    assert lam_min < sigma
    rp, c, v = _indefinite_shifted_poisson(n, sigma)
    h = oracle.Hierarchy(rp, c, v, coarse_max=20)
    b = P.rhs_uniform(n ** 3, 1)

    def solve(maxit):
        if kind == "pcg":
            return h.pcg(b, rtol=1e-10, maxit=maxit)
        return h.fcg(b, rtol=1e-10, maxit=maxit, form=0 if kind == "fcg64" else 1)
    bad = solve(300)
    assert bad["status"] == oracle.ERR_NOT_SPD and bad["iters"] >= 2
    last = solve(bad["iters"])
    assert last["status"] == oracle.NOCONV and last["iters"] == bad["iters"]
    np.testing.assert_array_equal(bad["x"], last["x"])
