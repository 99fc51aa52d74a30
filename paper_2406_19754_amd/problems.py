"""Seeded synthetic inputs for the AMG-PCG solve phase.

This module builds test problems and random inputs only; it holds none of the
solver's arithmetic (no aggregation, smoothing, transfer or Krylov step). Both
the CPU oracle's tests and the HIP path's tests and benchmark draw their
inputs from here, so that the two sides always see identical bytes.

Problems (all on an n^3 grid, row index ``i + n*(j + n*k)``, x fastest):

* ``poisson7(n)``: the 7-point finite-difference Laplacian of the paper's
  test problem (Section "Numerical Example"), unscaled: 6 on the diagonal,
  -1 per in-range face neighbour, Dirichlet neighbours dropped.
* ``diffusion7(n, seed, sigma, az)``: a cell-centred finite-volume
  discretisation of -div(k grad u) with lognormal k, harmonic-mean face
  transmissibilities and an optional z-anisotropy factor. With k = 1 and
  az = 1 it reproduces ``poisson7`` bit for bit.

CSR arrays are (rowptr int32, col int32, val float64) with ascending columns.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "poisson7", "diffusion7", "poisson_nnz", "x_true", "rhs_from_solution",
    "rhs_uniform", "rhs_bumps", "net_param_count", "net_init", "crop_origins",
    "random_spd_csr",
]

# neighbour order in a row = ascending column order
_OFFS = ("mz", "my", "mx", "d", "px", "py", "pz")


def poisson_nnz(n: int) -> int:
    """Number of stored entries of the 7-point operator on an n^3 grid."""
    return 7 * n ** 3 - 6 * n ** 2


def _grid_masks(n: int):
    N = n ** 3
    idx = np.arange(N, dtype=np.int64)
    i = idx % n
    j = (idx // n) % n
    k = idx // (n * n)
    have = {
        "mz": k > 0, "my": j > 0, "mx": i > 0,
        "d": np.ones(N, dtype=bool),
        "px": i < n - 1, "py": j < n - 1, "pz": k < n - 1,
    }
    step = {"mz": -n * n, "my": -n, "mx": -1, "d": 0, "px": 1, "py": n, "pz": n * n}
    return N, idx, have, step


def _assemble(n: int, values: dict):
    """Scatter per-neighbour value arrays (length N each) into CSR."""
    N, idx, have, step = _grid_masks(n)
    counts = np.zeros(N, dtype=np.int32)
    for t in _OFFS:
        counts += have[t]
    rowptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    nnz = int(rowptr[-1])
    if nnz >= 2 ** 31:
        raise ValueError("nnz exceeds int32 range")
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    pos = rowptr[:-1].copy()
    for t in _OFFS:
        m = have[t]
        p = pos[m]
        col[p] = (idx[m] + step[t]).astype(np.int32)
        v = values[t]
        val[p] = v if np.isscalar(v) else v[m]
        pos[m] += 1
    return rowptr.astype(np.int32), col, val


def poisson7(n: int):
    """7-point Laplacian on an n^3 grid with Dirichlet boundary (unscaled)."""
    vals = {t: -1.0 for t in _OFFS}
    vals["d"] = 6.0
    return _assemble(n, vals)


def diffusion7(n: int, seed: int = 0, sigma: float = 1.5, az: float = 1.0,
               k: np.ndarray | None = None):
    """Finite-volume -div(k grad u) on an n^3 grid.

    k = exp(sigma * g) with g ~ N(0,1) i.i.d. per cell from
    ``numpy.random.default_rng(seed)`` unless ``k`` is given. A face between
    cells lo < hi has transmissibility T = 2*k_lo*k_hi/(k_lo+k_hi) (one value
    shared by both rows, so the matrix is bitwise symmetric); a Dirichlet
    boundary face has T = k_i (ghost cell with equal k and u = 0). Every
    z-face is multiplied by ``az``. Diagonal = sum of the six face values in
    the order -z, -y, -x, +x, +y, +z; off-diagonal = -T.
    """
    N = n ** 3
    if k is None:
        g = np.random.default_rng(seed).standard_normal(N)
        k = np.exp(sigma * g)
    k = np.asarray(k, dtype=np.float64).reshape(n, n, n)  # [z, y, x]
    fac = {"x": 1.0, "y": 1.0, "z": float(az)}

    def face(axis):
        ax = {"z": 0, "y": 1, "x": 2}[axis]
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(0, n - 1)
        hi[ax] = slice(1, n)
        klo = k[tuple(lo)]
        khi = k[tuple(hi)]
        t = 2.0 * klo * khi / (klo + khi)
        if fac[axis] != 1.0:
            t = t * fac[axis]
        # minus-face of cell c (towards c-1) and plus-face (towards c+1)
        tm = np.empty_like(k)
        tp = np.empty_like(k)
        first = [slice(None)] * 3
        last = [slice(None)] * 3
        first[ax] = slice(0, 1)
        last[ax] = slice(n - 1, n)
        bnd_lo = k[tuple(first)] * fac[axis] if fac[axis] != 1.0 else k[tuple(first)]
        bnd_hi = k[tuple(last)] * fac[axis] if fac[axis] != 1.0 else k[tuple(last)]
        tm[tuple(hi)] = t
        tm[tuple(first)] = bnd_lo
        tp[tuple(lo)] = t
        tp[tuple(last)] = bnd_hi
        return tm.reshape(-1), tp.reshape(-1)

    tmz, tpz = face("z")
    tmy, tpy = face("y")
    tmx, tpx = face("x")
    diag = tmz + tmy
    diag = diag + tmx
    diag = diag + tpx
    diag = diag + tpy
    diag = diag + tpz
    vals = {"mz": -tmz, "my": -tmy, "mx": -tmx, "d": diag,
            "px": -tpx, "py": -tpy, "pz": -tpz}
    return _assemble(n, vals)


def x_true(N: int, seed: int = 0) -> np.ndarray:
    """Manufactured solution, U[0,1) from ``default_rng(seed)``."""
    return np.random.default_rng(seed).random(N)


def rhs_from_solution(rowptr, col, val, x) -> np.ndarray:
    """b = A x for a manufactured solution (input construction only)."""
    import scipy.sparse as sp
    n = len(rowptr) - 1
    A = sp.csr_matrix((val, col, rowptr), shape=(n, n))
    return A @ np.asarray(x, dtype=np.float64)


def projection_signs(N: int, j: int) -> np.ndarray:
    """The j-th random +-1 test vector of length N (``default_rng(50000 + j)``).

    Comparison harness only: for a difference d, (w.d)^2 has mean |d|^2 over
    such w, so a few projections of a long vector stand in for its norm
    without storing it."""
    return np.random.default_rng(50000 + j).integers(0, 2, N, dtype=np.int8).astype(np.float64) * 2.0 - 1.0


def rhs_uniform(N: int, seed: int) -> np.ndarray:
    """Right-hand side with entries U[-1,1) from ``default_rng(seed)``."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, N)


def rhs_bumps(n: int, seed: int) -> np.ndarray:
    """Smooth right-hand side: a sum of 1..4 Gaussian bumps.

    b(x) = sum_m a_m exp(-|x - c_m|^2 / (2 s_m^2)) at cell centres
    x = (i+1)/(n+1), with c_m ~ U[0.1,0.9]^3, s_m ~ U[0.03,0.15],
    a_m ~ U[-1,1].
    """
    rng = np.random.default_rng(seed)
    M = int(rng.integers(1, 5))
    t = (np.arange(n, dtype=np.float64) + 1.0) / (n + 1.0)
    Z, Y, X = np.meshgrid(t, t, t, indexing="ij")
    b = np.zeros((n, n, n))
    for _ in range(M):
        c = rng.uniform(0.1, 0.9, 3)
        s = rng.uniform(0.03, 0.15)
        a = rng.uniform(-1.0, 1.0)
        d2 = (X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2
        b += a * np.exp(-d2 / (2.0 * s * s))
    return b.reshape(-1)


# ---------------------------------------------------------------------------
# learned preconditioner: parameter layout and random inputs
#   W1[16][1][27] b1[16] W2[16][16][27] b2[16] W3[1][16][27] b3[1]
# tap index t = (dz*3 + dy)*3 + dx, offset (dz-1, dy-1, dx-1)
# ---------------------------------------------------------------------------
NET_C = 16


def net_param_count(c: int = NET_C) -> int:
    return c * 27 + c + c * c * 27 + c + c * 27 + 1


def net_init(seed: int, c: int = NET_C, last_scale: float = 1.0) -> np.ndarray:
    """Kaiming-normal initial weights (std sqrt(2/fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    w1 = rng.standard_normal(c * 27) * np.sqrt(2.0 / 27)
    w2 = rng.standard_normal(c * c * 27) * np.sqrt(2.0 / (c * 27))
    w3 = rng.standard_normal(c * 27) * np.sqrt(2.0 / (c * 27)) * last_scale
    p = np.concatenate([w1, np.zeros(c), w2, np.zeros(c), w3, np.zeros(1)])
    return p.astype(np.float32)


def crop_origins(seed: int, count: int, dims, crop: int) -> np.ndarray:
    """Random crop corners (z, y, x) inside a grid of shape ``dims``."""
    rng = np.random.default_rng(seed)
    out = np.empty((count, 3), dtype=np.int32)
    for a in range(3):
        out[:, a] = rng.integers(0, dims[a] - crop + 1, count)
    return out


def random_spd_csr(n: int, seed: int, density: float = 0.05, maxrow: int | None = None):
    """A random sparse symmetric diagonally dominant matrix (SPD), CSR.

    Off-diagonal entries are negative or positive; the diagonal is
    1 + sum |a_ij| + U[0,1), so the matrix is SPD. Rows have unequal
    lengths (useful for exercising slice padding).
    """
    rng = np.random.default_rng(seed)
    A = np.zeros((n, n))
    for i in range(n):
        for j in range(i + 1, n):
            if rng.random() < density:
                v = rng.uniform(-1.0, 0.5)
                A[i, j] = v
                A[j, i] = v
    if maxrow is not None:
        # force a few long rows
        for i in rng.choice(n, size=min(3, n), replace=False):
            js = rng.choice(n, size=min(maxrow, n - 1), replace=False)
            for j in js:
                if j != i:
                    v = rng.uniform(-1.0, 0.0)
                    A[i, j] = v
                    A[j, i] = v
    np.fill_diagonal(A, 0.0)
    d = 1.0 + np.abs(A).sum(axis=1) + rng.random(n)
    A[np.arange(n), np.arange(n)] = d
    rowptr = np.zeros(n + 1, dtype=np.int32)
    cols, vals = [], []
    for i in range(n):
        nz = np.nonzero(A[i])[0]
        cols.append(nz.astype(np.int32))
        vals.append(A[i, nz])
        rowptr[i + 1] = rowptr[i] + len(nz)
    return rowptr, np.concatenate(cols), np.concatenate(vals)
