"""Pins for the oracle's learned flexible-CG branch (orc_fcg with a network).

The schedule is the reading taken for "the network applied alternately with
one V-cycle, V-cycle fallback on stagnation": iterations k = 1, 3, 5, ...
(counting from 0) try z = s net(r/s) with s = ||r||_2 / sqrt(N); a step with
z.r <= 0 runs the V-cycle instead, two such scheduled steps in a row switch
the network off, and so does a network step that leaves
||r_new|| > 0.9 ||r_old||. Every scheduled step that ran the V-cycle counts as
a fallback, also after the switch-off.

These tests hold the oracle to an independent FCG(1) written here in NumPy
from that statement (dense-free, scipy sparse products), which takes its
preconditioners from the oracle's separately pinned V-cycle and network
application, and compare every iterate. Nets and problems are chosen so that
each branch of the schedule is taken; the reference's event log asserts it.
The scale s is pinned against torch's convolution applied to r/s: the
network is not homogeneous (GELU, biases), so any other scale shows.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import torch
import torch.nn.functional as F

import oracle
from paper_2406_19754_amd import problems as P

C = 16


def identity_like_net(a, c, b3=0.0):
    """A net that acts on each cell alone: out = c (G(G(a u)) - G(G(-a u))) + b3
    with G = GELU (centre taps only), an odd increasing map of u when b3 = 0,
    so u.out > 0 for every u != 0."""
    W1 = np.zeros((C, 1, 27))
    W2 = np.zeros((C, C, 27))
    W3 = np.zeros((1, C, 27))
    W1[0, 0, 13], W1[1, 0, 13] = a, -a
    W2[0, 0, 13] = W2[1, 1, 13] = 1.0
    W3[0, 0, 13], W3[0, 1, 13] = c, -c
    return np.concatenate([W1.ravel(), np.zeros(C), W2.ravel(), np.zeros(C), W3.ravel(), [b3]])


def fcg_learned_reference(A, b, vcycle, net, rtol, maxit):
    """FCG(1) from x0 = 0 with the network schedule stated in the module doc.

    Returns the iterates x_1..x_K, K, the fallback count, the number of
    network applications and an event log [(k, what)]."""
    nb = np.linalg.norm(b)
    x = np.zeros_like(b)
    r = b.copy()
    iterates, events = [], []
    net_on, fails, fallbacks, evals = net is not None, 0, 0, 0
    p_prev = q_prev = None
    pq_prev = 0.0
    k = 0
    while k < maxit and np.linalg.norm(r) > rtol * nb:
        took_net = False
        if net is not None and k % 2 == 1 and net_on:
            z = net(r)
            evals += 1
            if z @ r > 0:
                took_net, fails = True, 0
                events.append((k, "net"))
            else:
                fails += 1
                fallbacks += 1
                events.append((k, "z.r<=0"))
                if fails == 2:
                    net_on = False
                    events.append((k, "off: two failures"))
                z = vcycle(r)
        else:
            if net is not None and k % 2 == 1:
                fallbacks += 1
            z = vcycle(r)
        # flexible direction: A-orthogonal to the previous one only
        p = z if p_prev is None else z - (z @ q_prev) / pq_prev * p_prev
        q = A @ p
        pq = p @ q
        assert pq > 0
        r_before = np.linalg.norm(r)
        alpha = (p @ r) / pq
        x = x + alpha * p
        r = r - alpha * q
        k += 1
        iterates.append(x.copy())
        if took_net and np.linalg.norm(r) > 0.9 * r_before:
            net_on = False
            events.append((k - 1, "off: stagnation"))
        p_prev, q_prev, pq_prev = p, q, pq
        if np.linalg.norm(r) <= rtol * nb:
            rt = b - A @ x
            if np.linalg.norm(rt) <= rtol * nb:
                break
            r, p_prev = rt, None          # residual replacement, directions restart
            events.append((k, "replace"))
    return iterates, k, fallbacks, evals, events


def shifted_poisson(n, shift):
    rp, c, v = P.poisson7(n)
    v = v.copy()
    rows = np.repeat(np.arange(n ** 3), np.diff(rp))
    v[rows == c] += shift
    return rp, c, v


# (name, grid, diagonal shift, net, rhs seed, expected event kinds)
CASES = [
    # an odd increasing map is always a descent direction and, on Poisson,
    # always cuts ||r|| by more than 10 %: every scheduled step is a network step
    ("all_accepted", 8, 0.0, identity_like_net(4.0, 1.0), 1, ["net"] * 10),
    # its negative is never one: two failures switch the network off
    ("two_failures", 8, 0.0, identity_like_net(4.0, -1.0), 1, ["z.r<=0", "z.r<=0", "off: two failures"]),
    # a large bias makes the sign of z.r follow sum(r): one failure, then an
    # accepted step that stagnates
    ("fail_accept_stagnate", 8, 0.0, identity_like_net(4.0, 0.02, -10.0), 1,
     ["z.r<=0", "net", "off: stagnation"]),
    # on a strongly diagonally dominant operator the V-cycle converges so fast
    # that the biased network step cannot keep up
    ("accept_stagnate", 8, 20.0, identity_like_net(4.0, 1.0 / 26.0, -0.5), 1, ["net", "off: stagnation"]),
]


@pytest.mark.parametrize("name,n,shift,params,seed,kinds", CASES, ids=[c[0] for c in CASES])
def test_learned_fcg_iterates_match_independent_reference(name, n, shift, params, seed, kinds):
    rp, c, v = shifted_poisson(n, shift)
    N = n ** 3
    A = sp.csr_matrix((v, c, rp), shape=(N, N))
    h = oracle.Hierarchy(rp, c, v, coarse_max=20)
    assert h.nlevels >= 3
    b = P.rhs_uniform(N, seed)
    dims = (n, n, n)
    xs, K, fb, ne, events = fcg_learned_reference(A, b, h.vcycle, lambda r: oracle.net_apply(params, r, dims),
                                                  1e-6, 200)
    assert [e for _, e in events] == kinds
    full = h.fcg(b, rtol=1e-6, params=params, dims=dims)
    assert full["status"] == oracle.OK
    assert (full["iters"], full["fallbacks"], full["net_evals"]) == (K, fb, ne)
    # iterate by iterate: the oracle stopped after k iterations equals x_k
    for k in range(1, K + 1):
        o = h.fcg(b, rtol=1e-6, maxit=k, params=params, dims=dims)
        assert o["iters"] == k
        np.testing.assert_allclose(o["x"], xs[k - 1], rtol=0, atol=1e-12 * np.abs(xs[k - 1]).max())
    assert full["relres"] <= 1e-6


def test_schedule_differs_from_plain_fcg():
    # the accepted-network case really changes the iterates (the comparison
    # above is not a comparison of two plain V-cycle solves)
    n = 8
    rp, c, v = shifted_poisson(n, 0.0)
    h = oracle.Hierarchy(rp, c, v, coarse_max=20)
    b = P.rhs_uniform(n ** 3, 1)
    a = h.fcg(b, rtol=1e-6, maxit=2, params=identity_like_net(4.0, 1.0), dims=(n, n, n))
    p = h.fcg(b, rtol=1e-6, maxit=2)
    assert np.linalg.norm(a["x"] - p["x"]) > 1e-3 * np.linalg.norm(p["x"])


def torch_net(p, u):
    """The network in float64 with the same bfloat16 roundings (torch ops)."""
    p = torch.as_tensor(np.asarray(p, dtype=np.float64))
    shapes = [(C, 1, 3, 3, 3), (C,), (C, C, 3, 3, 3), (C,), (1, C, 3, 3, 3), (1,)]
    parts, o = [], 0
    for s in shapes:
        k = int(np.prod(s))
        parts.append(p[o:o + k].reshape(s))
        o += k
    W1, b1, W2, b2, W3, b3 = parts
    bf = lambda t: t.to(torch.float32).to(torch.bfloat16).to(torch.float64)
    x = bf(torch.as_tensor(u))[None, None]
    h1 = bf(F.gelu(F.conv3d(x, bf(W1), b1, padding=1)))
    h2 = bf(F.gelu(F.conv3d(h1, bf(W2), b2, padding=1)))
    return F.conv3d(h2, bf(W3), b3, padding=1)[0, 0].numpy()


def test_net_apply_scale_is_rms_of_residual():
    # z = s net(r / s) with s = ||r||_2 / sqrt(N): compare with torch's
    # convolution at that s, and check that s = ||r||_2 (a scale that also
    # makes z(c r) = c z(r)) would be told apart
    nz, ny, nx = 6, 7, 9
    N = nz * ny * nx
    p = P.net_init(3).astype(np.float64)
    p += 0.2 * np.random.default_rng(4).standard_normal(p.size)      # biases too
    r = 5.0 * np.random.default_rng(5).standard_normal(N)
    z = oracle.net_apply(p, r, (nz, ny, nx))
    u = r.reshape(nz, ny, nx)

    def close_fraction(s):
        ref = s * torch_net(p, u / s).reshape(-1)
        return np.mean(np.abs(z - ref) <= 1e-12 * np.abs(ref).max()), np.abs(z - ref).max() / np.abs(ref).max()

    s = np.linalg.norm(r) / np.sqrt(N)
    frac, worst = close_fraction(s)
    # both sides round the same operands to bfloat16; only a sum landing on
    # the other side of a rounding boundary can differ
    assert frac > 0.95 and worst <= 2e-2
    frac_wrong, worst_wrong = close_fraction(np.linalg.norm(r))
    assert frac_wrong < 0.05 and worst_wrong > 0.1


@pytest.mark.parametrize("n,shift", [(8, 0.0), (10, 0.5)])
def test_l1_jacobi_alternate_matches_independent_reference(n, shift):
    """The comparison arm of the learned form: the same schedule with one
    l1-Jacobi sweep from zero, z = r / (a_ii + sum_j |a_ij|), in place of the
    network. The l1 diagonal is formed here from the CSR arrays."""
    rp, c, v = shifted_poisson(n, shift)
    N = n ** 3
    A = sp.csr_matrix((v, c, rp), shape=(N, N))
    rows = np.repeat(np.arange(N), np.diff(rp))
    l1 = np.zeros(N)
    np.add.at(l1, rows, np.abs(v))          # a_ii > 0, so |a_ii| + sum |a_ij|
    h = oracle.Hierarchy(rp, c, v, coarse_max=20)
    b = P.rhs_uniform(N, 2)
    xs, K, fb, ne, events = fcg_learned_reference(A, b, h.vcycle, lambda r: r / l1, 1e-6, 200)
    assert ne >= 1 and "net" in [e for _, e in events]
    full = h.fcg(b, rtol=1e-6, alt_jacobi=True)
    assert full["status"] == oracle.OK
    assert (full["iters"], full["fallbacks"], full["net_evals"]) == (K, fb, ne)
    for k in range(1, K + 1):
        o = h.fcg(b, rtol=1e-6, maxit=k, alt_jacobi=True)
        np.testing.assert_allclose(o["x"], xs[k - 1], rtol=0, atol=1e-12 * np.abs(xs[k - 1]).max())
