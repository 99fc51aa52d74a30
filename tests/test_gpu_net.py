"""GPU parity of the learned preconditioner's kernels against the CPU oracle.

Both sides round the same operands to bfloat16; the GPU accumulates in FP32
(MFMA for the 16 -> 16 layers) and the oracle in FP64, so an activation can
land on the other side of a bfloat16 rounding boundary, which moves that
cell's output by about one bfloat16 step of the activation times its weight.
Tolerances, element by element against max|ref| (see elementwise()): the
99th percentile of |gpu - ref| within 1e-4 max|ref| (flips touched 0.09 -
0.45 % of the cells in measurements, the others agree to FP32 summation
error) and the largest within 2e-3 max|ref| (one flip moved an output by at
most 4.1e-4 max|ref| in measurements); gradients per parameter group 1e-2
relative in norm (measured: at most 8.8e-4, W1, whose gradient sums the
flips of both layers) and 99th percentile 1e-2 element-wise.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle
from paper_2406_19754_amd import problems as P

GROUPS = {"W1": (0, 432), "b1": (432, 448), "W2": (448, 7360), "b2": (7360, 7376), "W3": (7376, 7808), "b3": (7808, 7809)}


@pytest.fixture(scope="module")
def psc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_19754_amd import psc as m
    return m


def params(seed, scale=0.7):
    p = P.net_init(seed).astype(np.float64)
    p += 0.05 * np.random.default_rng(seed + 7).standard_normal(p.size)
    return (p * scale).astype(np.float32)


def relerr(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def elementwise(gpu, ref, what, q_tol=1e-4, max_tol=2e-3):
    """|gpu - ref| against max|ref|: the 99th percentile and the largest."""
    gpu, ref = np.asarray(gpu, np.float64).ravel(), np.asarray(ref, np.float64).ravel()
    scale = np.abs(ref).max()
    d = np.abs(gpu - ref) / scale
    q, m = float(np.quantile(d, 0.99)), float(d.max())
    frac = float(np.mean(d > 1e-4))
    print(f"[net parity] {what}: q99 {q:.1e} max {m:.1e} (x max|ref|), cells beyond 1e-4: {frac:.2%}", flush=True)
    assert q <= q_tol, (what, q)
    assert m <= max_tol, (what, m)


@pytest.mark.parametrize("B,D", [(2, 10), (3, 20), (1, 33)])
def test_forward_batch_matches_oracle(psc, B, D):
    p = params(1)
    u = np.random.default_rng(B * D).standard_normal((B, D, D, D)).astype(np.float32)
    net = psc.Net(p)
    out = torch.empty(B, D, D, D, dtype=torch.float32, device="cuda")
    net.forward_batch(torch.from_numpy(u).cuda(), out)
    ref = oracle.net_forward(p.astype(np.float64), u.astype(np.float64), round_bf16=True)
    elementwise(out.cpu().numpy(), ref, f"forward B={B} D={D}")


def test_loss_and_gradients_match_oracle(psc):
    p = params(2)
    rng = np.random.default_rng(3)
    B, D, margin = 2, 12, 2
    u = rng.standard_normal((B, D, D, D)).astype(np.float32)
    y = rng.standard_normal((B, D, D, D)).astype(np.float32)
    net = psc.Net(p)
    loss, g = net.loss_grad(torch.from_numpy(u).cuda(), torch.from_numpy(y).cuda(), margin)
    lref, gref = oracle.net_loss_grad(p.astype(np.float64), u.astype(np.float64), y.astype(np.float64), margin,
                                      round_bf16=True)
    assert abs(loss - lref) <= 1e-3 * lref
    for name, (a, b) in GROUPS.items():
        e = relerr(g[a:b], gref[a:b])
        print(f"[net parity] gradient {name}: relative error {e:.1e}", flush=True)
        assert e <= 1e-2, name
        if b - a > 1:
            elementwise(g[a:b], gref[a:b], f"gradient {name}", q_tol=1e-2, max_tol=2e-2)


def test_adam_step_and_training_lowers_loss(psc):
    p = params(4)
    rng = np.random.default_rng(5)
    ncrops, D, margin = 8, 12, 2
    r = rng.standard_normal((ncrops, D, D, D)).astype(np.float32)
    z = (0.3 * r).astype(np.float32)            # a learnable target: a scaled identity
    rd, zd = torch.from_numpy(r).cuda(), torch.from_numpy(z).cuda()
    net = psc.Net(p)
    order = np.array([0, 1], np.int32)
    _, g = net.loss_grad(rd[:2].contiguous(), zd[:2].contiguous(), margin)
    net.train(rd, zd, order, steps=1, batch=2, margin=margin, lr=1e-3)
    p1 = net.params()
    ref, _, _ = oracle.adam_step(p.astype(np.float64), np.zeros(p.size), np.zeros(p.size), g.astype(np.float64), 1, lr=1e-3)
    np.testing.assert_allclose(p1, ref, rtol=0, atol=2e-6)
    order = np.random.default_rng(6).integers(0, ncrops, 2 * 60).astype(np.int32)
    losses = net.train(rd, zd, order, steps=60, batch=2, margin=margin, lr=3e-3)
    assert np.mean(losses[-10:]) < 0.5 * np.mean(losses[:5])


def test_net_apply_matches_oracle(psc):
    p = params(8)
    dims = (9, 10, 12)                              # (nz, ny, nx), not cubic
    N = int(np.prod(dims))
    r = np.random.default_rng(9).standard_normal(N)
    net = psc.Net(p)
    z = torch.empty(N, dtype=torch.float64, device="cuda")
    net.apply(torch.from_numpy(r).cuda(), z, dims)
    ref = oracle.net_apply(p.astype(np.float64), r, dims)
    elementwise(z.cpu().numpy(), ref, "apply 9x10x12")


@pytest.mark.parametrize("dims", [(9, 10, 12), (40, 33, 35), (17, 48, 16)])
def test_fused_and_unfused_apply_match_oracle(psc, dims):
    """Both inference paths (psc_net_tune) against the oracle and each other.
    (40, 33, 35) cuts z into 5 chunks of 8 planes with ragged 16-wide x and y
    tiles; (17, 48, 16) has whole tiles in x and three in y."""
    p = params(21)
    N = int(np.prod(dims))
    r = np.random.default_rng(22).standard_normal(N)
    ref = oracle.net_apply(p.astype(np.float64), r, dims)
    net = psc.Net(p)
    rd = torch.from_numpy(r).cuda()
    out = {}
    for fused in (1, 0, 1):
        net.tune(psc.NET_TUNE_FUSED, fused)
        z = torch.full_like(rd, float("nan"))
        net.apply(rd, z, dims)
        out[fused] = z.cpu().numpy()
        elementwise(out[fused], ref, f"apply {dims} fused={fused}")
    elementwise(out[1], out[0], f"fused vs unfused {dims}")


def test_fused_apply_sampled_at_128(psc):
    """The fused kernel on the learned form's 128^3 grid, checked at 256 cells
    (corners, faces and interior) against the oracle on the part of the 7^3
    neighbourhood each output depends on that lies in the grid (the oracle's
    zero padding then falls where the grid's does), with s = ||r|| / sqrt(N)."""
    n = 128
    dims, N = (n, n, n), n ** 3
    p = params(23)
    rng = np.random.default_rng(24)
    r = rng.standard_normal(N)
    net = psc.Net(p)
    rd = torch.from_numpy(r).cuda()
    z = torch.full_like(rd, float("nan"))
    net.apply(rd, z, dims)
    zg = z.cpu().numpy().reshape(dims)
    assert np.isfinite(zg).all()
    s = np.linalg.norm(r) / np.sqrt(N)
    u = (r / s).reshape(dims)
    cells = [(0, 0, 0), (n - 1, n - 1, n - 1), (0, n - 1, 5), (n - 1, 0, 64), (3, 2, 1)]
    cells += [tuple(c) for c in rng.integers(0, n, (251, 3))]
    ref = []
    for c in cells:
        lo = [max(0, a - 3) for a in c]
        hi = [min(n, a + 4) for a in c]
        crop = u[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]]
        out = oracle.net_forward(p.astype(np.float64), crop[None], round_bf16=True)[0]
        ref.append(out[c[0] - lo[0], c[1] - lo[1], c[2] - lo[2]] * s)
    ref = np.array(ref)
    gpu = np.array([zg[c] for c in cells])
    elementwise(gpu, ref, "fused apply 128^3, 256 sampled cells", q_tol=2e-3)


def test_zero_network_falls_back_to_vcycle(psc):
    n = 16
    rp, c, v = P.poisson7(n)
    h = psc.Hierarchy(rp, c, v)
    net = psc.Net(np.zeros(psc.net_param_count(), np.float32))
    net.set_grid((n, n, n))
    b = torch.from_numpy(P.rhs_uniform(n ** 3, 1)).cuda()
    x = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
    g = h.fcg(b, x, net=net)
    x2 = torch.zeros_like(x)
    g0 = h.fcg(b, x2)
    assert g["status"] == psc.OK and g["relres"] <= 1e-6 and g["fallbacks"] >= 1
    # every scheduled network step counts: the two that failed z.r > 0 and,
    # once that switched the network off, the rest
    assert g["fallbacks"] == g["iters"] // 2
    assert g["iters"] == g0["iters"]
    assert torch.equal(x, x2)


def identity_like_net(a, c):
    """Each cell alone (centre taps): out = c (G(G(a u)) - G(G(-a u))), G = GELU,
    an odd increasing map of u, so z.r > 0 for every r != 0: every scheduled
    network step is taken, and on Poisson each cuts ||r|| by more than 10 %."""
    C = 16
    W1, W2, W3 = np.zeros((C, 1, 27)), np.zeros((C, C, 27)), np.zeros((1, C, 27))
    W1[0, 0, 13], W1[1, 0, 13] = a, -a
    W2[0, 0, 13] = W2[1, 1, 13] = 1.0
    W3[0, 0, 13], W3[0, 1, 13] = c, -c
    return np.concatenate([W1.ravel(), np.zeros(C), W2.ravel(), np.zeros(C), W3.ravel(), [0.0]]).astype(np.float32)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_learned_fcg_accepted_steps_match_oracle(psc, prec):
    """Every network step accepted (no fallback): iterations within one of the
    oracle's, and the solutions after the same number of iterations agree."""
    n = 16
    rp, c, v = P.poisson7(n)
    p = identity_like_net(4.0, 1.0)
    pr, form = (psc.FP32, 1) if prec == "fp32" else (psc.FP64, 0)
    h = psc.Hierarchy(rp, c, v, build_fp32=True)
    o = oracle.Hierarchy(rp, c, v)
    net = psc.Net(p)
    net.set_grid((n, n, n))
    b = P.rhs_uniform(n ** 3, 12)
    bd = torch.from_numpy(b).cuda()
    x = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
    g = h.fcg(bd, x, net=net, prec=pr)
    r = o.fcg(b, params=p.astype(np.float64), dims=(n, n, n), form=form)
    assert g["status"] == psc.OK and r["status"] == oracle.OK and g["relres"] <= 1e-6
    assert g["fallbacks"] == 0 and r["fallbacks"] == 0 and r["net_evals"] == r["iters"] // 2 > 0
    assert abs(g["iters"] - r["iters"]) <= 1
    k = min(g["iters"], r["iters"]) - 1
    x.zero_()
    h.fcg(bd, x, rtol=1e-30, maxit=k, net=net, prec=pr)
    ref = o.fcg(b, rtol=1e-30, maxit=k, params=p.astype(np.float64), dims=(n, n, n), form=form)["x"]
    err = np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref)
    print(f"[net parity] learned FCG ({prec}) after {k} iterations: |x_gpu - x_orc|/|x_orc| = {err:.1e}", flush=True)
    assert err <= 1e-6


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_l1_jacobi_alternate_matches_oracle(psc, prec):
    """The learned schedule's comparison arm (z = M_0^-1 r in place of the
    network): same iterations and accounting as the oracle, iterates equal."""
    n = 20
    rp, c, v = P.poisson7(n)
    pr, form = (psc.FP32, 1) if prec == "fp32" else (psc.FP64, 0)
    h = psc.Hierarchy(rp, c, v, build_fp32=True)
    o = oracle.Hierarchy(rp, c, v)
    jac = psc.Net.l1jacobi(h)
    b = P.rhs_uniform(n ** 3, 14)
    bd = torch.from_numpy(b).cuda()
    x = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
    g = h.fcg(bd, x, net=jac, prec=pr)
    r = o.fcg(b, form=form, alt_jacobi=True)
    assert g["status"] == psc.OK and r["status"] == oracle.OK and g["relres"] <= 1e-6
    assert r["net_evals"] >= 1
    assert g["iters"] == r["iters"] and g["fallbacks"] == r["fallbacks"]
    ref = r["x"]
    tol = 1e-8 if prec == "fp64" else 1e-6
    assert np.linalg.norm(x.cpu().numpy() - ref) <= tol * np.linalg.norm(ref)
    # the arm has no weights
    with pytest.raises(psc.PscError):
        jac.params()


def test_learned_fcg_matches_oracle(psc):
    n = 16
    rp, c, v = P.poisson7(n)
    p = params(11, scale=0.3)
    h = psc.Hierarchy(rp, c, v)
    o = oracle.Hierarchy(rp, c, v)
    net = psc.Net(p)
    net.set_grid((n, n, n))
    b = P.rhs_uniform(n ** 3, 12)
    x = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
    g = h.fcg(torch.from_numpy(b).cuda(), x, net=net)
    r = o.fcg(b, params=p.astype(np.float64), dims=(n, n, n))
    assert g["status"] == psc.OK and r["status"] == oracle.OK
    assert g["relres"] <= 1e-6
    assert abs(g["iters"] - r["iters"]) <= 2
    # graph replay and stream launch give the same iterates
    h2 = psc.Hierarchy(rp, c, v, use_graph=False)
    x2 = torch.zeros_like(x)
    g2 = h2.fcg(torch.from_numpy(b).cuda(), x2, net=net)
    assert g2["iters"] == g["iters"] and torch.equal(x, x2)


def test_pairs_collect_first_pair_matches_oracle(psc):
    n, crop, cpi = 16, 8, 2
    rp, c, v = P.poisson7(n)
    h = psc.Hierarchy(rp, c, v)
    o = oracle.Hierarchy(rp, c, v)
    b = P.rhs_uniform(n ** 3, 21)
    origins = P.crop_origins(22, 200, (n, n, n), crop)
    cap = 64
    rout = torch.zeros(cap, crop, crop, crop, dtype=torch.float32, device="cuda")
    zout = torch.zeros_like(rout)
    cnt = psc.pairs_collect(h, torch.from_numpy(b).cuda(), (n, n, n), crop, cpi, origins, rout, zout)
    iters = o.pcg(b)["iters"]
    assert cnt == cpi * iters                       # pairs (r_k, B r_k), k = 0 .. iters-1
    s0 = np.linalg.norm(b) / np.sqrt(n ** 3)
    z0 = o.vcycle(b)
    for k in range(cpi):
        oz, oy, ox = origins[k]
        sl = (slice(oz, oz + crop), slice(oy, oy + crop), slice(ox, ox + crop))
        np.testing.assert_allclose(rout[k].cpu().numpy(), (b.reshape(n, n, n)[sl] / s0).astype(np.float32),
                                   rtol=1e-6, atol=1e-6)
        np.testing.assert_allclose(zout[k].cpu().numpy(), (z0.reshape(n, n, n)[sl] / s0), rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_learned_fused_unfused_and_switch_off(psc, prec):
    # A network that fails the progress test gets switched off for the rest of
    # the solve; the host then replays iterations without its kernels. The
    # fused and the one-kernel-per-operation learned iterations agree, and
    # graph replay equals stream launch bit for bit.
    n = 16
    rp, c, v = P.poisson7(n)
    pr = psc.FP32 if prec == "fp32" else psc.FP64
    net = psc.Net(params(5, scale=0.5))
    net.set_grid((n, n, n))
    b = torch.from_numpy(P.rhs_uniform(n ** 3, 3)).cuda()
    res = {}
    for fused in (1, 0):
        for graph in (True, False):
            h = psc.Hierarchy(rp, c, v, build_fp32=True, use_graph=graph)
            h.tune(psc.TUNE_FUSED_PCG, fused)
            x = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
            g = h.fcg(b, x, net=net, prec=pr)
            assert g["status"] == psc.OK and g["relres"] <= 1e-6
            res[(fused, graph)] = (g, x.clone())
    for fused in (1, 0):
        (ga, xa), (gb, xb) = res[(fused, True)], res[(fused, False)]
        assert ga["iters"] == gb["iters"] and ga["fallbacks"] == gb["fallbacks"] and torch.equal(xa, xb)
    assert abs(res[(1, True)][0]["iters"] - res[(0, True)][0]["iters"]) <= 1
    # scheduled network steps that ran the V-cycle are counted (also after the switch)
    assert res[(1, True)][0]["fallbacks"] >= 1


def test_save_load_round_trip_resumes_training(psc, tmp_path):
    """psc_net_save / psc_net_load: weights and Adam state survive the file;
    the loaded handle applies identically and its next training steps equal
    those of the handle that kept running."""
    p = params(8)
    rng = np.random.default_rng(9)
    ncrops, D, margin = 6, 12, 2
    r = torch.from_numpy(rng.standard_normal((ncrops, D, D, D)).astype(np.float32)).cuda()
    z = torch.from_numpy(rng.standard_normal((ncrops, D, D, D)).astype(np.float32)).cuda()
    net = psc.Net(p)
    net.train(r, z, np.arange(6, dtype=np.int32), steps=3, batch=2, margin=margin, lr=1e-3)
    path = str(tmp_path / "net.ckpt")
    net.save(path)
    assert os.path.getsize(path) == 40 + 3 * 4 * psc.net_param_count()
    net2 = psc.Net.load(path)
    np.testing.assert_array_equal(net2.params(), net.params())
    n = 20
    rv = torch.from_numpy(rng.standard_normal(n ** 3)).cuda()
    z1, z2 = torch.empty_like(rv), torch.empty_like(rv)
    net.apply(rv, z1, (n, n, n))
    net2.apply(rv, z2, (n, n, n))
    assert torch.equal(z1, z2)
    order = np.array([5, 1, 4, 0], np.int32)
    l1 = net.train(r, z, order, steps=2, batch=2, margin=margin, lr=1e-3)
    l2 = net2.train(r, z, order, steps=2, batch=2, margin=margin, lr=1e-3)
    np.testing.assert_array_equal(l1, l2)
    np.testing.assert_array_equal(net2.params(), net.params())
    # a fresh handle with the same weights but no Adam state takes a different step
    net3 = psc.Net(np.fromfile(path, dtype=np.float32, count=psc.net_param_count(), offset=40))
    net3.train(r, z, order, steps=2, batch=2, margin=margin, lr=1e-3)
    assert not np.array_equal(net3.params(), net.params())
