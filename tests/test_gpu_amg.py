"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Sizes are ones the oracle finishes in seconds but that still span many
64-row slices, several levels and a ragged last slice. Tolerances:
  * SpMV and the FP64 V-cycle: 1e-12 relative (FMA and summation order only);
  * FP32 V-cycle: 1e-5 relative to the oracle's FP32 V-cycle;
  * full solves: iteration counts within +-1 and, at equal iteration count,
    ||x_gpu - x_orc|| / ||x_orc|| <= 1e-8 (FP64), true residual <= rtol.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle
from paper_2406_19754_amd import problems as P


@pytest.fixture(scope="module")
def psc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_19754_amd import psc as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


CASES = {
    "poisson32": lambda: P.poisson7(32),
    "poisson13": lambda: P.poisson7(13),                      # odd size: singletons, ragged slices
    "diffusion20_az100": lambda: P.diffusion7(20, seed=0, az=100.0),
    "random_long_rows": lambda: P.random_spd_csr(700, 5, density=0.01, maxrow=90),
    # coarsening stalls above 2000 rows: coarsest solved by 30 l1-Jacobi sweeps
    "diffusion48_lognormal": lambda: P.diffusion7(48, seed=0),
}


@pytest.mark.parametrize("case", list(CASES))
def test_hierarchy_matches_oracle(psc, case):
    rp, c, v = CASES[case]()
    cm = 40 if case == "random_long_rows" else 200
    h = psc.Hierarchy(rp, c, v, coarse_max=cm)
    o = oracle.Hierarchy(rp, c, v, coarse_max=cm)
    inf = h.info()
    assert inf["rows"] == o.sizes()
    for l in range(inf["levels"]):
        a, b = h.export_level(l), o.level(l)
        assert np.array_equal(a["col"], b["col"]) and np.array_equal(a["rowptr"], b["rowptr"])
        np.testing.assert_allclose(a["val"], b["val"], rtol=1e-13, atol=0)
        if l < inf["levels"] - 1:
            assert np.array_equal(a["agg"], b["agg"])


@pytest.mark.parametrize("case", list(CASES))
def test_spmv_matches_oracle(psc, case):
    rp, c, v = CASES[case]()
    h = psc.Hierarchy(rp, c, v, build_fp32=True, coarse_max=40)
    x = np.random.default_rng(1).standard_normal(len(rp) - 1)
    ref = oracle.spmv(rp, c, v, x)
    y = torch.empty(len(x), dtype=torch.float64, device="cuda")
    h.spmv(dev(x), y)
    got = y.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    # FP32 copy on the same operator
    y32 = torch.empty(len(x), dtype=torch.float32, device="cuda")
    h.spmv(dev(x.astype(np.float32)), y32, prec=psc.FP32)
    ref32 = oracle.spmv(rp, c, v.astype(np.float32).astype(np.float64), x.astype(np.float32).astype(np.float64))
    assert np.abs(y32.cpu().numpy() - ref32).max() <= 1e-5 * np.abs(ref32).max()
    # every level's operator
    o = oracle.Hierarchy(rp, c, v, coarse_max=40)
    for l in range(1, o.nlevels):
        L = o.level(l)
        xl = np.random.default_rng(l).standard_normal(L["n"])
        yl = torch.empty(L["n"], dtype=torch.float64, device="cuda")
        h.spmv(dev(xl), yl, level=l)
        refl = oracle.spmv(L["rowptr"], L["col"], L["val"], xl)
        assert np.abs(yl.cpu().numpy() - refl).max() <= 1e-13 * np.abs(refl).max()


@pytest.mark.parametrize("case", ["diffusion48_lognormal", "random_long_rows"])
def test_capped_layout_matches_plain_and_oracle(psc, case):
    """Levels whose row lengths vary widely (a few long rows in most slices)
    are read from a capped hacked-ELL copy, the long rows' remaining entries in
    overflow records that one wavefront sums: SpMV on those levels, the V-cycle
    and PCG agree with the plain layout up to rounding and with the oracle."""
    rp, c, v = CASES[case]()
    cm = 40 if case == "random_long_rows" else 200
    # small operators: every level where a cap pays gets the copy
    h = psc.Hierarchy(rp, c, v, build_fp32=True, coarse_max=cm, capped_min_rows=1)
    o = oracle.Hierarchy(rp, c, v, coarse_max=cm)
    inf = h.info()
    capped = [l for l in range(inf["levels"]) if inf["capped_cap"][l] > 0]
    assert capped, "the case has no level with a capped copy"
    assert psc.Hierarchy(rp, c, v, coarse_max=cm).info()["capped_cap"] == [0] * inf["levels"]
    for l in capped:
        # the copy stores fewer slots than the plain slices (overflow included)
        assert inf["capped_slots"][l] < inf["ell_slots"][l]
        L = o.level(l)
        xl = np.random.default_rng(10 + l).standard_normal(L["n"])
        yl = torch.empty(L["n"], dtype=torch.float64, device="cuda")
        h.spmv(dev(xl), yl, level=l)
        refl = oracle.spmv(L["rowptr"], L["col"], L["val"], xl)
        scale = oracle.spmv(L["rowptr"], L["col"], np.abs(L["val"]), np.abs(xl))
        assert np.all(np.abs(yl.cpu().numpy() - refl) <= 1e-14 * scale + 1e-300)
        y32 = torch.empty(L["n"], dtype=torch.float32, device="cuda")
        h.spmv(dev(xl.astype(np.float32)), y32, level=l, prec=psc.FP32)
        assert np.all(np.abs(y32.cpu().numpy() - refl) <= 1e-5 * scale + 1e-30)
    n = len(rp) - 1
    r = np.random.default_rng(3).standard_normal(n)
    zc = torch.empty(n, dtype=torch.float64, device="cuda")
    zp = torch.empty(n, dtype=torch.float64, device="cuda")
    h.vcycle(dev(r), zc)
    h.tune(psc.TUNE_CAPPED, 0)
    h.vcycle(dev(r), zp)
    h.tune(psc.TUNE_CAPPED, 1)
    zc, zp = zc.cpu().numpy(), zp.cpu().numpy()
    assert np.linalg.norm(zc - zp) <= 1e-13 * np.linalg.norm(zp)
    ref = o.vcycle(r)
    assert np.linalg.norm(zc - ref) <= 1e-12 * np.linalg.norm(ref)
    z32 = torch.empty(n, dtype=torch.float64, device="cuda")
    h.vcycle(dev(r), z32, prec=psc.FP32)
    ref32 = o.vcycle32(r)
    assert np.linalg.norm(z32.cpu().numpy() - ref32) <= 1e-5 * np.linalg.norm(ref32)
    b = np.random.default_rng(4).standard_normal(n)
    xs = []
    for on in (1, 0):
        h.tune(psc.TUNE_CAPPED, on)
        x = torch.zeros(n, dtype=torch.float64, device="cuda")
        g = h.pcg(dev(b), x, rtol=1e-6, maxit=500)
        xs.append((g["iters"], x.cpu().numpy()))
    h.tune(psc.TUNE_CAPPED, 1)
    r_o = o.pcg(b, rtol=1e-6, maxit=500)
    assert xs[0][0] == xs[1][0] and abs(xs[0][0] - r_o["iters"]) <= 1
    assert np.linalg.norm(xs[0][1] - xs[1][1]) <= 1e-10 * np.linalg.norm(xs[1][1])


def test_pair_restriction_matches_plain_and_oracle(psc):
    """On levels whose rows 2k and 2k+1 share an aggregate and a prolongator
    value (Poisson's 2x2x1 aggregates), the pre-smoothing pass also writes the
    pair sums and the restriction reads them: the V-cycle in both precisions
    and the fused PCG / FCG(1) solves agree with the plain restriction up to
    rounding, and the V-cycle with the oracle."""
    rp, c, v = P.poisson7(32)
    h = psc.Hierarchy(rp, c, v, build_fp32=True)
    inf = h.info()
    assert inf["pair_restrict"][:2] == [1, 1]
    # odd row counts are never eligible
    assert psc.Hierarchy(*P.poisson7(13)).info()["pair_restrict"][0] == 0
    n = len(rp) - 1
    r = np.random.default_rng(5).standard_normal(n)
    out = {}
    for on in (1, 0):
        h.tune(psc.TUNE_PAIR_R, on)
        assert h.info()["pair_restrict"][0] == on
        for prec in (psc.FP64, psc.FP32):
            z = torch.empty(n, dtype=torch.float64, device="cuda")
            h.vcycle(dev(r), z, prec=prec)
            out[(on, prec)] = z.cpu().numpy()
        b = np.random.default_rng(6).standard_normal(n)
        for form in ("pcg", "fcg64", "fcg32"):
            x = torch.zeros(n, dtype=torch.float64, device="cuda")
            if form == "pcg":
                g = h.pcg(dev(b), x, rtol=1e-6, maxit=200)
            else:
                g = h.fcg(dev(b), x, rtol=1e-6, maxit=200, prec=psc.FP32 if form == "fcg32" else psc.FP64)
            out[(on, form)] = (g["iters"], x.cpu().numpy())
    h.tune(psc.TUNE_PAIR_R, 1)
    ref = oracle.Hierarchy(rp, c, v).vcycle(r)
    for on in (1, 0):
        assert np.linalg.norm(out[(on, psc.FP64)] - ref) <= 1e-12 * np.linalg.norm(ref)
    assert np.linalg.norm(out[(1, psc.FP64)] - out[(0, psc.FP64)]) <= 1e-14 * np.linalg.norm(ref)
    assert np.linalg.norm(out[(1, psc.FP32)] - out[(0, psc.FP32)]) <= 1e-6 * np.linalg.norm(ref)
    for form in ("pcg", "fcg64", "fcg32"):
        (i1, x1), (i0, x0) = out[(1, form)], out[(0, form)]
        assert i1 == i0
        assert np.linalg.norm(x1 - x0) <= 1e-9 * np.linalg.norm(x0)


@pytest.mark.parametrize("n", [32, 33])
def test_mixed_form_fp32_z_is_bit_identical(psc, n):
    """The mixed form keeps the FP32 V-cycle's output z in FP32 (the
    precision it is computed in) and the outer pass widens it: iterates,
    iteration count and residual are bit for bit those of the FP64 copy."""
    rp, c, v = P.poisson7(n)
    h = psc.Hierarchy(rp, c, v, build_fp32=True)
    b = np.random.default_rng(7).standard_normal(len(rp) - 1)
    out = []
    for on in (1, 0):
        h.tune(psc.TUNE_MIXED_Z32, on)
        x = torch.zeros(len(b), dtype=torch.float64, device="cuda")
        g = h.fcg(dev(b), x, rtol=1e-8, maxit=200, prec=psc.FP32)
        out.append((g["iters"], g["relres"], x.cpu().numpy()))
    h.tune(psc.TUNE_MIXED_Z32, 1)
    assert out[0][0] == out[1][0] and out[0][1] == out[1][1]
    assert np.array_equal(out[0][2], out[1][2])


@pytest.mark.parametrize("case", list(CASES))
def test_vcycle_matches_oracle(psc, case):
    rp, c, v = CASES[case]()
    h = psc.Hierarchy(rp, c, v, build_fp32=True)
    o = oracle.Hierarchy(rp, c, v)
    r = np.random.default_rng(2).standard_normal(len(rp) - 1)
    z = torch.empty(len(r), dtype=torch.float64, device="cuda")
    h.vcycle(dev(r), z)
    ref = o.vcycle(r)
    assert np.linalg.norm(z.cpu().numpy() - ref) <= 1e-12 * np.linalg.norm(ref)
    h.vcycle(dev(r), z, prec=psc.FP32)
    ref32 = o.vcycle32(r)
    assert np.linalg.norm(z.cpu().numpy() - ref32) <= 1e-5 * np.linalg.norm(ref32)
    assert np.linalg.norm(z.cpu().numpy() - ref) <= 1e-4 * np.linalg.norm(ref)


@pytest.mark.parametrize("K", [1, 2, 7])
def test_jacobi_coarsest_sweep_counts_match_oracle(psc, K):
    rp, c, v = P.diffusion7(48, seed=0)
    h = psc.Hierarchy(rp, c, v, build_fp32=True, coarse_sweeps=K)
    o = oracle.Hierarchy(rp, c, v, coarse_sweeps=K)
    assert h.info()["coarse_sweeps"] == K == o.coarse_sweeps
    r = np.random.default_rng(K).standard_normal(len(rp) - 1)
    z = torch.empty(len(r), dtype=torch.float64, device="cuda")
    h.vcycle(dev(r), z)
    ref = o.vcycle(r)
    assert np.linalg.norm(z.cpu().numpy() - ref) <= 1e-12 * np.linalg.norm(ref)
    h.vcycle(dev(r), z, prec=psc.FP32)
    ref32 = o.vcycle32(r)
    assert np.linalg.norm(z.cpu().numpy() - ref32) <= 1e-5 * np.linalg.norm(ref32)


def _solve_pair(psc, rp, c, v, b, form, maxit=1000, use_graph=True):
    h = psc.Hierarchy(rp, c, v, build_fp32=True, use_graph=use_graph)
    o = oracle.Hierarchy(rp, c, v)
    x = torch.zeros(len(b), dtype=torch.float64, device="cuda")
    if form == "pcg":
        g = h.pcg(dev(b), x, rtol=1e-6, maxit=maxit)
        r = o.pcg(b, rtol=1e-6, maxit=maxit)
    else:
        prec = psc.FP32 if form == "fcg32" else psc.FP64
        g = h.fcg(dev(b), x, rtol=1e-6, maxit=maxit, prec=prec)
        r = o.fcg(b, rtol=1e-6, maxit=maxit, form=1 if form == "fcg32" else 0)
    return h, o, g, x.cpu().numpy(), r


@pytest.mark.parametrize("form", ["pcg", "fcg64", "fcg32"])
@pytest.mark.parametrize("case", ["poisson32", "diffusion20_az100", "diffusion48_lognormal"])
def test_solve_matches_oracle(psc, case, form):
    rp, c, v = CASES[case]()
    b = P.rhs_from_solution(rp, c, v, P.x_true(len(rp) - 1, 0))
    h, o, g, xg, r = _solve_pair(psc, rp, c, v, b, form)
    assert g["status"] == psc.OK and r["status"] == oracle.OK
    assert abs(g["iters"] - r["iters"]) <= 1
    assert g["relres"] <= 1e-6
    k = min(g["iters"], r["iters"])
    if form == "fcg32":
        # FP32 V-cycle: checked by the true FP64 residual; the error to the
        # FP64 oracle solution is stated, not bounded tightly
        assert np.linalg.norm(xg - r["x"]) <= 1e-4 * np.linalg.norm(r["x"])
        return
    # equal iteration count comparison
    x = torch.zeros(len(b), dtype=torch.float64, device="cuda")
    if form == "pcg":
        h.pcg(dev(b), x, rtol=1e-30, maxit=k)
        ref = o.pcg(b, rtol=1e-30, maxit=k)["x"]
    else:
        h.fcg(dev(b), x, rtol=1e-30, maxit=k)
        ref = o.fcg(b, rtol=1e-30, maxit=k, form=0)["x"]
    assert np.linalg.norm(x.cpu().numpy() - ref) <= 1e-8 * np.linalg.norm(ref)


def test_graph_and_stream_launch_agree_bitwise(psc):
    rp, c, v = P.poisson7(24)
    b = P.rhs_uniform(24 ** 3, 3)
    xs = []
    for use_graph in (True, False, True):
        h = psc.Hierarchy(rp, c, v, use_graph=use_graph)
        x = torch.zeros(len(b), dtype=torch.float64, device="cuda")
        g = h.pcg(dev(b), x)
        xs.append((g["iters"], x.cpu().numpy()))
    assert xs[0][0] == xs[1][0] == xs[2][0]
    assert np.array_equal(xs[0][1], xs[1][1]) and np.array_equal(xs[0][1], xs[2][1])


def test_repeated_solves_reuse_hierarchy(psc):
    rp, c, v = P.poisson7(20)
    h = psc.Hierarchy(rp, c, v, build_fp32=True)
    o = oracle.Hierarchy(rp, c, v)
    for seed in range(3):
        b = P.rhs_uniform(20 ** 3, seed)
        for fn in ("pcg", "fcg"):
            x = torch.zeros(len(b), dtype=torch.float64, device="cuda")
            g = getattr(h, fn)(dev(b), x)
            r = o.pcg(b) if fn == "pcg" else o.fcg(b)
            assert abs(g["iters"] - r["iters"]) <= 1 and g["relres"] <= 1e-6


def test_single_level_and_initial_guess(psc):
    rp, c, v = P.poisson7(5)                     # 125 rows: the coarsest level is level 0
    h = psc.Hierarchy(rp, c, v)
    assert h.info()["levels"] == 1
    b = P.rhs_uniform(125, 1)
    x = torch.zeros(125, dtype=torch.float64, device="cuda")
    g = h.pcg(dev(b), x, rtol=1e-10)
    assert g["iters"] == 1 and g["relres"] <= 1e-12
    # a converged initial guess takes zero iterations
    g2 = h.pcg(dev(b), x, rtol=1e-6)
    assert g2["iters"] == 0 and g2["status"] == psc.OK


def test_failure_paths(psc):
    rp, c, v = P.poisson7(12)
    h = psc.Hierarchy(rp, c, v)
    n = 12 ** 3
    x = torch.full((n,), 5.0, dtype=torch.float64, device="cuda")
    g = h.pcg(torch.zeros(n, dtype=torch.float64, device="cuda"), x)
    assert g["iters"] == 0 and g["status"] == psc.OK and not x.any()
    b = P.rhs_uniform(n, 0)
    x.zero_()
    g = h.pcg(dev(b), x, rtol=1e-12, maxit=1)
    assert g["status"] == psc.NOCONV and g["iters"] == 1 and 0 < g["relres"] < 1
    bn = b.copy()
    bn[7] = np.nan
    with pytest.raises(psc.PscError) as e:
        h.pcg(dev(bn), x)
    assert e.value.status == psc.ERR_NAN
    with pytest.raises(psc.PscError) as e:
        h.fcg(dev(b), x, prec=psc.FP32)              # FP32 copies were not built
    assert e.value.status == psc.ERR_STATE
    v2 = v.copy()
    v2[rp[3] + list(c[rp[3]:rp[4]]).index(3)] = -6.0
    with pytest.raises(psc.PscError) as e:
        psc.Hierarchy(rp, c, v2)
    assert e.value.status == psc.ERR_NOT_SPD
    c2 = c.copy()
    c2[1], c2[0] = c[0], c[1]                       # unsorted row
    with pytest.raises(psc.PscError) as e:
        psc.Hierarchy(rp, c2, v)
    assert e.value.status == psc.ERR_ARG


@pytest.mark.parametrize("form", ["pcg", "fcg64", "fcg32"])
@pytest.mark.parametrize("case", ["poisson32", "diffusion20_az100", "random_long_rows"])
def test_fused_and_unfused_iterations_agree(psc, case, form):
    rp, c, v = CASES[case]()
    cm = 40 if case == "random_long_rows" else 200
    b = P.rhs_from_solution(rp, c, v, P.x_true(len(rp) - 1, 1))
    out = []
    for fused in (1, 0):
        h = psc.Hierarchy(rp, c, v, coarse_max=cm, build_fp32=True)
        h.tune(psc.TUNE_FUSED_PCG, fused)
        x = torch.zeros(len(b), dtype=torch.float64, device="cuda")
        if form == "pcg":
            g = h.pcg(dev(b), x)
        else:
            g = h.fcg(dev(b), x, prec=psc.FP32 if form == "fcg32" else psc.FP64)
        out.append((g, x.cpu().numpy()))
    (g1, x1), (g0, x0) = out
    assert g1["status"] == g0["status"] == psc.OK
    assert g1["iters"] == g0["iters"] and g1["relres"] <= 1e-6
    assert np.linalg.norm(x1 - x0) <= 1e-10 * np.linalg.norm(x0)


@pytest.mark.parametrize("n", [64, 48])
def test_plane_aligned_grid_gives_the_same_iterates(psc, n):
    """The level grids (at least one 128-row block per wavefront; at 64^3 the
    blocks per workgroup also divide a z-plane's blocks over the 8 dies, at
    48^3 a plane of 2304 rows cannot be aligned) change only how the
    reductions' partial sums are grouped: the same iterations as with the
    alignment off and with the old workgroup cap, x to 1e-12, and the
    oracle's iteration count within one."""
    rp, c, v = P.poisson7(n)
    b = P.rhs_from_solution(rp, c, v, P.x_true(n ** 3, 0))
    h = psc.Hierarchy(rp, c, v, build_fp32=True)
    out = {}
    for key, align, gmax in (("aligned", 1, 131072), ("unaligned", 0, 131072), ("cap65536", 1, 65536)):
        h.tune(psc.TUNE_DIA_ALIGN, align)
        h.tune(psc.TUNE_GRID_MAX, gmax)
        for form in ("pcg", "fcg32"):
            x = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
            g = h.pcg(dev(b), x) if form == "pcg" else h.fcg(dev(b), x, prec=psc.FP32)
            assert g["status"] == psc.OK and g["relres"] <= 1e-6
            out[key, form] = (g["iters"], x.cpu().numpy())
    h.tune(psc.TUNE_DIA_ALIGN, 1)
    h.tune(psc.TUNE_GRID_MAX, 131072)
    for form in ("pcg", "fcg32"):
        it0, x0 = out["aligned", form]
        for key in ("unaligned", "cap65536"):
            it, xk = out[key, form]
            assert it == it0, (key, form)
            assert np.linalg.norm(xk - x0) <= 1e-12 * np.linalg.norm(x0), (key, form)
    ref = oracle.Hierarchy(rp, c, v).pcg(b)
    assert abs(out["aligned", "pcg"][0] - ref["iters"]) <= 1


@pytest.mark.parametrize("knob", ["tail_off", "tail_4096", "dia_off", "split_off", "bufload_all", "bufload_none", "unroll4", "grid256",
                                  "spmv2", "dia_per_slice", "xcd_chunks", "mixed_fused"])
@pytest.mark.parametrize("case", ["poisson13", "random_long_rows", "diffusion20_az100"])
def test_kernel_variants_match_oracle(psc, case, knob):
    rp, c, v = CASES[case]()
    cm = 40 if case == "random_long_rows" else 200
    h = psc.Hierarchy(rp, c, v, coarse_max=cm, build_fp32=True)
    dia = h.info()["dia_slots"]
    if case == "random_long_rows":
        assert dia[0] == 0                           # no diagonal structure: ELL only
    else:
        assert dia[0] > 0                            # a 7-point stencil keeps a hacked-DIA copy
    if knob == "dia_off":
        h.tune(psc.TUNE_DIA, 0)
    if knob == "tail_off":
        h.tune(psc.TUNE_TAIL, 0)
    if knob == "tail_4096":
        h.tune(psc.TUNE_TAIL, 4096)
    if knob == "dia_per_slice":
        h.tune(psc.TUNE_DIA_UNIFORM, 0)
    if knob == "xcd_chunks":
        h.tune(psc.TUNE_XCD, 1)
    if knob == "mixed_fused":
        h.tune(psc.TUNE_MIXED_SPLIT, 0)
    if knob in ("split_off", "bufload_all", "bufload_none", "unroll4"):
        h.tune(psc.TUNE_SPLIT, 0)                    # sweeps gather through A, M^-1, P
    if knob == "bufload_all":
        h.tune(psc.TUNE_BUFLOAD, 1)
    elif knob == "bufload_none":
        h.tune(psc.TUNE_BUFLOAD, 0)
    elif knob == "unroll4":
        h.tune(psc.TUNE_BUFLOAD, 0)
        h.tune(psc.TUNE_UNROLL4, 1)
    elif knob == "spmv2":
        h.tune(psc.TUNE_SPMV2, 1)
    elif knob == "grid256":
        h.tune(psc.TUNE_GRID_MAX, 256)               # several slices per wavefront
    o = oracle.Hierarchy(rp, c, v, coarse_max=cm)
    n = len(rp) - 1
    x = np.random.default_rng(3).standard_normal(n)
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    h.spmv(dev(x), y)
    ref = oracle.spmv(rp, c, v, x)
    assert np.abs(y.cpu().numpy() - ref).max() <= 1e-13 * np.abs(ref).max()
    h.vcycle(dev(x), y)
    ref = o.vcycle(x)
    assert np.linalg.norm(y.cpu().numpy() - ref) <= 1e-12 * np.linalg.norm(ref)
    h.vcycle(dev(x), y, prec=psc.FP32)
    ref = o.vcycle32(x)
    assert np.linalg.norm(y.cpu().numpy() - ref) <= 1e-5 * np.linalg.norm(ref)
    b = P.rhs_uniform(n, 4)
    xg = torch.zeros(n, dtype=torch.float64, device="cuda")
    g = h.pcg(dev(b), xg)
    r = o.pcg(b)
    assert abs(g["iters"] - r["iters"]) <= 1 and g["relres"] <= 1e-6
    xg.zero_()
    g = h.fcg(dev(b), xg, prec=psc.FP32)
    r = o.fcg(b, form=1)
    assert abs(g["iters"] - r["iters"]) <= 1 and g["relres"] <= 1e-6
    if knob == "xcd_chunks":
        h.tune(psc.TUNE_XCD, 0)                      # per device: restore the default for later tests


@pytest.mark.parametrize("rows", [1024, 4096])
def test_tail_in_lds_matches_oracle(psc, rows):
    """Levels 4000, 1000, 250 and 63 (coarsest) of Poisson 40^3 in the
    one-workgroup tail: 21 KB of LDS at 1024 rows, 85 KB at 4096."""
    rp, c, v = P.poisson7(40)
    h = psc.Hierarchy(rp, c, v, build_fp32=True)
    h.tune(psc.TUNE_TAIL, rows)
    info = h.info()
    assert info["rows"][2:] == [4000, 1000, 250, 63]
    assert info["tail_level"] == (2 if rows == 4096 else 3)
    assert info["tail_lds_bytes"] == 16 * sum(info["rows"][info["tail_level"]:])
    o = oracle.Hierarchy(rp, c, v)
    n = len(rp) - 1
    x = np.random.default_rng(5).standard_normal(n)
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    h.vcycle(dev(x), y)
    ref = o.vcycle(x)
    assert np.linalg.norm(y.cpu().numpy() - ref) <= 1e-12 * np.linalg.norm(ref)
    h.vcycle(dev(x), y, prec=psc.FP32)
    ref = o.vcycle32(x)
    assert np.linalg.norm(y.cpu().numpy() - ref) <= 1e-5 * np.linalg.norm(ref)
    b = P.rhs_uniform(n, 4)
    for form in ("pcg", "fcg32"):
        xg = torch.zeros(n, dtype=torch.float64, device="cuda")
        if form == "pcg":
            g, r = h.pcg(dev(b), xg), o.pcg(b)
        else:
            g, r = h.fcg(dev(b), xg, prec=psc.FP32), o.fcg(b, form=1)
        assert g["status"] == psc.OK and abs(g["iters"] - r["iters"]) <= 1 and g["relres"] <= 1e-6
    h.tune(psc.TUNE_TAIL, 0)
    assert h.info()["tail_level"] == 0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fcg_tight_tolerance_residual_replacement(psc, prec):
    """At rtol 1e-11 the recursive residual can pass before the true one;
    the FCG forms then replace r by b - A x and continue (fused and not)."""
    rp, c, v = P.diffusion7(24, seed=3, az=0.01)
    b = P.rhs_from_solution(rp, c, v, P.x_true(24 ** 3, 2))
    res = []
    for fused in (1, 0):
        h = psc.Hierarchy(rp, c, v, build_fp32=True)
        h.tune(psc.TUNE_FUSED_PCG, fused)
        x = torch.zeros(len(b), dtype=torch.float64, device="cuda")
        g = h.fcg(dev(b), x, rtol=1e-11, maxit=400, prec=psc.FP32 if prec == "fp32" else psc.FP64)
        assert g["status"] == psc.OK and g["relres"] <= 1e-11
        res.append(g["iters"])
    assert abs(res[0] - res[1]) <= 3


SMOOTHING = {
    # name: options of both the library and the oracle
    "smatch": dict(sweeps=3, prol=1, nu=4),
    "vmatch": dict(sweeps=3, nu=2, double=True),
    "vbm": dict(aggr=1, prol=1, nu=4),
    "tentative_nu2": dict(nu=2),
    "smoothed_nu1": dict(prol=1),
    "smoothed_nu3": dict(sweeps=3, prol=1, nu=3),
}


@pytest.mark.parametrize("tail", [True, False])
@pytest.mark.parametrize("cfg", list(SMOOTHING))
@pytest.mark.parametrize("case", ["poisson24", "diffusion20_az100", "random_long_rows"])
def test_smoothing_configurations_match_oracle(psc, case, cfg, tail):
    """tail: the levels up to 4096 rows (several sweeps each) in the
    one-workgroup LDS kernel, or launched level by level."""
    o_ = dict(sweeps=2, prol=0, nu=1, double=False, aggr=0)
    o_.update(SMOOTHING[cfg])
    sweeps, smoothed, nu, double, aggr = o_["sweeps"], o_["prol"], o_["nu"], o_["double"], o_["aggr"]
    rp, c, v = P.poisson7(24) if case == "poisson24" else CASES[case]()
    cm = 40 if case == "random_long_rows" else 200
    h = psc.Hierarchy(rp, c, v, coarse_max=cm, sweeps=sweeps, build_fp32=True, smoothed_prol=bool(smoothed),
                      smoother_sweeps=nu, vcycle_double=double, aggregation=aggr, vbm_theta=0.05)
    o = oracle.Hierarchy(rp, c, v, coarse_max=cm, sweeps=sweeps, prol=smoothed, nu=nu, nu_double=double,
                         aggr=aggr, theta=0.05)
    assert h.info()["rows"] == o.sizes()
    # an explicit row limit takes the small levels whatever their operator bytes
    h.tune(psc.TUNE_TAIL, 4096 if tail else 0)
    assert (h.info()["tail_level"] > 0) == (tail and h.info()["levels"] >= 3)
    n = len(rp) - 1
    x = np.random.default_rng(5).standard_normal(n)
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    h.vcycle(dev(x), y)
    ref = o.vcycle(x)
    assert np.linalg.norm(y.cpu().numpy() - ref) <= 1e-12 * np.linalg.norm(ref)
    h.vcycle(dev(x), y, prec=psc.FP32)
    ref32 = o.vcycle32(x)
    assert np.linalg.norm(y.cpu().numpy() - ref32) <= 1e-5 * np.linalg.norm(ref32)
    b = P.rhs_from_solution(rp, c, v, P.x_true(n, 1))
    xg = torch.zeros(n, dtype=torch.float64, device="cuda")
    r = o.pcg(b)
    for fused in (1, 0):
        h.tune(psc.TUNE_FUSED_PCG, fused)
        xg.zero_()
        g = h.pcg(dev(b), xg)
        assert g["status"] == psc.OK and abs(g["iters"] - r["iters"]) <= 1 and g["relres"] <= 1e-6
    k = min(g["iters"], r["iters"])
    xg.zero_()
    h.pcg(dev(b), xg, rtol=1e-30, maxit=k)
    refk = o.pcg(b, rtol=1e-30, maxit=k)["x"]
    assert np.linalg.norm(xg.cpu().numpy() - refk) <= 1e-8 * np.linalg.norm(refk)
    h.tune(psc.TUNE_FUSED_PCG, 1)
    r32 = o.fcg(b, form=1)
    xg.zero_()
    g = h.fcg(dev(b), xg, prec=psc.FP32)
    assert abs(g["iters"] - r32["iters"]) <= 1 and g["relres"] <= 1e-6
    if nu > 1 or smoothed or double:
        with pytest.raises(psc.PscError):
            h.tune(psc.TUNE_SPLIT, 0)


@pytest.mark.parametrize("case,sweeps,cm,smoothed", [("poisson32", 2, 200, False), ("poisson13", 2, 200, False),
                                                     ("poisson24", 3, 200, False), ("diffusion20_az100", 2, 200, False),
                                                     ("random_long_rows", 2, 40, False),
                                                     ("diffusion48_lognormal", 2, 200, False),
                                                     # smoothed prolongator: device aggregates and products
                                                     ("poisson24", 3, 200, True), ("poisson13", 3, 200, True),
                                                     ("diffusion20_az100", 3, 200, True),
                                                     ("random_long_rows", 2, 40, True)])
def test_device_setup_bit_identical_to_host(psc, case, sweeps, cm, smoothed):
    rp, c, v = P.poisson7(24) if case == "poisson24" else CASES[case]()
    hd = psc.Hierarchy(rp, c, v, sweeps=sweeps, coarse_max=cm, setup_device=True, smoothed_prol=smoothed,
                       setup_device_products=smoothed)
    hh = psc.Hierarchy(rp, c, v, sweeps=sweeps, coarse_max=cm, setup_device=False, host_only=True,
                       smoothed_prol=smoothed)
    a, b = hd.info(), hh.info()
    assert a["rows"] == b["rows"] and a["nnz"] == b["nnz"] and a["coarse_sweeps"] == b["coarse_sweeps"]
    for l in range(a["levels"]):
        x, y = hd.export_level(l), hh.export_level(l)
        for key in ["rowptr", "col", "val", "minv"]:
            assert np.array_equal(x[key], y[key]), (l, key)
        if l < a["levels"] - 1:
            assert np.array_equal(x["agg"], y["agg"]) and np.array_equal(x["p"], y["p"]), l
            if smoothed:
                px, py = hd.export_prolongator(l), hh.export_prolongator(l)
                assert all(np.array_equal(u, w) for u, w in zip(px, py)), l


@pytest.mark.parametrize("case", ["poisson24", "diffusion20_az100", "random_long_rows"])
def test_device_products_of_vbm_smoothed_hierarchy_bit_identical_to_host(psc, case):
    """VBM aggregation stays on the host; its smoothed prolongator's products
    (omega, P, A P, P^T A P) run on the GPU and must equal the host's."""
    rp, c, v = P.poisson7(24) if case == "poisson24" else CASES[case]()
    cm = 40 if case == "random_long_rows" else 200
    kw = dict(coarse_max=cm, aggregation=psc.AGGR_VBM, smoothed_prol=True, smoother_sweeps=4)
    hd = psc.Hierarchy(rp, c, v, setup_device=True, setup_device_products=True, **kw)
    hh = psc.Hierarchy(rp, c, v, setup_device=False, host_only=True, **kw)
    a, b = hd.info(), hh.info()
    assert a["rows"] == b["rows"] and a["nnz"] == b["nnz"] and a["omega"] == b["omega"]
    assert a["levels"] >= 2
    for l in range(a["levels"]):
        x, y = hd.export_level(l), hh.export_level(l)
        for key in ["rowptr", "col", "val", "minv"]:
            assert np.array_equal(x[key], y[key]), (l, key)
        if l < a["levels"] - 1:
            px, py = hd.export_prolongator(l), hh.export_prolongator(l)
            assert all(np.array_equal(u, w) for u, w in zip(px, py)), l


def _diag_csr(d):
    n = len(d)
    return np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.asarray(d, dtype=np.float64)


def _block_diag(*mats):
    rps, cs, vs, off, nnz = [np.zeros(1, np.int32)], [], [], 0, 0
    for rp, c, v in mats:
        rps.append((rp[1:] + nnz).astype(np.int32))
        cs.append((c + off).astype(np.int32))
        vs.append(v)
        off += len(rp) - 1
        nnz += rp[-1]
    return np.concatenate(rps), np.concatenate(cs), np.concatenate(vs)


@pytest.mark.parametrize("case", ["one_by_one", "diagonal_3000", "two_components"])
def test_degenerate_systems_match_oracle(psc, case):
    """A 1x1 system, a diagonal matrix (nothing to match: every aggregate a
    singleton, so coarsening stalls at once) and two disconnected Poisson
    blocks of different sizes: GPU PCG and mixed FCG against the oracle."""
    if case == "one_by_one":
        rp, c, v = _diag_csr([4.0])
    elif case == "diagonal_3000":
        rp, c, v = _diag_csr(1.0 + np.random.default_rng(4).random(3000))
    else:
        rp, c, v = _block_diag(P.poisson7(10), P.poisson7(9))
    n = len(rp) - 1
    h = psc.Hierarchy(rp, c, v, build_fp32=True)
    o = oracle.Hierarchy(rp, c, v)
    assert h.info()["levels"] == o.nlevels
    b = P.rhs_uniform(n, 6)
    ro = o.pcg(b)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    g = h.pcg(dev(b), x)
    assert g["status"] == psc.OK and ro["status"] == oracle.OK
    assert abs(g["iters"] - ro["iters"]) <= 1 and g["relres"] <= 1e-6
    assert np.linalg.norm(x.cpu().numpy() - ro["x"]) <= 1e-8 * np.linalg.norm(ro["x"])
    x.zero_()
    g = h.fcg(dev(b), x, prec=psc.FP32)
    assert g["status"] == psc.OK and g["relres"] <= 1e-6


def test_tail_lds_limit_holds_across_handles(psc):
    """The dynamic-LDS limit of the tail kernel is per kernel and process-wide:
    a handle built later with a smaller tail above 64 KB must not shrink it
    below what an earlier handle launches (85 KB after 73 KB here)."""
    hs, outs = [], []
    for n in (40, 38):
        rp, c, v = P.poisson7(n)
        h = psc.Hierarchy(rp, c, v)
        h.tune(psc.TUNE_TAIL, 4096)
        assert h.info()["tail_lds_bytes"] > 64 * 1024
        hs.append((h, rp, c, v))
    assert hs[0][0].info()["tail_lds_bytes"] > hs[1][0].info()["tail_lds_bytes"]
    for h, rp, c, v in hs:                    # the larger tail runs after the smaller one was set up
        n = len(rp) - 1
        x = np.random.default_rng(7).standard_normal(n)
        y = torch.empty(n, dtype=torch.float64, device="cuda")
        h.vcycle(dev(x), y)
        ref = oracle.Hierarchy(rp, c, v).vcycle(x)
        assert np.linalg.norm(y.cpu().numpy() - ref) <= 1e-12 * np.linalg.norm(ref)


def test_mixed_split_passes_equal_fused_bit_for_bit(psc):
    """The mixed form's split second pass (r -= alpha q with an FP32 copy of r,
    the FP32 pre-smoothing and the level-0 post-smoothing reading that copy)
    equals the fused pass that rounds FP64 r at every use: the same FP32
    values in the same order, so the same iterates bit for bit, also across
    residual replacements (rtol 1e-11)."""
    rp, c, v = P.diffusion7(24, seed=3, az=0.01)
    b = dev(P.rhs_from_solution(rp, c, v, P.x_true(24 ** 3, 2)))
    out = []
    for split in (1, 0):
        h = psc.Hierarchy(rp, c, v, build_fp32=True)
        h.tune(psc.TUNE_MIXED_SPLIT, split)
        x = torch.zeros(len(b), dtype=torch.float64, device="cuda")
        g = h.fcg(b, x, rtol=1e-11, maxit=400, prec=psc.FP32)
        assert g["status"] == psc.OK and g["relres"] <= 1e-11
        out.append((g["iters"], x))
    assert out[0][0] == out[1][0]
    assert torch.equal(out[0][1], out[1][1])


@pytest.mark.parametrize("form", ["pcg", "fcg"])
def test_fp64_split_update_equals_fused_bit_for_bit(psc, form):
    """FP64 second pass as two kernels (r -= alpha q, then the level-0
    pre-smoothing residual gathering r) equals the fused pass that recomputes
    r at every gathered neighbour: bit-identical iterates, also across FCG's
    residual replacements (rtol 1e-11)."""
    rp, c, v = P.diffusion7(24, seed=3, az=0.01)
    b = dev(P.rhs_from_solution(rp, c, v, P.x_true(24 ** 3, 2)))
    out = []
    for split in (1, 0):
        h = psc.Hierarchy(rp, c, v)
        h.tune(psc.TUNE_FP64_SPLIT, split)
        x = torch.zeros(len(b), dtype=torch.float64, device="cuda")
        g = h.pcg(b, x, rtol=1e-9) if form == "pcg" else h.fcg(b, x, rtol=1e-11, maxit=400)
        assert g["status"] == psc.OK
        out.append((g["iters"], x))
    assert out[0][0] == out[1][0]
    assert torch.equal(out[0][1], out[1][1])
