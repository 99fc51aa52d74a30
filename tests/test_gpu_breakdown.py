"""GPU: a CG breakdown returns PSC_ERR_NOT_SPD and leaves the last valid
iterate in x, like the oracle (whose behaviour is pinned in
test_oracle_amg.py::test_breakdown_returns_last_valid_iterate)."""
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


@pytest.mark.parametrize("fused", [1, 0])
@pytest.mark.parametrize("kind", ["pcg", "fcg64", "fcg32"])
def test_breakdown_leaves_last_valid_iterate(psc, kind, fused):
    n, sigma = 8, 0.40
    rp, c, v = P.poisson7(n)
    v = v.copy()
    rows = np.repeat(np.arange(n ** 3), np.diff(rp))
    v[rows == c] -= sigma                       # one negative eigenvalue
    h = psc.Hierarchy(rp, c, v, coarse_max=20, build_fp32=True)
    h.tune(psc.TUNE_FUSED_PCG, fused)
    o = oracle.Hierarchy(rp, c, v, coarse_max=20)
    b = P.rhs_uniform(n ** 3, 1)
    if kind == "pcg":
        ref = o.pcg(b, rtol=1e-10, maxit=300)
    else:
        ref = o.fcg(b, rtol=1e-10, maxit=300, form=0 if kind == "fcg64" else 1)
    assert ref["status"] == oracle.ERR_NOT_SPD and ref["iters"] >= 2
    x = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
    bd = torch.from_numpy(b).cuda()
    with pytest.raises(psc.PscError) as e:
        if kind == "pcg":
            h.pcg(bd, x, rtol=1e-10, maxit=300)
        else:
            h.fcg(bd, x, rtol=1e-10, maxit=300, prec=psc.FP64 if kind == "fcg64" else psc.FP32)
    assert e.value.status == psc.ERR_NOT_SPD
    xg = x.cpu().numpy()
    tol = 1e-10 if kind != "fcg32" else 1e-5
    assert np.linalg.norm(xg - ref["x"]) <= tol * np.linalg.norm(ref["x"])
