"""One call over more rows than a 32-bit index can count (2^31 + 4099): every
kernel indexes rows in 64 bits.  Sampled rows of the direct and tree routes,
among them the last rows and those around row 2^31, against the oracle; and
closed forms that hold on every row: a unit source at the phase centre gives
V = 1 exactly, its adjoint at the centre pixel is the row count, chi^2 of V
against a zero model at inv_sigma2 = 1/2 is half the row count, and the flux
gradient of the centred source with y = V is the row count."""
import numpy as np
import pytest

from oracle import tree as ot
from oracle import visibility as ov

from .gpu_util import errors, fp64_row_bound, host, note, require_gpu

pytestmark = pytest.mark.gpu
N = (1 << 31) + 4099
TOL64 = 1e-12


def test_rows_past_2_31():
    torch, swv = require_gpu()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()   # blocks cached by earlier tests
    free, _ = torch.cuda.mem_get_info()
    need = N * (3 * 8 + 2 * 16) + (8 << 30)   # u, v, w; V and a zero model; headroom
    if free < need:
        pytest.skip(f"needs {need / 2**30:.0f} GiB of free device memory")
    note(f"rows past 2^31: {N} rows")
    j = torch.arange(N, dtype=torch.float64, device="cuda")
    # smooth tracks of a few km, from the row index
    u = torch.mul(j, 3.7e-7).add_(0.1).sin_().mul_(2e4)
    v = torch.mul(j, 5.3e-7).add_(0.2).sin_().mul_(2e4)
    w = torch.mul(j, 1.1e-7).add_(0.5).sin_().mul_(3e3)
    del j
    rng = np.random.default_rng(231)
    rows = np.unique(np.concatenate([rng.integers(0, N, 2000), np.arange(N - 600, N),
                                     np.arange((1 << 31) - 300, (1 << 31) + 300)]))
    idx = torch.as_tensor(rows, device="cuda")
    us, vs, ws = (host(a.index_select(0, idx)) for a in (u, v, w))

    # direct sum, three components
    l = rng.uniform(-0.02, 0.02, 3)
    m = rng.uniform(-0.02, 0.02, 3)
    f = rng.lognormal(-1.0, 0.5, 3)
    L, M, F = (torch.as_tensor(a, device="cuda") for a in (l, m, f))
    out = torch.empty(N, dtype=torch.complex128, device="cuda")
    swv.predict_direct(u, v, w, L, M, F, out=out)
    got = host(out.index_select(0, idx))
    ref = ov.predict_direct(us, vs, ws, l, m, f)
    bound = fp64_row_bound(us, vs, ws, l, m, ov.n_minus_1(l, m), f)
    assert np.all(np.abs(got - ref) <= bound)

    # tree route of the same components
    ra, dec = 1.0, 0.5
    T = swv.Tree(6, ra, dec, l, m, f)
    T.predict(u, v, w, out=out)
    got = host(out.index_select(0, idx))
    ref = ot.predict_tree(ot.build_tree(6, ra, dec, l, m, f), us, vs, ws)
    e_max, _ = errors(got, ref, f.sum())
    note(f"tree over {N} rows, sampled: E_max={e_max:.3e}")
    assert e_max <= TOL64
    T.close()

    # closed forms on every row
    zero = torch.zeros(1, dtype=torch.float64, device="cuda")
    one = torch.ones(1, dtype=torch.float64, device="cuda")
    swv.predict_direct(u, v, w, zero, zero, one, out=out)
    assert float((out - 1).abs().max()) == 0.0
    img = host(swv.adjoint(u, v, w, out, zero, zero, zero))
    assert img[0] == complex(N, 0.0)
    g = [host(x) for x in swv.grad_direct(u, v, w, out, zero, zero, one)]
    assert g[0][0] == float(N) and g[1][0] == 0.0 and g[2][0] == 0.0
    model = torch.zeros(N, dtype=torch.complex128, device="cuda")
    r, chi2 = swv.residual_chi2(out, model, 0.5, out=out)
    assert float(chi2[0]) == 0.5 * N
    assert float((r - 1).abs().max()) == 0.0
    swv.synchronize()
    del u, v, w, out, model, r, idx
    torch.cuda.empty_cache()
