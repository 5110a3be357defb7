"""GPU parity of the FFT + degridding comparator (swv_predict_degrid) against
oracle/degrid.py on the same inputs, and against the exact direct sum at the
error the kernel width allows, up to the seven-source 707,616-row workload
(sampled rows)."""
import numpy as np
import pytest

from oracle import clean as oc
from oracle import degrid as od
from oracle import visibility as ov
from synth import configs
from synth.configs import TrackSpec

from .gpu_util import dev, host, note, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    return require_gpu()


def _model(nx, ny, k, seed):
    rng = np.random.default_rng(seed)
    img = np.zeros((ny, nx))
    idx = rng.choice(nx * ny, k, replace=False)
    img.flat[idx] = rng.uniform(-0.3, 1.0, k)
    return img, idx


def _gpu(torch, swv, img, u, v, w, cell, W, sign=-1):
    vis, st = swv.predict_degrid(torch.as_tensor(img, device="cuda"), dev(u, torch),
                                 dev(v, torch), dev(w, torch), cell, W, sign)
    return host(vis), st


@pytest.mark.parametrize("nx,ny,cell,W,sign", [(32, 24, 0.006, 6, -1), (24, 24, 0.02, 12, -1),
                                               (17, 31, 0.01, 10, +1), (40, 40, 0.0017, 14, -1),
                                               (1, 1, 0.01, 8, -1)])
def test_degrid_vs_oracle(env, nx, ny, cell, W, sign):
    torch, swv = env
    u, v, w = TrackSpec(27, 1.7e3, 45.0, 2016.0, 4, 1.0e7, seed=731).uvw()
    img, idx = _model(nx, ny, min(10, nx * ny), nx * 100 + ny)
    got, st = _gpu(torch, swv, img, u, v, w, cell, W, sign)
    ref = od.predict_degrid(img, cell, u, v, w, W, sign)
    P = od.plan(nx, ny, cell, w, W)
    assert st["n_planes"] == P["n_planes"] and st["grid"] == (P["Ny"], P["Nx"])
    scale = np.abs(img).sum()
    e = np.abs(got - ref).max() / scale
    l, m, nm1, _ = oc.image_grid(nx, ny, cell)
    exact = ov.predict_direct(u, v, w, l[idx], m[idx], img.flat[idx], sign)
    ex = np.abs(got - exact).max() / scale
    note(f"degrid {ny}x{nx} W={W} s={sign}: {st['n_planes']} planes; vs oracle {e:.2e}, "
         f"vs exact {ex:.2e}")
    assert e <= 1e-12
    assert ex <= 10.0 ** (2 - W)


def test_degrid_clean7_sampled_rows(env):
    """The seven sources on their nearest pixels of the 256 x 256 clean7 grid,
    all 707,616 rows, W = 12: sampled rows against the exact sum."""
    torch, swv = env
    S = configs.CLEAN7
    u, v, w = S.track.uvw()
    l, m, _ = S.sources()
    n = S.n_pix
    ix = np.rint(l / S.cell).astype(int) + n // 2
    iy = np.rint(m / S.cell).astype(int) + n // 2
    img = np.zeros((n, n))
    img[iy, ix] = 1.0
    got, st = _gpu(torch, swv, img, u, v, w, S.cell, 12)
    rows = configs.sample_rows(u.size, 2000, seed=12)
    gl, gm, _, _ = oc.image_grid(n, n, S.cell)
    idx = iy * n + ix
    exact = ov.predict_direct(u[rows], v[rows], w[rows], gl[idx], gm[idx], np.ones(idx.size))
    e = np.abs(got[rows] - exact).max() / idx.size
    note(f"clean7 degrid W=12: {st['n_planes']} planes of {st['grid']}, "
         f"{st['plane_bytes'] / 2**20:.0f} MiB; E_max={e:.2e} on {rows.size} rows")
    assert e <= 1e-10


def test_degrid_edge_cases(env):
    torch, swv = env
    u = np.array([0.0, np.nan, 3.0])
    v = np.array([0.0, 1.0, -2.0])
    w = np.array([0.0, 0.5, 1.0])
    img = np.zeros((8, 8))
    img[4, 4] = 1.0
    got, _ = _gpu(torch, swv, img, u, v, w, 0.01, 8)
    assert np.isnan(got[1]) and np.all(np.isfinite(got[[0, 2]]))
    assert abs(got[0] - 1.0) <= 1e-6
    with pytest.raises(swv.SwvError, match="SWV_EINVAL"):
        _gpu(torch, swv, img, u[[0]], v[[0]], w[[0]], 0.01, 17)
    with pytest.raises(swv.SwvError, match="SWV_EDOMAIN"):
        _gpu(torch, swv, np.zeros((64, 64)), u[[0]], v[[0]], w[[0]], 0.05, 8)
