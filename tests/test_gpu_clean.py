"""GPU parity of the clean loop (sections 2.1, 2.2, 3.5) against oracle/clean.py:
image grids, dirty images and the dirty beam, the Hogbom minor cycle
(bit-exact: one product and one subtraction per pixel on both sides, the same
peak rule), the clean image of Eq. 6 and the whole major/minor loop; the
seven-source 707,616-row workload at full size on sampled pixels."""
import numpy as np
import pytest

from oracle import clean as oc
from oracle import visibility as ov
from synth import configs

from .gpu_util import dev, dev_c, host, note, require_gpu

pytestmark = pytest.mark.gpu
TOL64 = 1e-12


@pytest.fixture(scope="module")
def env():
    return require_gpu()


def _beam_like(rng, ny, nx, quantum=None):
    """A peaked, asymmetric synthetic beam with sidelobes, centre 1."""
    dy, dx = np.meshgrid(np.arange(-(ny - 1), ny), np.arange(-(nx - 1), nx), indexing="ij")
    b = np.exp(-(0.02 * dx * dx + 0.01 * dx * dy + 0.05 * dy * dy))
    b += 0.2 * np.cos(0.7 * dx + 0.3 * dy) * np.exp(-0.002 * (dx * dx + dy * dy))
    b *= 1 + 0.05 * rng.uniform(-1, 1, b.shape)
    if quantum:
        b = np.round(b / quantum) * quantum
    b[ny - 1, nx - 1] = 1.0
    return b


def _image_like(rng, ny, nx, beam, n_src=6, quantum=None):
    img = 0.02 * rng.normal(size=(ny, nx))
    for _ in range(n_src):
        p = int(rng.integers(nx * ny))
        py, px = divmod(p, nx)
        img += rng.uniform(-0.5, 1.5) * beam[ny - 1 - py:2 * ny - 1 - py, nx - 1 - px:2 * nx - 1 - px]
    if quantum:
        img = np.round(img / quantum) * quantum
    return img


def _hogbom_gpu(torch, swv, img, beam, gain, thr, k, absolute, single=False):
    t_img = torch.as_tensor(img.copy(), device="cuda")
    t_beam = torch.as_tensor(beam, device="cuda")
    pix, val = swv.hogbom(t_img, t_beam, gain, thr, k, absolute, single_workgroup=single)
    return host(t_img), host(pix), host(val)


# ------------------------------------------------------------------ grid --
def test_image_grid_vs_oracle(env):
    torch, swv = env
    for nx, ny, cx, cy, cell in ((40, 40, 20, 20, 1.7e-3), (37, 23, 18, 11, 0.01),
                                 (21, 21, 10, 10, 0.09)):
        l, m, nm1 = (host(t) for t in swv.image_grid(nx, ny, cell, cx, cy))
        rl, rm, rn, inside = oc.image_grid(nx, ny, cell, cx, cy)
        rl[~inside] = 0.0
        rm[~inside] = 0.0
        assert np.array_equal(l, rl) and np.array_equal(m, rm)
        assert np.all(np.abs(nm1 - rn) <= np.spacing(np.abs(rn)))


# ---------------------------------------------------------- dirty images --
@pytest.fixture(scope="module")
def small():
    S = configs.CLEAN_SMALL
    u, v, w = S.track.uvw()
    l, m, f = S.sources()
    vis = ov.predict_direct(u, v, w, l, m, f) + S.noise()
    return S, u, v, w, vis


def test_dirty_image_and_beam_vs_oracle(env, small):
    torch, swv = env
    S, u, v, w, vis = small
    n = S.n_pix
    U, V, W = dev(u, torch), dev(v, torch), dev(w, torch)
    img = host(swv.dirty_image(U, V, W, dev_c(vis, torch), n, n, S.cell)).ravel()
    l, m, nm1, _ = oc.image_grid(n, n, S.cell)
    ref = oc.dirty_image(u, v, w, vis, l, m, nm1)
    e = np.abs(img - ref).max() / (np.abs(vis).sum() / u.size)
    beam = host(swv.dirty_beam(U, V, W, n, n, S.cell))
    rb = oc.dirty_beam(u, v, w, n, n, S.cell)
    eb = np.abs(beam - rb).max()
    note(f"clean_small dirty image E_max={e:.3e}, beam E_max={eb:.3e} ({u.size} rows)")
    assert e <= TOL64 and eb <= TOL64
    assert beam[n - 1, n - 1] == 1.0


def test_dirty_beam_off_disk_is_zero(env, small):
    torch, swv = env
    S, u, v, w, vis = small
    beam = host(swv.dirty_beam(dev(u, torch), dev(v, torch), dev(w, torch), 6, 6, 0.17))
    rb = oc.dirty_beam(u, v, w, 6, 6, 0.17)
    assert np.array_equal(beam == 0.0, rb == 0.0)
    assert np.abs(beam - rb).max() <= TOL64


# ---------------------------------------------------------------- Hogbom --
@pytest.mark.parametrize("ny,nx", [(40, 40), (23, 37), (1, 1), (50, 1), (1, 64), (200, 300),
                                   (3, 1500)])
def test_hogbom_bitwise_vs_oracle(env, ny, nx):
    torch, swv = env
    rng = np.random.default_rng(ny * 7919 + nx)
    beam = _beam_like(rng, ny, nx)
    img = _image_like(rng, ny, nx, beam)
    for gain, thr, k, absolute in ((0.1, 0.0, 150, False), (0.3, 0.05, 400, True),
                                   (1.0, -1.0, 7, False)):
        note(f"hogbom {ny}x{nx} gain={gain} thr={thr} k={k} abs={absolute}")
        got_img, got_pix, got_val = _hogbom_gpu(torch, swv, img, beam, gain, thr, k, absolute)
        ref_img, ref_pix, ref_val = oc.hogbom(img, beam, gain, thr, k, absolute)
        assert np.array_equal(got_pix, ref_pix)
        assert np.array_equal(got_val, ref_val)
        assert np.array_equal(got_img, ref_img)


def test_hogbom_ties_and_stops(env):
    torch, swv = env
    rng = np.random.default_rng(77)
    ny, nx = 31, 45
    beam = _beam_like(rng, ny, nx, quantum=1 / 64)
    img = _image_like(rng, ny, nx, beam, quantum=1 / 16)   # many exactly equal pixels
    for gain, thr, k, absolute in ((0.5, 0.0, 300, False), (0.5, 0.0, 300, True),
                                   (0.25, 0.4, 10_000, False), (0.1, 0.0, 0, False),
                                   (0.1, 1e9, 50, True)):
        got_img, got_pix, got_val = _hogbom_gpu(torch, swv, img, beam, gain, thr, k, absolute)
        ref_img, ref_pix, ref_val = oc.hogbom(img, beam, gain, thr, k, absolute)
        assert np.array_equal(got_pix, ref_pix) and np.array_equal(got_val, ref_val)
        assert np.array_equal(got_img, ref_img)


def test_hogbom_full_size_bitwise(env):
    """The 256 x 256 image and 511 x 511 beam of the seven-source workload,
    300 iterations (one major cycle's minor cycle)."""
    torch, swv = env
    S = configs.CLEAN7
    rng = np.random.default_rng(256)
    beam = _beam_like(rng, S.n_pix, S.n_pix)
    img = _image_like(rng, S.n_pix, S.n_pix, beam, n_src=7)
    got_img, got_pix, got_val = _hogbom_gpu(torch, swv, img, beam, S.gain, 0.0, S.minor_iter,
                                            False)
    ref_img, ref_pix, ref_val = oc.hogbom(img, beam, S.gain, 0.0, S.minor_iter)
    assert got_pix.size == S.minor_iter
    assert np.array_equal(got_pix, ref_pix) and np.array_equal(got_val, ref_val)
    assert np.array_equal(got_img, ref_img)


@pytest.mark.parametrize("ny,nx", [(256, 256), (128, 129), (181, 181), (3, 6000), (16384, 1)])
def test_hogbom_grid_and_single_workgroup_agree(env, ny, nx):
    """From 16,384 pixels the cycle runs grid-wide (one workgroup per compute
    unit, a grid barrier per iteration); forced into one workgroup it gives
    the same bits, and both equal the oracle, ties included."""
    torch, swv = env
    rng = np.random.default_rng(ny + 3 * nx)
    beam = _beam_like(rng, ny, nx, quantum=1 / 64)
    img = _image_like(rng, ny, nx, beam, n_src=5, quantum=1 / 16)
    for gain, thr, k, absolute in ((0.2, 0.0, 120, False), (0.5, 0.1, 200, True)):
        note(f"hogbom grid/single {ny}x{nx} gain={gain} k={k} abs={absolute}")
        g = _hogbom_gpu(torch, swv, img, beam, gain, thr, k, absolute)
        o = _hogbom_gpu(torch, swv, img, beam, gain, thr, k, absolute, single=True)
        ref_img, ref_pix, ref_val = oc.hogbom(img, beam, gain, thr, k, absolute)
        for got_img, got_pix, got_val in (g, o):
            assert np.array_equal(got_pix, ref_pix) and np.array_equal(got_val, ref_val)
            assert np.array_equal(got_img, ref_img)


def test_hogbom_argument_errors(env):
    torch, swv = env
    img = torch.zeros((4, 5), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        swv.hogbom(img, torch.zeros((9, 7), dtype=torch.float64, device="cuda"), 0.1, 0, 3)
    beam = torch.zeros((7, 9), dtype=torch.float64, device="cuda")
    with pytest.raises(swv.SwvError, match="SWV_EDOMAIN"):
        swv.hogbom(img, beam, float("inf"), 0.0, 3)


# --------------------------------------------------------------- restore --
def test_restore_vs_oracle(env):
    torch, swv = env
    rng = np.random.default_rng(9)
    nx, ny = 64, 48
    pix = rng.integers(0, nx * ny, 200)
    pix[:20] = pix[0]                       # repeated components
    val = rng.normal(size=200)
    abc = (0.08, -0.02, 0.12)
    res = rng.normal(size=(ny, nx))
    for r in (None, res):
        got = host(swv.restore(nx, ny, torch.as_tensor(pix, device="cuda"), dev(val, torch), abc,
                               None if r is None else torch.as_tensor(r, device="cuda")))
        ref = oc.restore(nx, ny, pix, val, abc, r)
        assert np.abs(got - ref).max() <= 1e-14 * np.abs(val).sum()
    empty = host(swv.restore(nx, ny, torch.zeros(0, dtype=torch.int64, device="cuda"),
                             torch.zeros(0, dtype=torch.float64, device="cuda"), abc))
    assert np.all(empty == 0.0)


# ------------------------------------------------------------- the loop --
def test_wavelet_clean_small_vs_oracle(env, small):
    torch, swv = env
    S, u, v, w, vis = small
    n = S.n_pix
    got = swv.wavelet_clean(dev(u, torch), dev(v, torch), dev(w, torch), dev_c(vis, torch), n,
                            n, S.cell, S.J, S.ra_p, S.dec_p, S.gain, 0.0, S.minor_iter,
                            S.n_major)
    ref = oc.wavelet_clean(u, v, w, vis, n, n, S.cell, S.J, S.ra_p, S.dec_p, S.gain, 0.0,
                           S.minor_iter, S.n_major)
    note(f"clean_small: {got['pix'].size} components, cycles {got['cycles']}")
    assert np.array_equal(got["pix"], ref["pix"])
    np.testing.assert_allclose(got["val"], ref["val"], rtol=1e-9, atol=1e-12)
    ymax = np.abs(vis).sum() / u.size
    assert np.abs(host(got["residual"]) - ref["residual"]).max() <= 1e-10 * ymax
    assert np.abs(host(got["beam"]) - ref["beam"]).max() <= TOL64
    vm = host(got["vis_model"])
    assert np.abs(vm - ref["vis_model"]).max() <= 1e-10 * np.abs(ref["val"]).sum()
    for cg, cr in zip(got["cycles"], ref["cycles"]):
        assert cg["found"] == cr["found"] and cg["leaves"] == cr["leaves"]
        assert abs(cg["chi2"] - cr["chi2"]) <= 1e-9 * cr["chi2"]
    # Eq. 6 on top of the loop's output, with the clean beam of its dirty beam
    abc = swv.fit_clean_beam(host(got["beam"]))
    np.testing.assert_allclose(abc, oc.fit_clean_beam(ref["beam"]), rtol=1e-9)


@pytest.mark.parametrize("predictor", ["degrid", "direct"])
def test_clean_small_other_predictors_vs_oracle(env, small, predictor):
    """The same loop with the conventional (FFT + degridding, W = 10) and the
    exact (direct) predictor against the oracle's loop."""
    torch, swv = env
    S, u, v, w, vis = small
    n = S.n_pix
    got = swv.wavelet_clean(dev(u, torch), dev(v, torch), dev(w, torch), dev_c(vis, torch), n,
                            n, S.cell, S.J, S.ra_p, S.dec_p, S.gain, 0.0, S.minor_iter,
                            S.n_major, predictor=predictor, support=10)
    ref = oc.wavelet_clean(u, v, w, vis, n, n, S.cell, S.J, S.ra_p, S.dec_p, S.gain, 0.0,
                           S.minor_iter, S.n_major, predictor=predictor, support=10)
    note(f"clean_small {predictor}: cycles {got['cycles']}")
    assert np.array_equal(got["pix"], ref["pix"])
    np.testing.assert_allclose(got["val"], ref["val"], rtol=1e-9, atol=1e-12)
    ymax = np.abs(vis).sum() / u.size
    assert np.abs(host(got["residual"]) - ref["residual"]).max() <= 1e-10 * ymax
    for cg, cr in zip(got["cycles"], ref["cycles"]):
        assert cg["found"] == cr["found"] and cg["leaves"] == cr["leaves"]
        assert abs(cg["chi2"] - cr["chi2"]) <= 1e-9 * cr["chi2"]


def test_clean7_full_size(env):
    """The seven-source workload at full size: 707,616 rows, 256 x 256 pixels,
    two major cycles of 300 Hogbom iterations at J = 9.  Checked: the dirty
    beam and the first residual image on sampled pixels against the oracle,
    chi^2 falling every cycle, and most of the 7 Jy found."""
    torch, swv = env
    S = configs.CLEAN7
    u, v, w = S.track.uvw()
    l, m, f = S.sources()
    vis = ov.predict_direct(u, v, w, l, m, f, chunk=65536) + S.noise()
    U, V, W, Y = dev(u, torch), dev(v, torch), dev(w, torch), dev_c(vis, torch)
    n = S.n_pix
    img = host(swv.dirty_image(U, V, W, Y, n, n, S.cell)).ravel()
    rng = np.random.default_rng(7)
    sel = np.unique(np.concatenate([[0, n * n - 1, (n // 2) * n + n // 2],
                                    rng.choice(n * n, 9, replace=False)]))
    gl, gm, gn, _ = oc.image_grid(n, n, S.cell)
    ref = oc.dirty_image(u, v, w, vis, gl[sel], gm[sel], gn[sel])
    e = np.abs(img[sel] - ref).max() / (np.abs(vis).sum() / u.size)
    note(f"clean7 dirty image: {sel.size} pixels of {n * n} checked, E_max={e:.3e}")
    assert e <= TOL64
    out = swv.wavelet_clean(U, V, W, Y, n, n, S.cell, S.J, S.ra_p, S.dec_p, S.gain, 0.0,
                            S.minor_iter, S.n_major)
    beam = host(out["beam"]).ravel()
    bl, bm, bn, inside = oc.image_grid(2 * n - 1, 2 * n - 1, S.cell, n - 1, n - 1)
    bsel = np.unique(np.concatenate([[(n - 1) * (2 * n - 1) + n - 1],
                                     rng.choice(np.nonzero(inside)[0], 9, replace=False)]))
    rb = oc.dirty_image(u, v, w, np.ones(u.size, np.complex128), bl[bsel], bm[bsel], bn[bsel])
    assert np.abs(beam[bsel] - rb).max() <= TOL64
    assert np.all(beam[~inside] == 0.0)
    # the FP32-compensated beam and image at full size (8 and 32 row chunks here)
    beam32 = host(swv.dirty_beam(U, V, W, n, n, S.cell, prec="f32c")).ravel()
    img32 = host(swv.dirty_image(U, V, W, Y, n, n, S.cell, prec="f32c")).ravel()
    e32 = np.abs(img32[sel] - ref).max() / (np.abs(vis).sum() / u.size)
    eb32 = np.abs(beam32[bsel] - rb).max()
    note(f"clean7 f32c: dirty image E_max={e32:.2e}, beam {eb32:.2e}")
    assert e32 <= 1e-6 and eb32 <= 1e-6 and np.all(beam32[~inside] == 0.0)
    chi2 = [c["chi2"] for c in out["cycles"]]
    note(f"clean7: cycles {out['cycles']}, beam {out['ms_beam']:.1f} ms, "
         f"dirty {out['ms_dirty']:.1f} ms, flux {out['val'].sum():.3f} Jy")
    assert len(chi2) == S.n_major and chi2[1] < chi2[0]
    assert chi2[0] < float(np.sum(np.abs(vis) ** 2))
    # where the model flux went: within 1.5 pixels of a true source
    px, py = l / S.cell + n // 2, m / S.cell + n // 2
    cy, cx = np.divmod(out["pix"], n)
    near = np.min(np.hypot(cx[:, None] - px[None, :], cy[:, None] - py[None, :]), axis=1) <= 1.5
    frac = out["val"][near].sum() / np.abs(out["val"]).sum()
    note(f"clean7: {frac:.3f} of the component flux lies within 1.5 pixels of a source")
    assert frac > 0.5


def test_wavelet_clean_edge_cases(env, small):
    """No cycles, no iterations, a threshold above every peak, absolute
    peaks (against the oracle), and argument errors of the driver."""
    torch, swv = env
    S, u, v, w, vis = small
    n = S.n_pix
    U, V, W, Y = dev(u, torch), dev(v, torch), dev(w, torch), dev_c(vis, torch)
    common = (U, V, W, Y, n, n, S.cell, S.J, S.ra_p, S.dec_p)
    out = swv.wavelet_clean(*common, gain=0.1, threshold=0.0, minor_iter=10, n_major=0)
    assert out["pix"].size == 0 and out["cycles"] == []
    l, m, nm1, _ = oc.image_grid(n, n, S.cell)
    dirty = oc.dirty_image(u, v, w, vis, l, m, nm1).reshape(n, n)
    ymax = np.abs(vis).sum() / u.size
    assert np.abs(host(out["residual"]) - dirty).max() <= 1e-12 * ymax
    assert np.all(host(out["vis_model"]) == 0)
    out = swv.wavelet_clean(*common, minor_iter=0, n_major=3)
    assert out["pix"].size == 0 and out["cycles"] == []
    out = swv.wavelet_clean(*common, threshold=1e6, minor_iter=50, n_major=3)
    assert out["pix"].size == 0 and out["cycles"] == []
    got = swv.wavelet_clean(*common, gain=0.3, minor_iter=40, n_major=2, absolute=True)
    ref = oc.wavelet_clean(u, v, w, vis, n, n, S.cell, S.J, S.ra_p, S.dec_p, 0.3, 0.0, 40, 2,
                           absolute=True)
    assert np.array_equal(got["pix"], ref["pix"])
    np.testing.assert_allclose(got["val"], ref["val"], rtol=1e-9, atol=1e-12)
    with pytest.raises(swv.SwvError, match="SWV_EDOMAIN"):
        swv.wavelet_clean(*common[:6], 0.3, S.J, S.ra_p, S.dec_p)    # grid off the disk
    with pytest.raises(swv.SwvError, match="SWV_EINVAL"):
        swv.wavelet_clean(*common, n_major=65)
    with pytest.raises(swv.SwvError, match="SWV_EINVAL"):
        swv.wavelet_clean(*common, predictor="degrid", support=1)


def test_restore_of_the_loop_output(env, small):
    """Eq. 6 on the loop's components with the clean beam fitted to its own
    dirty beam, against the oracle on the oracle's loop output."""
    torch, swv = env
    S, u, v, w, vis = small
    n = S.n_pix
    got = swv.wavelet_clean(dev(u, torch), dev(v, torch), dev(w, torch), dev_c(vis, torch), n,
                            n, S.cell, S.J, S.ra_p, S.dec_p, S.gain, 0.0, S.minor_iter, 1)
    abc = swv.fit_clean_beam(host(got["beam"]))
    img = host(swv.restore(n, n, torch.as_tensor(got["pix"], device="cuda"),
                           dev(got["val"], torch), abc, got["residual"]))
    ref = oc.wavelet_clean(u, v, w, vis, n, n, S.cell, S.J, S.ra_p, S.dec_p, S.gain, 0.0,
                           S.minor_iter, 1)
    rimg = oc.restore(n, n, ref["pix"], ref["val"], oc.fit_clean_beam(ref["beam"]),
                      ref["residual"])
    assert np.abs(img - rimg).max() <= 1e-9 * np.abs(ref["val"]).sum()


def test_f32c_images(env, small):
    """The FP32-compensated dirty image and beam against the oracle (1e-6 bar),
    and the whole loop with FP32C images against the oracle's FP64 loop."""
    torch, swv = env
    S, u, v, w, vis = small
    n = S.n_pix
    U, V, W, Y = dev(u, torch), dev(v, torch), dev(w, torch), dev_c(vis, torch)
    img = host(swv.dirty_image(U, V, W, Y, n, n, S.cell, prec="f32c")).ravel()
    l, m, nm1, _ = oc.image_grid(n, n, S.cell)
    ref = oc.dirty_image(u, v, w, vis, l, m, nm1)
    e = np.abs(img - ref).max() / (np.abs(vis).sum() / u.size)
    beam = host(swv.dirty_beam(U, V, W, n, n, S.cell, prec="f32c"))
    eb = np.abs(beam - oc.dirty_beam(u, v, w, n, n, S.cell)).max()
    note(f"clean_small f32c dirty image E_max={e:.2e}, beam {eb:.2e}")
    assert e <= 1e-6 and eb <= 1e-6
    got = swv.wavelet_clean(U, V, W, Y, n, n, S.cell, S.J, S.ra_p, S.dec_p, S.gain, 0.0,
                            S.minor_iter, S.n_major, image_prec="f32c")
    ref = oc.wavelet_clean(u, v, w, vis, n, n, S.cell, S.J, S.ra_p, S.dec_p, S.gain, 0.0,
                           S.minor_iter, S.n_major)
    same = np.mean(got["pix"] == ref["pix"])
    note(f"clean_small f32c loop: {same:.3f} of the components on the oracle's pixels; "
         f"chi2 {[c['chi2'] for c in got['cycles']]} vs {[c['chi2'] for c in ref['cycles']]}")
    assert same >= 0.9
    assert abs(got["val"].sum() - ref["val"].sum()) <= 1e-4 * np.abs(ref["val"]).sum()
    for cg, cr in zip(got["cycles"], ref["cycles"]):
        assert abs(cg["chi2"] - cr["chi2"]) <= 1e-3 * cr["chi2"]


def test_entry_point_argument_errors(env):
    """Bad arguments to the clean-loop and related entry points come back as
    status codes before any launch."""
    torch, swv = env
    import ctypes as C
    from paper_1909_03956_amd._lib import SWV_EDOMAIN, SWV_EINVAL, lib
    L = lib()
    ctx = swv.context().handle
    x = torch.zeros(16, dtype=torch.float64, device="cuda")
    p = C.c_void_p(x.data_ptr())
    assert L.swv_image_grid(ctx, 0, 4, 0, 0, 0.1, p, p, p) == SWV_EINVAL
    assert L.swv_image_grid(ctx, 4, 4, 2, 2, -0.1, p, p, p) == SWV_EDOMAIN
    assert L.swv_image_grid(ctx, 4, 4, 2, 2, 0.1, None, p, p) == SWV_EINVAL
    assert L.swv_dirty_image(ctx, 0, p, p, p, None, 4, 4, 2, 2, 0.1, -1, 0, p) == SWV_EINVAL
    assert L.swv_dirty_image(ctx, 4, p, p, p, None, 4, 4, 2, 2, 0.1, 2, 0, p) == SWV_EDOMAIN
    assert L.swv_dirty_image(ctx, 4, p, p, p, None, 4, 4, 2, 2, 0.1, -1, 7, p) == SWV_EINVAL
    assert L.swv_hogbom(ctx, 2, 2, p, p, 0.1, 0.0, 3, 8, p, p, p) == SWV_EINVAL   # unknown flag
    assert L.swv_hogbom(ctx, 2, 2, p, p, 0.1, 0.0, -1, 0, p, p, p) == SWV_EINVAL
    assert L.swv_hogbom(ctx, 2, 2, p, p, 0.1, float("nan"), 3, 0, p, p, p) == SWV_EDOMAIN
    abc = (C.c_double * 3)(0.1, 0.0, float("inf"))
    assert L.swv_restore(ctx, 2, 2, 1, p, p, abc, None, p) == SWV_EDOMAIN
    assert L.swv_restore(ctx, 2, 2, -1, p, p, abc, None, p) == SWV_EINVAL
    assert L.swv_predict_tree_leaves(ctx, None, 4, p, p, p, -1, 0, p) == SWV_EINVAL
    assert L.swv_predict_degrid(ctx, 4, 4, 0.01, p, 4, p, p, p, 1, -1, p, None) == SWV_EINVAL
    assert L.swv_predict_degrid(ctx, 4, 4, 0.01, p, 4, p, p, p, 8, 0, p, None) == SWV_EDOMAIN
    assert L.swv_cross_reference(0, 0.0, 0.0, 4, 4, 0.01, p) == SWV_EDOMAIN
    assert L.swv_fit_clean_beam(0, 4, p, p) == SWV_EINVAL
    assert b"swv_fit_clean_beam" in L.swv_last_error()
