"""GPU parity of the major-cycle kernels around the prediction: residual and
chi^2, the exact adjoint (residual image on sphere pixels) and the chi^2
gradients, against the oracle and against finite differences."""
import math

import numpy as np
import pytest

from oracle import sphere as sp
from oracle import visibility as ov
from synth import configs, models

from . import oracle_pool
from .gpu_util import U_R, dev, dev_c, errors, fp64_row_bound, host, note, require_gpu

pytestmark = pytest.mark.gpu
TOL64 = 1e-12
TOL32 = 1e-6


@pytest.fixture(scope="module")
def env():
    return require_gpu()


@pytest.fixture(scope="module")
def cfg5():
    """cfg2 tracks, the level-9 pixels within 4 deg, seeded residuals."""
    W = configs.CFG2
    u, v, w = W.track.uvw()
    rng = np.random.default_rng(configs.CFG5_SEED_NOISE)
    y = models.complex_noise(u.size, configs.CFG5_NOISE_SIGMA, rng)
    pix, pl, pm, pn = sp.pixels_in_disk(configs.CFG5_J, W.ra_p, W.dec_p,
                                        math.radians(configs.CFG5_DISK_RADIUS_DEG))
    return W, u, v, w, y, pix, pl, pm, pn


def _pixels(rng, n, far=False):
    l = rng.uniform(-0.3, 0.3, n)
    m = rng.uniform(-0.3, 0.3, n)
    nm1 = ov.n_minus_1(l, m)
    if far:   # directions behind the phase centre: n < 0
        nm1[: n // 3] = -2.0 - nm1[: n // 3]
    return l, m, nm1


@pytest.mark.parametrize("n_vis,n_pix", [(1, 1), (1000, 77), (4097, 300), (30000, 5)])
def test_adjoint_small_vs_oracle(env, n_vis, n_pix):
    torch, swv = env
    rng = np.random.default_rng(n_vis + n_pix)
    u, v, w = (rng.uniform(-3e4, 3e4, n_vis) for _ in range(3))
    y = models.random_complex(n_vis, rng)
    l, m, nm1 = _pixels(rng, n_pix, far=True)
    got = host(swv.adjoint(dev(u, torch), dev(v, torch), dev(w, torch), dev_c(y, torch),
                           dev(l, torch), dev(m, torch), dev(nm1, torch)))
    swv.synchronize()
    ref = ov.adjoint(u, v, w, y, l, m, nm1)
    bound = fp64_row_bound(l, m, nm1, u, v, w, np.abs(y))
    assert np.all(np.abs(got - ref) <= bound)


FAM_ADJOINT = 3


@pytest.mark.parametrize("ppl,block", [(p, b) for p in (1, 2, 4) for b in (64, 128, 256)])
def test_adjoint_every_shape_group_edges(env, ppl, block):
    """Every compiled tile shape at pixel counts on both sides of the 64-pixel
    groups each wave owns and of the tile width (groups past the last pixel
    are skipped): every pixel against the oracle, FP64 and F32C."""
    torch, swv = env
    ctx = swv.context()
    small = 0   # size class of fewer than 2^20 rows
    saved = ctx.tune_get(FAM_ADJOINT, small)
    rng = np.random.default_rng(1000 * ppl + block)
    n_vis = 777
    u, v, w = (rng.uniform(-3e4, 3e4, n_vis) for _ in range(3))
    y = models.random_complex(n_vis, rng)
    U, V, Wd, Y = dev(u, torch), dev(v, torch), dev(w, torch), dev_c(y, torch)
    tile = ppl * block
    sizes = sorted({1, 63, 64, 65, tile - 1, tile, tile + 1, 2 * tile + 63, 3 * tile - 64})
    try:
        ctx.tune_set(FAM_ADJOINT, small, ppl, block)
        for n_pix in sizes:
            l, m, nm1 = _pixels(rng, n_pix, far=True)
            L, M, N = dev(l, torch), dev(m, torch), dev(nm1, torch)
            got = host(swv.adjoint(U, V, Wd, Y, L, M, N))
            got32 = host(swv.adjoint(U, V, Wd, Y, L, M, N, prec="f32c"))
            swv.synchronize()
            ref = ov.adjoint(u, v, w, y, l, m, nm1)
            bound = fp64_row_bound(l, m, nm1, u, v, w, np.abs(y))
            assert np.all(np.abs(got - ref) <= bound), (ppl, block, n_pix)
            e_max, _ = errors(got32, ref, np.abs(y).sum())
            assert e_max <= TOL32, (ppl, block, n_pix, e_max)
    finally:
        ctx.tune_set(FAM_ADJOINT, small, *saved)


def test_adjoint_cfg5_sampled_pixels(env, cfg5):
    torch, swv = env
    W, u, v, w, y, pix, pl, pm, pn = cfg5
    # the library's pixel set is the oracle's
    lpix, ll, lm, ln = swv.pixels_in_disk(configs.CFG5_J, W.ra_p, W.dec_p,
                                          math.radians(configs.CFG5_DISK_RADIUS_DEG))
    assert np.array_equal(lpix, pix)
    img = swv.adjoint(dev(u, torch), dev(v, torch), dev(w, torch), dev_c(y, torch),
                      dev(ll, torch), dev(lm, torch), dev(ln, torch))
    swv.synchronize()
    sel = np.unique(np.concatenate([[0, pix.size - 1],
                                    np.random.default_rng(5).choice(np.arange(1, pix.size - 1),
                                                                    62, False)]))
    assert sel.size >= 64
    got = host(img)[sel]
    ref = oracle_pool.adjoint(u, v, w, y, pl[sel], pm[sel], pn[sel])
    e_max, e_rms = errors(got, ref, np.abs(y).sum())
    note(f"cfg5 adjoint fp64: {pix.size} pixels, {sel.size} checked over {u.size} rows: "
         f"E_max={e_max:.3e} E_rms={e_rms:.3e}")
    assert e_max <= TOL64


def test_adjoint_f32c_vs_oracle(env, cfg5):
    torch, swv = env
    W, u, v, w, y, pix, pl, pm, pn = cfg5
    n = 1 << 18
    img = swv.adjoint(dev(u[:n], torch), dev(v[:n], torch), dev(w[:n], torch),
                      dev_c(y[:n], torch), dev(pl, torch), dev(pm, torch), dev(pn, torch),
                      prec="f32c")
    swv.synchronize()
    sel = np.arange(0, pix.size, 97)
    ref = ov.adjoint(u[:n], v[:n], w[:n], y[:n], pl[sel], pm[sel], pn[sel], chunk=65536)
    e_max, e_rms = errors(host(img)[sel], ref, np.abs(y[:n]).sum())
    note(f"adjoint f32c ({n} rows): E_max={e_max:.3e} E_rms={e_rms:.3e}")
    assert e_max <= TOL32


def test_adjoint_unit_centre_pixel(env):
    torch, swv = env
    rng = np.random.default_rng(3)
    n = 100003
    u, v, w = (dev(rng.uniform(-1e5, 1e5, n), torch) for _ in range(3))
    ones = torch.ones(n, dtype=torch.complex128, device="cuda")
    z = dev([0.0], torch)
    x = host(swv.adjoint(u, v, w, ones, z, z, z))
    assert x[0] == n


def test_adjoint_identity_on_gpu(env):
    # <A x, y> = <x, A^H y> with A the library's direct sum, A^H its adjoint
    torch, swv = env
    rng = np.random.default_rng(4)
    n, P = 20000, 300
    u, v, w = (rng.uniform(-2e3, 2e3, n) for _ in range(3))
    l, m = rng.uniform(-0.05, 0.05, P), rng.uniform(-0.05, 0.05, P)
    nm1 = ov.n_minus_1(l, m)
    xr, xi = rng.standard_normal(P), rng.standard_normal(P)
    y = models.random_complex(n, rng)
    U, V, W = dev(u, torch), dev(v, torch), dev(w, torch)
    L, M = dev(l, torch), dev(m, torch)
    Ax = host(swv.predict_direct(U, V, W, L, M, dev(xr, torch))) + 1j * host(
        swv.predict_direct(U, V, W, L, M, dev(xi, torch)))
    Ahy = host(swv.adjoint(U, V, W, dev_c(y, torch), L, M, dev(nm1, torch)))
    x = xr + 1j * xi
    lhs, rhs = np.vdot(Ax, y), np.vdot(x, Ahy)
    assert abs(lhs - rhs) <= 1e-12 * np.abs(x).sum() * np.abs(y).sum()


def test_residual_chi2(env):
    torch, swv = env
    rng = np.random.default_rng(6)
    for n in (0, 1, 1000, 3_000_001):
        a = models.random_complex(n, rng)
        b = models.random_complex(n, rng)
        r, chi2 = swv.residual_chi2(dev_c(a, torch), dev_c(b, torch), 1e4)
        swv.synchronize()
        rr, c2 = ov.residual_chi2(a, b, 1e4)
        assert np.array_equal(host(r), rr)
        assert host(chi2)[0] == pytest.approx(c2, rel=1e-13, abs=0)
        r2, chi2b = swv.residual_chi2(dev_c(a, torch), dev_c(b, torch), 1e4)
        assert host(chi2b)[0] == host(chi2)[0]   # fixed reduction order


def _grad_scales(u, v, w, l, m, flux, y):
    """Per-component magnitude sums the gradient errors are measured against:
    sum_j |y_j| for the flux, 2 pi |I| sum_j |y_j|(|u_j| + |w_j l / n|) for l."""
    n = 1 + ov.n_minus_1(l, m)
    ay = np.abs(y)
    s0 = np.full(l.size, ay.sum())
    sl = 2 * np.pi * np.abs(flux) * (ay @ np.abs(u) + (ay @ np.abs(w)) * np.abs(l / n))
    sm = 2 * np.pi * np.abs(flux) * (ay @ np.abs(v) + (ay @ np.abs(w)) * np.abs(m / n))
    phimax = (np.abs(u).max() * np.abs(l) + np.abs(v).max() * np.abs(m)
              + np.abs(w).max() * np.abs(n - 1))
    rel = 2 * np.pi * 3 * U_R * phimax + 1e-14
    return s0 * rel, sl * rel, sm * rel


@pytest.mark.parametrize("alpha", [1.0, -2e4])
def test_grad_small_vs_oracle(env, alpha):
    torch, swv = env
    rng = np.random.default_rng(7)
    n, K = 5001, 70
    u, v, w = (rng.uniform(-5e4, 5e4, n) for _ in range(3))
    l, m = rng.uniform(-0.03, 0.03, K), rng.uniform(-0.03, 0.03, K)
    f = rng.lognormal(-3, 1, K)
    y = models.random_complex(n, rng)
    got = [host(g) for g in swv.grad_direct(dev(u, torch), dev(v, torch), dev(w, torch),
                                             dev_c(y, torch), dev(l, torch), dev(m, torch),
                                             dev(f, torch), alpha=alpha)]
    ref = ov.grad_direct(u, v, w, y, l, m, f, alpha=alpha)
    for g, r, s in zip(got, ref, _grad_scales(u, v, w, l, m, f, y)):
        assert np.all(np.abs(g - r) <= abs(alpha) * s)


FAM_GRAD = 4


@pytest.mark.parametrize("cpl", [1, 2, 4])
def test_grad_every_shape_component_edges(env, cpl):
    """Each components-per-lane shape at component counts on both sides of the
    block widths it picks (128 .. 1024 threads) and of several tiles: every
    component's three gradients against the oracle."""
    torch, swv = env
    ctx = swv.context()
    small = 0   # size class of fewer than 2^20 rows
    saved = ctx.tune_get(FAM_GRAD, small)
    rng = np.random.default_rng(40 + cpl)
    n = 613
    u, v, w = (rng.uniform(-5e4, 5e4, n) for _ in range(3))
    y = models.random_complex(n, rng)
    U, V, Wd, Y = dev(u, torch), dev(v, torch), dev(w, torch), dev_c(y, torch)
    sizes = sorted({1, 63, 65, 128 * cpl - 1, 128 * cpl + 1, 1024 * cpl, 1024 * cpl + 1,
                    2048 * cpl + 63})
    try:
        ctx.tune_set(FAM_GRAD, small, cpl, 128)
        for K in sizes:
            l, m = rng.uniform(-0.03, 0.03, K), rng.uniform(-0.03, 0.03, K)
            f = rng.lognormal(-3, 1, K)
            got = [host(g) for g in swv.grad_direct(U, V, Wd, Y, dev(l, torch), dev(m, torch),
                                                     dev(f, torch), alpha=-2.0)]
            swv.synchronize()
            ref = ov.grad_direct(u, v, w, y, l, m, f, alpha=-2.0)
            for g, r, sc in zip(got, ref, _grad_scales(u, v, w, l, m, f, y)):
                assert np.all(np.abs(g - r) <= 2.0 * sc), (cpl, K)
    finally:
        ctx.tune_set(FAM_GRAD, small, *saved)


def test_grad_cfg5_sampled_components(env, cfg5):
    torch, swv = env
    W, u, v, w, y, *_ = cfg5
    l, m, f = W.components()
    alpha = -2.0 / configs.CFG5_NOISE_SIGMA ** 2
    got = [host(g) for g in swv.grad_direct(dev(u, torch), dev(v, torch), dev(w, torch),
                                             dev_c(y, torch), dev(l, torch), dev(m, torch),
                                             dev(f, torch), alpha=alpha)]
    swv.synchronize()
    sel = np.random.default_rng(9).choice(l.size, 64, False)
    ref = oracle_pool.grad_direct(u, v, w, y, l[sel], m[sel], f[sel], alpha)
    scales = _grad_scales(u, v, w, l[sel], m[sel], f[sel], y)
    for name, g, r, s in zip(("flux", "l", "m"), got, ref, scales):
        used = np.max(np.abs(g[sel] - r) / (abs(alpha) * s))
        note(f"cfg5 grad d/d{name}: max |gpu - oracle| is {used:.3e} of the derived bound")
        assert used <= 1.0


def test_cfg5_residual_image_and_gradients_vs_oracle(env, cfg5):
    # Config 5's own residual: the perturbed model (fluxes x (1 + N(0, 0.05)),
    # positions + N(0, 1")) plus complex noise (sigma 0.01 Jy), minus the
    # model, made by the oracle.  On one GPU's share of the rows under the
    # 8-way row sharding of the design (the first 32 of 256 time samples,
    # 1,044,480 rows): the full-size residual would cost the oracle 3.3e10
    # terms.  Every pixel and component on the GPU, 64 of each against the
    # oracle.
    torch, swv = env
    W, u_all, v_all, w_all, noise, pix, pl, pm, pn = cfg5
    n = u_all.size // 8
    u, v, w = u_all[:n], v_all[:n], w_all[:n]
    note(f"cfg5 residual on {n} rows: oracle in {oracle_pool.n_workers()} processes ...")
    y = oracle_pool.cfg5_residual(np.arange(n), noise[:n])
    l, m, f = W.components()
    alpha = -2.0 / configs.CFG5_NOISE_SIGMA ** 2
    U, V, Wt, Y = dev(u, torch), dev(v, torch), dev(w, torch), dev_c(y, torch)
    img = host(swv.adjoint(U, V, Wt, Y, dev(pl, torch), dev(pm, torch), dev(pn, torch)))
    grads = [host(g) for g in swv.grad_direct(U, V, Wt, Y, dev(l, torch), dev(m, torch),
                                               dev(f, torch), alpha=alpha)]
    swv.synchronize()
    rng = np.random.default_rng(55)
    ps = np.sort(rng.choice(pix.size, 64, False))
    ref = oracle_pool.adjoint(u, v, w, y, pl[ps], pm[ps], pn[ps])
    bound = fp64_row_bound(pl[ps], pm[ps], pn[ps], u, v, w, np.abs(y))
    e_img, _ = errors(img[ps], ref, np.abs(y).sum())
    assert np.all(np.abs(img[ps] - ref) <= bound)
    assert e_img <= TOL64
    ks = np.sort(rng.choice(l.size, 64, False))
    refg = oracle_pool.grad_direct(u, v, w, y, l[ks], m[ks], f[ks], alpha)
    worst = 0.0
    for name, g, r, sc in zip(("flux", "l", "m"), grads, refg,
                              _grad_scales(u, v, w, l[ks], m[ks], f[ks], y)):
        used = np.max(np.abs(g[ks] - r) / (abs(alpha) * sc))
        worst = max(worst, used)
        assert used <= 1.0, name
    note(f"cfg5 residual: |r| rms {np.sqrt(np.mean(np.abs(y) ** 2)):.3e}; image E_max "
         f"{e_img:.2e} over 64 pixels; gradients at most {worst:.2f} of the derived bound over "
         "64 components")


def test_grad_matches_finite_differences_of_gpu_chi2(env):
    # central differences of the library's own chi^2 (product path only)
    torch, swv = env
    W = configs.CFG2
    u, v, w = (dev(a[:400000], torch) for a in W.track.uvw())
    l, m, f = W.components()
    rng = np.random.default_rng(11)
    l2, m2, f2 = models.perturb_model(l, m, f, rng)
    inv_s2 = 1.0 / configs.CFG5_NOISE_SIGMA ** 2
    obs = swv.predict_direct(u, v, w, dev(l2, torch), dev(m2, torch), dev(f2, torch)) + \
        dev_c(models.complex_noise(u.numel(), configs.CFG5_NOISE_SIGMA, rng), torch)

    def chi2(ll, mm, ff):
        V = swv.predict_direct(u, v, w, dev(ll, torch), dev(mm, torch), dev(ff, torch))
        return float(host(swv.residual_chi2(obs, V, inv_s2)[1])[0])

    V0 = swv.predict_direct(u, v, w, dev(l, torch), dev(m, torch), dev(f, torch))
    r, _ = swv.residual_chi2(obs, V0, inv_s2)
    gI, gl, gm = (host(g) for g in swv.grad_direct(u, v, w, r, dev(l, torch), dev(m, torch),
                                                    dev(f, torch), alpha=-2 * inv_s2))
    for k in rng.choice(l.size, 4, False):
        def fd(which, h):
            def at(d):
                ll, mm, ff = l.copy(), m.copy(), f.copy()
                {"l": ll, "m": mm, "f": ff}[which][k] += d
                return chi2(ll, mm, ff)
            return (at(h) - at(-h)) / (2 * h)
        assert fd("f", 1e-6) == pytest.approx(gI[k], rel=1e-6, abs=1e-6 * np.abs(gI).max())
        for which, g, gall in (("l", gl[k], gl), ("m", gm[k], gm)):
            h = 1e-8
            rich = (4 * fd(which, h / 2) - fd(which, h)) / 3
            assert rich == pytest.approx(g, rel=1e-4, abs=1e-5 * np.abs(gall).max())
