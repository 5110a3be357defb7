"""Pins of the oracle's adjoint and gradients: the adjoint identity, closed
forms, the FFT special case and central finite differences."""
import numpy as np
import pytest

from oracle import visibility as ov


def _setup(seed, n_vis=300, n_comp=12, uv=2e3, half=0.03):
    rng = np.random.default_rng(seed)
    u, v, w = (rng.uniform(-uv, uv, n_vis) for _ in range(3))
    l, m = rng.uniform(-half, half, n_comp), rng.uniform(-half, half, n_comp)
    return rng, u, v, w, l, m


@pytest.mark.parametrize("sign", [-1, 1])
def test_adjoint_identity_complex(sign):
    rng, u, v, w, l, m = _setup(1)
    nm1 = ov.n_minus_1(l, m)
    x = rng.standard_normal(l.size) + 1j * rng.standard_normal(l.size)
    y = rng.standard_normal(u.size) + 1j * rng.standard_normal(u.size)
    Ax = ov.predict_direct(u, v, w, l, m, x, sign, nm1=nm1)
    Ahy = ov.adjoint(u, v, w, y, l, m, nm1, sign)
    lhs = np.vdot(Ax, y)          # <Ax, y>, conjugate-linear in the first slot
    rhs = np.vdot(x, Ahy)
    assert abs(lhs - rhs) <= 1e-12 * np.abs(x).sum() * np.abs(y).sum()


def test_adjoint_identity_real_restricted():
    rng, u, v, w, l, m = _setup(2)
    nm1 = ov.n_minus_1(l, m)
    x = rng.standard_normal(l.size)
    y = rng.standard_normal(u.size) + 1j * rng.standard_normal(u.size)
    lhs = np.real(np.vdot(ov.predict_direct(u, v, w, l, m, x, nm1=nm1), y))
    rhs = np.dot(x, np.real(ov.adjoint(u, v, w, y, l, m, nm1)))
    assert abs(lhs - rhs) <= 1e-12 * np.abs(x).sum() * np.abs(y).sum()


def test_adjoint_unit_centre_source():
    _, u, v, w, _, _ = _setup(3, n_vis=777)
    x = ov.adjoint(u, v, w, np.ones(u.size, complex), [0.0], [0.0], [0.0])
    assert x[0] == 777.0


def test_adjoint_grid_equals_inverse_fft():
    N, K = 8, 4
    rng = np.random.default_rng(4)
    y = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    uu, vv = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    u, v = (uu.ravel() * K).astype(float), (vv.ravel() * K).astype(float)
    w = np.zeros_like(u)
    p, q = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    l, m = (p / (N * K)).ravel(), (q / (N * K)).ravel()
    x = ov.adjoint(u, v, w, y.ravel(), l, m, ov.n_minus_1(l, m), sign=-1)
    ref = np.fft.ifft2(y) * N * N
    assert np.max(np.abs(x - ref.ravel())) < 1e-12 * np.abs(y).sum()


def _chi2(u, v, w, l, m, f, obs, inv_s2):
    return ov.residual_chi2(obs, ov.predict_direct(u, v, w, l, m, f), inv_s2)[1]


def test_flux_gradient_is_adjoint_closed_form():
    rng, u, v, w, l, m = _setup(5)
    f = rng.lognormal(-3, 1, l.size)
    r = rng.standard_normal(u.size) + 1j * rng.standard_normal(u.size)
    inv_s2 = 1e4
    gI, _, _ = ov.grad_direct(u, v, w, r, l, m, f, alpha=-2 * inv_s2)
    ref = -2 * inv_s2 * np.real(ov.adjoint(u, v, w, r, l, m, ov.n_minus_1(l, m)))
    assert np.max(np.abs(gI - ref)) < 1e-12 * np.abs(ref).max()


def test_gradients_match_central_differences():
    rng, u, v, w, l, m = _setup(6, n_vis=200, n_comp=6, uv=3e3)
    f = rng.lognormal(-3, 1, l.size)
    obs = ov.predict_direct(u, v, w, l + 1e-5, m - 2e-5, f * 1.1) + 0.01 * (
        rng.standard_normal(u.size) + 1j * rng.standard_normal(u.size))
    inv_s2 = 1e4
    obs_r = obs - ov.predict_direct(u, v, w, l, m, f)
    gI, gl, gm = ov.grad_direct(u, v, w, obs_r, l, m, f, alpha=-2 * inv_s2)
    for k in range(l.size):
        def fd(param, h):
            def at(delta):
                ll, mm, ff = l.copy(), m.copy(), f.copy()
                {"l": ll, "m": mm, "f": ff}[param][k] += delta
                return _chi2(u, v, w, ll, mm, ff, obs, inv_s2)
            return (at(h) - at(-h)) / (2 * h)
        # chi^2 is quadratic in the fluxes: central FD is exact up to rounding
        assert fd("f", 1e-6) == pytest.approx(gI[k], rel=1e-6)
        for name, g in (("l", gl[k]), ("m", gm[k])):
            h = 1e-7
            rich = (4 * fd(name, h / 2) - fd(name, h)) / 3
            assert rich == pytest.approx(g, rel=1e-5, abs=1e-6 * abs(g) + 1e-3)


def test_backward_convention_real_loss():
    # alpha = 1, y = dL/dV*: gradient of L = Re sum conj(y) V(theta)
    rng, u, v, w, l, m = _setup(7, n_comp=4)
    f = rng.lognormal(-3, 1, l.size)
    y = rng.standard_normal(u.size) + 1j * rng.standard_normal(u.size)
    gI, gl, gm = ov.grad_direct(u, v, w, y, l, m, f, alpha=1.0)

    def L(ll, mm, ff):
        return np.real(np.vdot(y, ov.predict_direct(u, v, w, ll, mm, ff)))
    h = 1e-7
    for k in range(l.size):
        e = np.zeros(l.size)
        e[k] = h
        assert (L(l, m, f + e) - L(l, m, f - e)) / (2 * h) == pytest.approx(gI[k], rel=1e-6)
        assert (L(l + e, m, f) - L(l - e, m, f)) / (2 * h) == pytest.approx(gl[k], rel=1e-4)
        assert (L(l, m + e, f) - L(l, m - e, f)) / (2 * h) == pytest.approx(gm[k], rel=1e-4)


def test_zero_residual_zero_gradient():
    rng, u, v, w, l, m = _setup(8)
    f = rng.lognormal(-3, 1, l.size)
    obs = ov.predict_direct(u, v, w, l, m, f)
    r, chi2 = ov.residual_chi2(obs, ov.predict_direct(u, v, w, l, m, f), 1e4)
    assert chi2 == 0.0
    g = ov.grad_direct(u, v, w, r, l, m, f, alpha=-2e4)
    assert all(np.all(x == 0) for x in g)
