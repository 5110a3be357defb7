"""Pins of the oracle's direct sum (Eq. 12) against closed forms, a library
FFT and 50-digit brute force.  CPU only."""
import mpmath
import numpy as np
import pytest

from oracle import visibility as ov


def _rng(s):
    return np.random.default_rng(s)


def test_unit_source_at_phase_centre_is_one():
    rng = _rng(1)
    u, v, w = (rng.uniform(-1e5, 1e5, 500) for _ in range(3))
    V = ov.predict_direct(u, v, w, [0.0], [0.0], [1.0])
    assert np.all(V == 1.0 + 0.0j)


@pytest.mark.parametrize("sign", [-1, 1])
def test_shifted_source_unit_modulus_and_character(sign):
    # A single source is a character of the additive group of baselines:
    # |V| = 1, V(0) = 1, V(B1 + B2) = V(B1) V(B2), V(-B) = conj V(B).
    rng = _rng(2)
    l, m = np.array([0.013]), np.array([-0.021])
    B1 = rng.integers(-20000, 20000, (3, 200)).astype(float)
    B2 = rng.integers(-20000, 20000, (3, 200)).astype(float)
    V1 = ov.predict_direct(*B1, l, m, [1.0], sign)
    V2 = ov.predict_direct(*B2, l, m, [1.0], sign)
    V12 = ov.predict_direct(*(B1 + B2), l, m, [1.0], sign)
    Vn = ov.predict_direct(*(-B1), l, m, [1.0], sign)
    assert np.max(np.abs(np.abs(V1) - 1)) < 1e-15
    assert np.max(np.abs(V12 - V1 * V2)) < 2e-14
    assert np.max(np.abs(Vn - np.conj(V1))) < 1e-14
    V0 = ov.predict_direct([0.0], [0.0], [0.0], l, m, [1.0], sign)
    assert V0[0] == 1.0


def test_small_field_grid_equals_fft():
    # Eq. 2 (w = 0): sources on the grid l = p/N, m = q/N and integer (u, v)
    # make the direct sum the 2-D DFT; s = -1 is numpy's forward FFT.
    N = 16
    rng = _rng(3)
    I = rng.lognormal(-3, 1, (N, N))
    p, q = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    # l = p/(N K), u = K x integer: u l = (integer) p / N, directions stay
    # well inside the unit disk
    K = 4
    l = (p / (N * K)).ravel()
    m = (q / (N * K)).ravel()
    uu, vv = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    u = (uu.ravel() * K).astype(float)
    v = (vv.ravel() * K).astype(float)
    w = np.zeros_like(u)
    V = ov.predict_direct(u, v, w, l, m, I.ravel(), sign=-1)
    F = np.fft.fft2(I)
    assert np.max(np.abs(V - F.ravel())) < 1e-12 * np.sum(I)


def test_pythagorean_directions_w_term():
    # l = 3/5, m = 0 -> n = 4/5, n - 1 = -1/5; l = 0, m = 5/13 -> n = 12/13.
    # Choosing (u, v, w) so that every phase is an integer gives V = 1.
    cases = [((3 / 5, 0.0), (5.0, 0.0, 5.0)), ((0.0, 5 / 13), (0.0, 13.0, 13.0)),
             ((3 / 5, 0.0), (10.0, 0.0, 15.0))]
    for (l, m), (u, v, w) in cases:
        V = ov.predict_direct([u], [v], [w], [l], [m], [1.0])
        assert abs(V[0] - 1.0) < 1e-13
    # half-integer phase gives -1: l = 3/5, u = 5, w = 5/2 -> 3 - 1/2
    V = ov.predict_direct([5.0], [0.0], [2.5], [0.6], [0.0], [1.0])
    assert abs(V[0] + 1.0) < 1e-13


@pytest.mark.parametrize("sign", [-1, 1])
def test_hermitian_and_sign_flip(sign):
    rng = _rng(4)
    u, v, w = (rng.uniform(-5e4, 5e4, 300) for _ in range(3))
    l, m = rng.uniform(-0.02, 0.02, 40), rng.uniform(-0.02, 0.02, 40)
    I = rng.lognormal(-3, 1, 40)
    V = ov.predict_direct(u, v, w, l, m, I, sign)
    Vneg = ov.predict_direct(-u, -v, -w, l, m, I, sign)
    Vflip = ov.predict_direct(u, v, w, l, m, I, -sign)
    assert np.max(np.abs(Vneg - np.conj(V))) < 1e-14 * I.sum()
    assert np.max(np.abs(Vflip - np.conj(V))) < 1e-14 * I.sum()


def test_linearity():
    rng = _rng(5)
    u, v, w = (rng.uniform(-5e4, 5e4, 100) for _ in range(3))
    l, m = rng.uniform(-0.02, 0.02, 30), rng.uniform(-0.02, 0.02, 30)
    a, b = rng.standard_normal(30), rng.standard_normal(30)
    Va = ov.predict_direct(u, v, w, l, m, a)
    Vb = ov.predict_direct(u, v, w, l, m, b)
    Vab = ov.predict_direct(u, v, w, l, m, 2 * a - 3 * b)
    assert np.max(np.abs(Vab - (2 * Va - 3 * Vb))) < 1e-13 * (np.abs(a).sum() + np.abs(b).sum()) * 5


def _mp_visibility(u, v, w, l, m, I, sign, nm1=None):
    """50-digit V; n - 1 exact from (l, m) unless FP64 values are given."""
    mpmath.mp.dps = 50
    out = []
    for j in range(len(u)):
        acc = mpmath.mpc(0)
        for k in range(len(l)):
            lk, mk = mpmath.mpf(l[k]), mpmath.mpf(m[k])
            if nm1 is None:
                q = mpmath.sqrt(1 - lk * lk - mk * mk) - 1
            else:
                q = mpmath.mpf(nm1[k])
            ph = mpmath.mpf(u[j]) * lk + mpmath.mpf(v[j]) * mk + mpmath.mpf(w[j]) * q
            acc += mpmath.mpf(I[k]) * mpmath.expjpi(2 * sign * ph)
        out.append(complex(acc))
    return np.array(out)


def _brute_inputs():
    rng = _rng(6)
    u = rng.uniform(-4e5, 4e5, 64)
    v = rng.uniform(-4e5, 4e5, 64)
    w = rng.uniform(-3e5, 3e5, 64)
    l = rng.uniform(-0.03, 0.03, 16)
    m = rng.uniform(-0.03, 0.03, 16)
    I = rng.lognormal(-3, 1, 16)
    return u, v, w, l, m, I


@pytest.mark.parametrize("sign", [-1, 1])
def test_brute_force_50_digits_same_inputs(sign):
    # The oracle's arithmetic on its FP64 inputs (l, m, n - 1): |phi| up to
    # ~2e4 cycles, where an FP64 ulp of phi is ~4e-12 cycles; the oracle
    # reduces phi exactly, so only sincos and the sum round.
    u, v, w, l, m, I = _brute_inputs()
    nm1 = ov.n_minus_1(l, m)
    ref = _mp_visibility(u, v, w, l, m, I, sign, nm1=nm1)
    got = ov.predict_direct(u, v, w, l, m, I, sign)
    err = np.max(np.abs(got - ref)) / I.sum()
    assert err < 2e-15, err


@pytest.mark.parametrize("sign", [-1, 1])
def test_brute_force_50_digits_exact_definition(sign):
    # Against Eq. 12 with n - 1 exact: the only extra error is the FP64
    # rounding of n - 1 (a few ulp of |n - 1| <= 1e-3) times |w| <= 3e5.
    u, v, w, l, m, I = _brute_inputs()
    ref = _mp_visibility(u, v, w, l, m, I, sign)
    got = ov.predict_direct(u, v, w, l, m, I, sign)
    nm1 = np.abs(ov.n_minus_1(l, m))
    bound = 2 * np.pi * np.max(np.abs(w)) * 4 * np.max(np.spacing(nm1)) + 2e-15
    err = np.max(np.abs(got - ref)) / I.sum()
    assert err < bound, (err, bound)


def test_reduced_phase_is_exact_mod_one():
    mpmath.mp.dps = 60
    rng = _rng(7)
    for _ in range(200):
        u, v, w = rng.uniform(-5e5, 5e5, 3)
        l, m = rng.uniform(-0.05, 0.05, 2)
        nm1 = float(ov.n_minus_1(l, m))
        r = float(ov.reduced_phase(u, v, w, l, m, nm1))
        ph = mpmath.mpf(u) * mpmath.mpf(l) + mpmath.mpf(v) * mpmath.mpf(m) + mpmath.mpf(w) * mpmath.mpf(nm1)
        ref = ph - mpmath.nint(ph)
        d = abs(mpmath.mpf(r) - ref)
        d = min(d, abs(1 - d))
        assert d < 4e-16


def test_n_minus_1_stable_form():
    mpmath.mp.dps = 50
    for l, m in [(1e-9, 2e-9), (0.01, -0.02), (0.3, 0.4), (0.6, 0.0)]:
        ref = mpmath.sqrt(1 - mpmath.mpf(l) ** 2 - mpmath.mpf(m) ** 2) - 1
        got = float(ov.n_minus_1(l, m))
        assert abs(got - float(ref)) <= 2e-16 * abs(float(ref))


def test_residual_chi2_closed_form():
    rng = _rng(8)
    obs = rng.integers(-100, 100, 1000) + 1j * rng.integers(-100, 100, 1000)
    r, chi2 = ov.residual_chi2(obs, obs - (3 + 4j), 1e4)
    assert np.all(r == 3 + 4j)
    assert abs(chi2 - 1000 * 25 * 1e4) < 1e-6


def test_plain_fp64_phase_form_agrees_with_the_exact_one():
    # predict_direct_fp64 (plain FP64 phase) against predict_direct (error-free
    # phase products): within the phase rounding 2 pi 3 2^-53 |phi| per term,
    # and the closed forms hold for it too
    from oracle import visibility as ov
    rng = np.random.default_rng(41)
    u, v, w = (rng.uniform(-1e5, 1e5, 3000) for _ in range(3))
    l, m = rng.uniform(-0.05, 0.05, 70), rng.uniform(-0.05, 0.05, 70)
    f = rng.lognormal(-3, 1, 70)
    a = ov.predict_direct_fp64(u, v, w, l, m, f)
    b = ov.predict_direct(u, v, w, l, m, f)
    nm1 = ov.n_minus_1(l, m)
    phi = np.abs(np.outer(u, l)) + np.abs(np.outer(v, m)) + np.abs(np.outer(w, nm1))
    bound = (2 * np.pi * 3 * 2.0 ** -53 * phi + 1e-15) @ f
    assert np.all(np.abs(a - b) <= bound)
    one = ov.predict_direct_fp64(u, v, w, np.zeros(1), np.zeros(1), np.ones(1))
    assert np.all(one == 1.0)
    assert np.allclose(ov.predict_direct_fp64(u, v, w, l, m, f, sign=1),
                       np.conj(a), rtol=0, atol=1e-13)
