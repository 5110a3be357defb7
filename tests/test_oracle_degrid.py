"""CPU pins of oracle/degrid.py, the FFT + degridding comparator.

The degridder approximates the direct sum over the image pixels; what fixes
it is that its error against that sum (oracle.visibility.predict_direct,
pinned on its own) falls with the kernel width W and stays below 10^(2 - W)
of sum |I|, on a narrow field and on a wide one where the w-term is several
turns; the phase sign flips to the complex conjugate; the kernel transform's
quadrature has converged.
"""
import numpy as np
import pytest

from oracle import clean as oc
from oracle import degrid as od
from oracle import visibility as ov
from synth.configs import TrackSpec

TRACK = TrackSpec(27, 1.7e3, 45.0, 2016.0, 4, 1.0e7, seed=731)


@pytest.fixture(scope="module")
def track():
    return TRACK.uvw()


def _model(nx, ny, k, seed):
    rng = np.random.default_rng(seed)
    img = np.zeros((ny, nx))
    idx = rng.choice(nx * ny, k, replace=False)
    img.flat[idx] = rng.uniform(-0.3, 1.0, k)
    return img, idx


def _exact(u, v, w, img, idx, cell, sign=-1):
    ny, nx = img.shape
    l, m, nm1, _ = oc.image_grid(nx, ny, cell)
    return ov.predict_direct(u, v, w, l[idx], m[idx], img.flat[idx], sign)


def test_error_falls_with_support(track):
    u, v, w = track
    img, idx = _model(32, 24, 10, 1)
    exact = _exact(u, v, w, img, idx, 0.006)
    scale = np.abs(img).sum()
    errs = []
    for W in (4, 6, 8, 10, 12, 14):
        e = np.abs(od.predict_degrid(img, 0.006, u, v, w, W) - exact).max() / scale
        assert e <= 10.0 ** (2 - W), (W, e)
        errs.append(e)
    assert all(b < a for a, b in zip(errs, errs[1:]))


def test_wide_field_w_term(track):
    u, v, w = track
    nx = ny = 24
    cell = 0.02                      # |l| to 0.24: n - 1 to -0.06, w (n - 1) several turns
    img, idx = _model(nx, ny, 12, 2)
    exact = _exact(u, v, w, img, idx, cell)
    P = od.plan(nx, ny, cell, w, 12)
    assert P["n_planes"] > 12 and abs(w).max() * abs(P["nm1"]).max() > 1.0
    e = np.abs(od.predict_degrid(img, cell, u, v, w, 12) - exact).max() / np.abs(img).sum()
    assert e <= 1e-10


def test_centre_source_and_sign(track):
    u, v, w = track
    img = np.zeros((16, 16))
    img[8, 8] = 2.0
    got = od.predict_degrid(img, 0.01, u, v, w, 12)
    assert np.abs(got - 2.0).max() <= 2.0 * 1e-10
    img2, idx = _model(20, 18, 6, 3)
    a = od.predict_degrid(img2, 0.01, u, v, w, 10, sign=-1)
    b = od.predict_degrid(img2, 0.01, u, v, w, 10, sign=+1)
    assert np.abs(a - np.conj(b)).max() <= 1e-13 * np.abs(img2).sum()
    exact = _exact(u, v, w, img2, idx, 0.01, sign=+1)
    assert np.abs(b - exact).max() <= 1e-8 * np.abs(img2).sum()


def test_kernel_transform_quadrature_converged():
    f = np.linspace(-0.3, 0.3, 41)
    for W in (4, 10, 16):
        a = od.es_hat(f, W, 100)
        b = od.es_hat(f, W, 150)
        assert np.abs(a - b).max() <= 2e-14 * np.abs(b).max()
        assert np.all(a > 0)
