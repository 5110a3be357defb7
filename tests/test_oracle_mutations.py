"""Planted mistakes in the oracle (CPU only): each plausible bug must make at
least one of the pins fail, so the pins are not vacuous."""
import numpy as np
import pytest

from oracle import sphere as sp
from oracle import tree as ot
from oracle import visibility as ov

from . import test_oracle_adjoint as TA
from . import test_oracle_direct as TD
from . import test_oracle_sphere as TS
from . import test_oracle_tree as TT

_orig_phase = ov.reduced_phase


def _phase_without_w(u, v, w, l, m, nm1):
    return _orig_phase(u, v, 0.0 * w, l, m, nm1)


def _phase_u_v_swapped(u, v, w, l, m, nm1):
    return _orig_phase(v, u, w, l, m, nm1)


def _phase_m_sign(u, v, w, l, m, nm1):
    return _orig_phase(u, v, w, l, -m, nm1)


@pytest.mark.parametrize("bad,pin", [
    (_phase_without_w, TD.test_pythagorean_directions_w_term),
    (_phase_u_v_swapped, TD.test_small_field_grid_equals_fft),
    (_phase_m_sign, TD.test_small_field_grid_equals_fft),
])
def test_phase_mutations_caught(monkeypatch, bad, pin):
    monkeypatch.setattr(ov, "reduced_phase", bad)
    with pytest.raises(AssertionError):
        pin()


def test_ignored_sign_caught(monkeypatch):
    orig = ov.phasors
    monkeypatch.setattr(ov, "phasors", lambda *a, **k: orig(*a[:6], sign=1))
    with pytest.raises(AssertionError):
        TD.test_small_field_grid_equals_fft()


def test_adjoint_missing_conjugate_caught(monkeypatch):
    def bad(u, v, w, y, l, m, nm1, sign=-1, chunk=2048):
        e = ov.phasors(u, v, w, l, m, nm1, sign)
        return e.T @ np.asarray(y, complex)
    monkeypatch.setattr(ov, "adjoint", bad)
    with pytest.raises(AssertionError):
        TA.test_adjoint_identity_complex(-1)


def test_gradient_missing_w_term_caught(monkeypatch):
    orig = ov.grad_direct

    def bad(u, v, w, y, l, m, flux, sign=-1, alpha=1.0, chunk=2048):
        # position derivative without the dn/dl = -l/n part
        gI, _, _ = orig(u, v, w, y, l, m, flux, sign, alpha, chunk)
        _, gl, gm = orig(u, v, 0 * np.asarray(w), y, l, m, flux, sign, alpha, chunk)
        return gI, gl, gm
    monkeypatch.setattr(ov, "grad_direct", bad)
    with pytest.raises(AssertionError):
        TA.test_backward_convention_real_loss()


def test_wrong_wavelet_scale_caught(monkeypatch):
    orig = sp.pixel_area
    calls = {"n": 0}

    def area_off_by_level(j):
        # sqrt(A_{j+1}) instead of sqrt(A_j) inside the coefficient recursion
        return orig(j + 1) if j < 30 else orig(j)
    orig_build = ot.build_levels

    def bad_levels(J, pix, F):
        monkeypatch.setattr(sp, "pixel_area", area_off_by_level)
        try:
            out = orig_build(J, pix, F)
        finally:
            monkeypatch.setattr(sp, "pixel_area", orig)
        calls["n"] += 1
        # restore lambda_J normalisation so only the gamma scale is wrong
        out[-1].lam = F / orig(J)
        return out
    monkeypatch.setattr(ot, "build_levels", bad_levels)
    with pytest.raises(AssertionError):
        TT.test_eq17_equals_snapped_direct(5, -1)
    assert calls["n"] > 0


def test_missing_A1_factor_caught(monkeypatch):
    def bad(tree, eta, sig):
        V = eta[0] @ tree.levels[0].lam
        for j in range(1, tree.J):
            V = V + np.einsum("rkm,km->r", sig[j - 1], tree.levels[j - 1].gamma)
        return V
    monkeypatch.setattr(ot, "reconstruct", bad)
    with pytest.raises(AssertionError):
        TT.test_eq17_equals_snapped_direct(5, -1)


def test_swapped_sign_rows_caught(monkeypatch, golden):
    monkeypatch.setattr(ot, "WAVELET_SIGNS", ot.WAVELET_SIGNS[[1, 0, 2]])
    with pytest.raises(AssertionError):
        TT.test_sign_table_matches_eq10(golden)


def test_swapped_in_face_axes_caught(monkeypatch):
    orig_i, orig_d = sp._interleave, sp._deinterleave
    monkeypatch.setattr(sp, "_interleave", lambda ix, iy, b: orig_i(iy, ix, b))
    monkeypatch.setattr(sp, "_deinterleave", lambda p, b: orig_d(p, b)[::-1])
    with pytest.raises(AssertionError):
        TS.test_nested_child_layout()


def test_wrong_south_face_offset_caught(monkeypatch):
    orig = sp.ang2pix_xyz

    def bad(j, xyz):
        p = orig(j, xyz)
        nside2 = 1 << (2 * (j - 1))
        face = p // nside2
        return np.where(face >= 8, p - 4 * nside2, p)
    monkeypatch.setattr(sp, "ang2pix_xyz", bad)
    with pytest.raises(AssertionError):
        TS.test_round_trip_every_pixel(3)
