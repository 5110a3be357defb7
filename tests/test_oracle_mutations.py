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


def _swap_east_west(pix, j, rows):
    """Pixel ids with children 1 and 2 exchanged at every level inside the
    base pixels of `rows` (0 north, 1 equatorial, 2 south)."""
    pix = np.asarray(pix, dtype=np.int64)
    face = pix >> (2 * (j - 1))
    low = pix & ((1 << (2 * (j - 1))) - 1)
    swapped = np.zeros_like(low)
    for b in range(j - 1):
        c = (low >> (2 * b)) & 3
        c = np.where(c == 1, 2, np.where(c == 2, 1, c))
        swapped |= c << (2 * b)
    return np.where(np.isin(face // 4, rows), (face << (2 * (j - 1))) | swapped, pix)


def _plant_transposition(monkeypatch, rows):
    orig_a, orig_c = sp.ang2pix_xyz, sp.pixel_plane_centre
    monkeypatch.setattr(sp, "ang2pix_xyz",
                        lambda j, xyz: _swap_east_west(orig_a(j, xyz), j, rows))
    monkeypatch.setattr(sp, "pixel_plane_centre",
                        lambda j, pix: orig_c(j, _swap_east_west(pix, j, rows)))


def test_swapped_in_face_axes_caught(monkeypatch):
    # ix and iy transposed in every base pixel
    _plant_transposition(monkeypatch, [0, 1, 2])
    TS.test_round_trip_every_pixel(3)         # still a consistent pixelisation
    with pytest.raises(AssertionError):
        TS.test_nested_child_layout()


def test_south_face_transposition_caught(monkeypatch):
    # ix and iy transposed inside the south-row base pixels only, consistently
    # in ang2pix and the centres: a valid equal-area nested pixelisation that
    # differs from HEALPix NESTED only in the labels of the southern children,
    # so V is unchanged but the Eq. 10 coefficients of those nodes are not.
    _plant_transposition(monkeypatch, [2])
    for j in (2, 3, 4):
        TS.test_round_trip_every_pixel(j)
        TS.test_centres_are_the_ring_scheme_centres(j)
    TS.test_children_centres_inside_parent(3)
    TS.test_nested_parent_rule_random_points()
    TS.test_equal_area_monte_carlo()
    with pytest.raises(AssertionError):
        TS.test_nested_child_layout()
    with pytest.raises(AssertionError):
        TS.test_level2_children_closed_form()
    with pytest.raises(AssertionError):
        TS.test_child_layout_every_pixel(3)


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


# ------------------------------------------------- clean loop, degridding --
from oracle import clean as oc  # noqa: E402
from oracle import degrid as od  # noqa: E402

from . import test_oracle_clean as TC  # noqa: E402
from . import test_oracle_degrid as TG  # noqa: E402


def _hogbom_variant(mirror=False, record_peak=False, last_tie=False, add=False):
    def bad(image, beam, gain, threshold, max_iter, absolute=False):
        I = np.array(image, dtype=np.float64, copy=True)
        ny, nx = I.shape
        B = np.asarray(beam, np.float64)
        pix, val = [], []
        for _ in range(int(max_iter)):
            key = np.abs(I) if absolute else I
            flat = key.ravel()
            p = int(flat.size - 1 - np.argmax(flat[::-1])) if last_tie else int(np.argmax(flat))
            if not flat[p] > threshold:
                break
            py, px = divmod(p, nx)
            gC = gain * I.flat[p]
            win = B[ny - 1 - py:2 * ny - 1 - py, nx - 1 - px:2 * nx - 1 - px]
            if mirror:
                win = win[::-1, ::-1]
            I = I + gC * win if add else I - gC * win
            pix.append(p)
            val.append(I.flat[p] / gain if record_peak else gC)
        return I, np.asarray(pix, np.int64), np.asarray(val, np.float64)
    return bad


@pytest.mark.parametrize("kw,pin", [
    ({"mirror": True}, TC.test_hogbom_model_plus_residual_gives_back_the_image),
    ({"record_peak": True}, TC.test_hogbom_single_source_is_geometric),
    ({"last_tie": True}, lambda: TC.test_hogbom_delta_beam_gain_one_sorts_pixels(False)),
    ({"add": True}, TC.test_hogbom_single_source_is_geometric),
])
def test_hogbom_mutations_caught(monkeypatch, kw, pin):
    monkeypatch.setattr(oc, "hogbom", _hogbom_variant(**kw))
    with pytest.raises(AssertionError):
        pin()


def test_dirty_image_without_normalisation_caught(monkeypatch):
    monkeypatch.setattr(oc, "dirty_image",
                        lambda u, v, w, y, l, m, nm1, sign=-1:
                        ov.adjoint(u, v, w, y, l, m, nm1, sign).real)
    with pytest.raises(AssertionError):
        TC.test_dirty_image_of_unit_source_peaks_on_its_pixel(TC.SMALL.uvw())


def test_dirty_beam_without_w_term_caught(monkeypatch):
    orig = oc.dirty_image

    def beam_no_w(u, v, w, nx, ny, cell, sign=-1):
        bl, bm, bn, inside = oc.image_grid(2 * nx - 1, 2 * ny - 1, cell, nx - 1, ny - 1)
        b = np.zeros(bl.shape[0])
        b[inside] = orig(u, v, np.zeros_like(w), np.ones(u.size, complex), bl[inside],
                         bm[inside], bn[inside], sign)
        return b.reshape(2 * ny - 1, 2 * nx - 1)
    monkeypatch.setattr(oc, "dirty_beam", beam_no_w)
    with pytest.raises(AssertionError):
        TC.test_dirty_beam_is_the_image_of_a_centre_source(TC.SMALL.uvw())


def test_clean_beam_swapped_axes_caught(monkeypatch):
    orig = oc.fit_clean_beam
    monkeypatch.setattr(oc, "fit_clean_beam", lambda beam: orig(beam)[::-1])
    with pytest.raises(AssertionError):
        TC.test_fit_clean_beam_recovers_a_sampled_gaussian()


def test_restore_wrong_sign_caught(monkeypatch):
    orig = oc.restore
    monkeypatch.setattr(oc, "restore", lambda nx, ny, p, v, abc, residual=None:
                        orig(nx, ny, p, v, (abc[0], -abc[1], abc[2]), residual))
    with pytest.raises(AssertionError):
        TC.test_restore_linear_peaked_symmetric()


def test_cross_reference_wrong_frame_caught(monkeypatch):
    orig = oc.cross_reference
    monkeypatch.setattr(oc, "cross_reference",
                        lambda J, ra, dec, l, m: orig(J, ra, -dec, l, m))
    with pytest.raises(AssertionError):
        TC.test_cross_reference_and_tree_from_pixels()


def test_degrid_missing_w_correction_caught(monkeypatch):
    orig = od.es_hat
    # the w direction's correction is the only call with per-pixel (2-D) arguments
    monkeypatch.setattr(od, "es_hat", lambda f, W, n_quad=od.N_QUAD:
                        np.ones_like(np.asarray(f, float)) * orig(np.zeros(1), W, n_quad)[0]
                        if np.ndim(f) == 2 else orig(f, W, n_quad))
    with pytest.raises(AssertionError):
        TG.test_wide_field_w_term(TG.TRACK.uvw())


def test_degrid_wrong_fft_direction_caught(monkeypatch):
    orig_fft2, orig_ifft2 = np.fft.fft2, np.fft.ifft2
    monkeypatch.setattr(od.np.fft, "fft2", lambda a: orig_ifft2(a) * a.size)
    with pytest.raises(AssertionError):
        TG.test_error_falls_with_support(TG.TRACK.uvw())
    monkeypatch.setattr(od.np.fft, "fft2", orig_fft2)


def test_degrid_missing_centring_phase_caught(monkeypatch):
    orig = od.predict_degrid

    def bad(image, cell, u, v, w, W=10, sign=-1):
        P = od.plan(image.shape[1], image.shape[0], cell, w, W)
        return orig(image, cell, u, v, w, W, sign) * np.exp(-sign * 2j * np.pi * np.asarray(w) * P["c"])
    monkeypatch.setattr(od, "predict_degrid", bad)
    with pytest.raises(AssertionError):
        TG.test_wide_field_w_term(TG.TRACK.uvw())


# ------------------------------------------------------------- thresholding --
from oracle import threshold as oth  # noqa: E402

from . import test_oracle_threshold as TT2  # noqa: E402


def test_threshold_collapsed_node_at_wrong_centre_caught(monkeypatch):
    # a collapsed node sampled at its parent's pixel centre instead of its own
    # (planted in the thresholding oracle only, through a copy of the module)
    import types
    orig = sp.pixel_centres_lmn

    def parent_centre(j, pix, ra, dec):
        if j >= 2:
            return orig(j - 1, np.asarray(pix) >> 2, ra, dec)
        return orig(j, pix, ra, dec)
    shim = types.SimpleNamespace(**{k: getattr(sp, k) for k in dir(sp) if not k.startswith("__")})
    shim.pixel_centres_lmn = parent_centre
    monkeypatch.setattr(oth, "sphere", shim)
    with pytest.raises(AssertionError):
        TT2.test_levels_kept_whole_give_the_direct_sum_one_level_down(4)


def test_threshold_dropped_coefficients_kept_caught(monkeypatch):
    # collapse only: the dropped coefficients of remaining nodes left in V
    monkeypatch.setattr(oth, "keep_masks",
                        lambda tree, flat: [np.ones_like(k) | k for k in
                                            _orig_keep_masks(tree, flat)])
    with pytest.raises(AssertionError):
        TT2.test_two_leaf_tree_by_hand()


_orig_keep_masks = oth.keep_masks


def test_threshold_signed_ranking_caught(monkeypatch):
    # ranking by gamma instead of |gamma|
    def signed(tree):
        vals = np.concatenate([lv.gamma.ravel() for lv in tree.levels[:-1]])
        return np.argsort(-vals, kind="stable")
    monkeypatch.setattr(oth, "coefficient_ranking", signed)
    with pytest.raises(AssertionError):
        TT2.test_ranking_order_and_count()
