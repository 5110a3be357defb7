"""Pins of the oracle's wavelet tree (Eqs. 9, 10, 16, 17; section 3.5)."""
import numpy as np
import pytest

from oracle import sphere as sp
from oracle import tree as ot
from oracle import visibility as ov

RA, DEC = 3.1, 0.62


def _model(n, seed, half=0.05):
    rng = np.random.default_rng(seed)
    return (rng.uniform(-half, half, n), rng.uniform(-half, half, n), rng.lognormal(-3, 1, n))


def _uvw(n, seed, scale=3e3):
    rng = np.random.default_rng(seed)
    return tuple(rng.uniform(-scale, scale, n) for _ in range(3))


def test_sign_table_matches_eq10(golden):
    g = golden["wavelet_signs"]
    assert ot.WAVELET_SIGNS.tolist() == [g["gamma0"], g["gamma1"], g["gamma2"]]
    H = np.vstack([np.ones(4), ot.WAVELET_SIGNS])
    assert np.array_equal(H @ H.T, 4 * np.eye(4))


@pytest.mark.parametrize("J", [1, 2, 3, 4])
def test_analysis_then_synthesis_recovers_level_J(J):
    l, m, f = _model(40, J, half=0.6)
    t = ot.build_tree(J, RA, DEC, l, m, f)
    rec = ot.synthesise(t)
    lamJ = dict(zip(t.leaf_pix.tolist(), (t.leaf_flux / sp.pixel_area(J)).tolist()))
    scale = max(abs(x) for x in lamJ.values())
    for k, val in rec.items():
        assert abs(val - lamJ.get(k, 0.0)) <= 1e-12 * scale, k


def test_ancestor_ids_follow_shift_rule():
    J = 8
    l, m, f = _model(300, 3)
    t = ot.build_tree(J, RA, DEC, l, m, f)
    for j in range(1, J):
        assert np.array_equal(t.levels[j - 1].pix, np.unique(t.leaf_pix >> (2 * (J - j))))
    # every component lies in its leaf
    kJ, _, _ = ot.snap_components(J, RA, DEC, l, m, f)
    assert np.isin(kJ, t.leaf_pix).all()
    assert t.leaf_flux.sum() == pytest.approx(f.sum(), rel=1e-14)


def test_uniform_model_has_zero_wavelets():
    # one unit of flux in every pixel of a small J: a constant function
    J = 3
    allpix = np.arange(sp.n_pixels(J))
    levels = ot.build_levels(J, allpix, np.ones(allpix.shape[0]))
    for lv in levels[:-1]:
        assert np.max(np.abs(lv.gamma)) < 1e-15
        assert np.allclose(lv.lam, 1 / sp.pixel_area(J), rtol=1e-14)


def test_single_component_is_flux_times_leaf_plane_wave():
    J = 9
    t = ot.build_tree(J, RA, DEC, [0.011], [-0.007], [2.5])
    u, v, w = _uvw(200, 4, 2e4)
    V = ot.predict_tree(t, u, v, w)
    eta = ov.phasors(u, v, w, t.leaf_l, t.leaf_m, t.leaf_nm1)[:, 0]
    assert np.max(np.abs(V - 2.5 * eta)) < 1e-14 * 2.5


def test_level_one_tree_is_the_snapped_sum():
    l, m, f = _model(30, 5, half=0.7)
    t = ot.build_tree(1, RA, DEC, l, m, f)
    assert len(t.levels) == 1 and t.levels[0].gamma is None
    u, v, w = _uvw(100, 6, 50.0)
    V = ot.predict_tree(t, u, v, w)
    assert np.max(np.abs(V - ot.predict_snapped(t, u, v, w))) < 1e-14 * f.sum()


@pytest.mark.parametrize("J", [2, 5, 8, 12, 20])
@pytest.mark.parametrize("sign", [-1, 1])
def test_eq17_equals_snapped_direct(J, sign):
    l, m, f = _model(150, 10 + J)
    t = ot.build_tree(J, RA, DEC, l, m, f)
    u, v, w = _uvw(300, 20 + J, 1e4)
    V = ot.predict_tree(t, u, v, w, sign)
    Vd = ot.predict_snapped(t, u, v, w, sign)
    assert np.max(np.abs(V - Vd)) < (J + 1) * 1e-15 * f.sum()


@pytest.mark.parametrize("J", [2, 3, 4])
def test_unmasked_tree_gives_same_visibilities(J):
    # zero branches may be skipped: the full-sphere tree (every pixel a leaf,
    # plane-wave coefficients of empty pixels included) gives the same V
    l, m, f = _model(25, 30 + J, half=0.5)
    t = ot.build_tree(J, RA, DEC, l, m, f)
    full = ot.build_full_tree(J, RA, DEC, l, m, f)
    assert full.n_leaves == sp.n_pixels(J)
    u, v, w = _uvw(64, 40 + J, 30.0)
    Vs = ot.predict_tree(t, u, v, w)
    Vf = ot.predict_tree(full, u, v, w)
    assert np.max(np.abs(Vs - Vf)) < 1e-13 * f.sum()
    # with zero model but non-zero plane waves the full tree still gives 0
    empty = ot.Tree(J, RA, DEC, full.leaf_pix, 0 * full.leaf_flux, full.leaf_l,
                    full.leaf_m, full.leaf_nm1,
                    ot.build_levels(J, full.leaf_pix, 0 * full.leaf_flux))
    assert np.max(np.abs(ot.predict_tree(empty, u, v, w))) == 0.0


def test_snapping_moves_positions_by_at_most_a_pixel():
    J = 10
    l, m, f = _model(200, 50, half=0.03)
    t = ot.build_tree(J, RA, DEC, l, m, f)
    kJ, leaf, _ = ot.snap_components(J, RA, DEC, l, m, f)
    idx = np.searchsorted(t.leaf_pix, kJ)
    d = np.hypot(l - t.leaf_l[idx], m - t.leaf_m[idx])
    assert d.max() < sp.angular_size(J)
