"""CPU pins of oracle/clean.py: the clean loop around the predictor.

Each check comes from what the paper's description fixes or from mathematics
that the oracle's code does not restate: the dirty image of a unit source
peaks at 1 on its pixel (Cauchy-Schwarz bounds it elsewhere); the dirty beam
is that image for a source at the phase centre; Hogbom with gain 1 and a
delta beam is a sort of the pixels; with a single beam-shaped source it is a
geometric series; the model convolved with the beam plus the residual gives
back the dirty image (Eq. 4 summed); the clean-beam fit recovers an exactly
sampled rotated Gaussian; Eq. 6 is linear and peaks at the component value;
the whole loop lowers chi^2 every major cycle and recovers the flux of
sources placed on pixel centres.
"""
import math

import numpy as np
import pytest

from oracle import clean as oc
from oracle import tree as ot
from oracle import visibility as ov
from synth import configs, models
from synth.configs import TrackSpec

SMALL = TrackSpec(27, 1.7e3, 45.0, 2016.0, 6, 1.0e7, seed=721)   # 2,106 rows
RA, DEC = math.radians(180.0), math.radians(45.0)


@pytest.fixture(scope="module")
def track():
    return SMALL.uvw()


def _shift(beam, ny, nx, p):
    """Beam window centred on pixel p, element by element."""
    py, px = divmod(int(p), nx)
    out = np.empty((ny, nx))
    for iy in range(ny):
        for ix in range(nx):
            out[iy, ix] = beam[iy - py + ny - 1, ix - px + nx - 1]
    return out


def _gauss_beam(ny, nx, a, b, c):
    dy, dx = np.meshgrid(np.arange(-(ny - 1), ny), np.arange(-(nx - 1), nx), indexing="ij")
    return np.exp(-(a * dx * dx + 2 * b * dx * dy + c * dy * dy))


# ------------------------------------------------------------------ grid --
def test_grid_directions():
    l, m, nm1, inside = oc.image_grid(9, 6, 0.01)
    assert inside.all()
    c = 3 * 9 + 4
    assert l[c] == 0.0 and m[c] == 0.0 and nm1[c] == 0.0
    assert l[c + 1] == 0.01 and m[c + 9] == 0.01
    np.testing.assert_allclose((nm1 + 1.0) ** 2 + l * l + m * m, 1.0, rtol=0, atol=4e-16)
    _, _, nm1b, inside_b = oc.image_grid(5, 5, 0.4)
    assert not inside_b.all() and np.all(nm1b[~inside_b] == 0.0)


# ---------------------------------------------------------- dirty images --
def test_dirty_image_of_unit_source_peaks_on_its_pixel(track):
    u, v, w = track
    nx, ny, cell = 15, 11, 2e-3
    l, m, nm1, _ = oc.image_grid(nx, ny, cell)
    q = 4 * nx + 11
    vis = ov.predict_direct(u, v, w, l[q:q + 1], m[q:q + 1], np.ones(1))
    img = oc.dirty_image(u, v, w, vis, l, m, nm1)
    assert abs(img[q] - 1.0) <= 1e-12
    assert np.all(np.abs(img) <= 1.0 + 1e-12) and int(np.argmax(img)) == q


def test_dirty_beam_is_the_image_of_a_centre_source(track):
    u, v, w = track
    nx, ny, cell = 12, 9, 3e-3
    beam = oc.dirty_beam(u, v, w, nx, ny, cell)
    assert beam.shape == (2 * ny - 1, 2 * nx - 1)
    assert abs(beam[ny - 1, nx - 1] - 1.0) <= 1e-15
    assert np.all(np.abs(beam) <= 1.0 + 1e-12)
    l, m, nm1, _ = oc.image_grid(nx, ny, cell)
    vis = ov.predict_direct(u, v, w, np.zeros(1), np.zeros(1), np.ones(1))
    img = oc.dirty_image(u, v, w, vis, l, m, nm1).reshape(ny, nx)
    np.testing.assert_allclose(img, _shift(beam, ny, nx, (ny // 2) * nx + nx // 2),
                               rtol=0, atol=1e-13)


def test_dirty_beam_off_disk_offsets_are_zero(track):
    u, v, w = track
    beam = oc.dirty_beam(u, v, w, 6, 6, 0.17)   # offsets reach 5 * 0.17 * sqrt(2) > 1
    _, _, _, inside = oc.image_grid(11, 11, 0.17, 5, 5)
    assert (~inside).any()
    assert np.all(beam.ravel()[~inside] == 0.0) and np.all(beam.ravel()[inside] != 0.0)


# ---------------------------------------------------------------- Hogbom --
@pytest.mark.parametrize("absolute", [False, True])
def test_hogbom_delta_beam_gain_one_sorts_pixels(absolute):
    rng = np.random.default_rng(3)
    ny, nx = 7, 9
    img = np.round(rng.normal(size=(ny, nx)), 1)   # rounding makes ties
    beam = np.zeros((2 * ny - 1, 2 * nx - 1))
    beam[ny - 1, nx - 1] = 1.0
    thr = 0.35
    res, pix, val = oc.hogbom(img, beam, 1.0, thr, 1000, absolute)
    key = np.abs(img.ravel()) if absolute else img.ravel()
    order = np.lexsort((np.arange(key.size), -key))   # by key descending, then pixel id
    want = order[key[order] > thr]
    assert np.array_equal(pix, want)
    assert np.array_equal(val, img.ravel()[want])
    expect = img.copy().ravel()
    expect[want] = 0.0
    assert np.array_equal(res.ravel(), expect)


def test_hogbom_single_source_is_geometric():
    ny, nx = 13, 10
    beam = _gauss_beam(ny, nx, 0.3, 0.1, 0.5)
    q = 6 * nx + 3
    S, g, n = 2.5, 0.2, 25
    res, pix, val = oc.hogbom(S * _shift(beam, ny, nx, q), beam, g, 0.0, n)
    assert np.all(pix == q)
    np.testing.assert_allclose(val, g * S * (1 - g) ** np.arange(n), rtol=1e-13)
    np.testing.assert_allclose(res, S * (1 - g) ** n * _shift(beam, ny, nx, q), rtol=0,
                               atol=1e-13)


def test_hogbom_model_plus_residual_gives_back_the_image():
    rng = np.random.default_rng(11)
    ny, nx = 16, 21
    beam = _gauss_beam(ny, nx, 0.15, -0.05, 0.35) * (1 + 0.3 * rng.uniform(size=(2 * ny - 1, 2 * nx - 1)))
    beam[ny - 1, nx - 1] = 1.0
    img = 0.01 * rng.normal(size=(ny, nx))
    for q, f in zip(rng.choice(nx * ny, 4, replace=False), [1.0, 0.7, 0.5, -0.4]):
        img += f * _shift(beam, ny, nx, q)
    res, pix, val = oc.hogbom(img, beam, 0.1, 0.0, 200)
    assert pix.size == 200
    rebuilt = res.copy()
    for p, g in zip(pix, val):
        rebuilt += g * _shift(beam, ny, nx, p)
    np.testing.assert_allclose(rebuilt, img, rtol=0, atol=1e-12)
    # every recorded value was g times the image's peak when it was taken
    assert np.all(val > 0)


def test_hogbom_stops_at_threshold_and_max_iter():
    rng = np.random.default_rng(5)
    ny, nx = 10, 10
    beam = _gauss_beam(ny, nx, 0.4, 0.0, 0.4)
    img = rng.normal(size=(ny, nx))
    res, pix, val = oc.hogbom(img, beam, 0.5, 1.2, 10_000)
    assert res.max() <= 1.2 and np.all(val / 0.5 > 1.2)
    res0, pix0, val0 = oc.hogbom(img, beam, 0.5, 0.0, 0)
    assert pix0.size == 0 and np.array_equal(res0, img)
    _, pix3, _ = oc.hogbom(img, beam, 0.5, -np.inf, 3)
    assert pix3.size == 3


# ------------------------------------------------- cross reference, tree --
def test_cross_reference_and_tree_from_pixels():
    nx, ny, cell, J = 24, 18, 4e-3, 12
    l, m, _, _ = oc.image_grid(nx, ny, cell)
    kJ = oc.cross_reference(J, RA, DEC, l, m)
    ref_kJ, _, _ = ot.snap_components(J, RA, DEC, l, m, np.ones(l.size))
    assert np.array_equal(kJ, ref_kJ)
    # ancestors by the shift rule k_j = k_J >> 2 (J - j)
    t_parent = oc.cross_reference(J - 3, RA, DEC, l, m)
    assert np.array_equal(kJ >> 6, t_parent)
    rng = np.random.default_rng(2)
    pick = rng.choice(l.size, 40)
    flux = rng.normal(size=40)
    a = oc.tree_from_pixels(J, RA, DEC, kJ[pick], flux)
    b = ot.build_tree(J, RA, DEC, l[pick], m[pick], flux)
    assert np.array_equal(a.leaf_pix, b.leaf_pix)
    np.testing.assert_allclose(a.leaf_flux, b.leaf_flux, rtol=1e-15, atol=1e-15)
    for la, lb in zip(a.levels, b.levels):
        assert np.array_equal(la.pix, lb.pix)
        np.testing.assert_allclose(la.lam, lb.lam, rtol=1e-14)


# ------------------------------------------------------------ clean beam --
def test_fit_clean_beam_recovers_a_sampled_gaussian():
    a, b, c = 0.11, 0.04, 0.07
    beam = _gauss_beam(20, 25, a, b, c)
    # a disconnected ring above 1/2 far out: not part of the main lobe
    beam[0, :] = 0.9
    got = oc.fit_clean_beam(beam)
    np.testing.assert_allclose(got, (a, b, c), rtol=1e-10)
    assert oc.main_lobe(beam).shape[0] < 200


def test_fit_clean_beam_rejects_an_unresolved_lobe():
    beam = np.zeros((9, 9))
    beam[4, 4] = 1.0
    beam[4, 5] = beam[4, 3] = beam[3, 4] = beam[5, 4] = 0.6
    with pytest.raises(ValueError):
        oc.fit_clean_beam(beam)


# ---------------------------------------------------------------- restore --
def test_restore_linear_peaked_symmetric():
    nx, ny = 17, 14
    abc = (0.2, 0.05, 0.3)
    p1 = np.array([3 * nx + 4, 8 * nx + 12])
    v1 = np.array([1.5, -0.5])
    p2 = np.array([7 * nx + 8])
    v2 = np.array([0.75])
    r1 = oc.restore(nx, ny, p1, v1, abc)
    r2 = oc.restore(nx, ny, p2, v2, abc)
    r12 = oc.restore(nx, ny, np.concatenate([p1, p2]), np.concatenate([v1, v2]), abc)
    np.testing.assert_allclose(r12, r1 + r2, rtol=0, atol=1e-15)
    assert r2[7, 8] == 0.75 and r2.max() == 0.75
    np.testing.assert_allclose(r2[7 + 3, 8 + 2], r2[7 - 3, 8 - 2], rtol=1e-15)
    # a component restored with the fit of a Gaussian beam is that beam
    beam = _gauss_beam(ny, nx, *abc)
    np.testing.assert_allclose(oc.restore(nx, ny, p2, [1.0], oc.fit_clean_beam(beam)),
                               _shift(beam, ny, nx, p2[0]), rtol=0, atol=1e-12)
    res = np.full((ny, nx), 0.25)
    np.testing.assert_allclose(oc.restore(nx, ny, p2, v2, abc, res), r2 + 0.25, atol=1e-15)


# ------------------------------------------------------------- the loop --
def test_wavelet_clean_recovers_pixel_centred_sources(track):
    u, v, w = track
    nx = ny = 24
    cell = 4e-3
    l, m, _, _ = oc.image_grid(nx, ny, cell)
    src = np.array([5 * nx + 6, 12 * nx + 17, 19 * nx + 9])
    flux = np.array([1.0, 0.6, 0.8])
    vis = ov.predict_direct(u, v, w, l[src], m[src], flux)
    # J = 22: sphere pixels (0.1") far below the image pixels (0.23 deg)
    out = oc.wavelet_clean(u, v, w, vis, nx, ny, cell, 22, RA, DEC, 0.2, 0.0, 60, 4)
    chi2 = [c["chi2"] for c in out["cycles"]]
    assert len(chi2) == 4 and all(b < a for a, b in zip(chi2, chi2[1:]))
    assert chi2[-1] < 1e-3 * float(np.sum(np.abs(vis) ** 2))
    # the flux sits on the source pixels
    model = np.bincount(out["pix"], weights=out["val"], minlength=nx * ny)
    np.testing.assert_allclose(model[src], flux, rtol=0, atol=0.02)
    assert np.abs(np.delete(model, src)).sum() < 0.05
    # the residual image is the dirty image of the final residual visibilities
    ll, mm, nn, _ = oc.image_grid(nx, ny, cell)
    again = oc.dirty_image(u, v, w, vis - out["vis_model"], ll, mm, nn).reshape(ny, nx)
    np.testing.assert_allclose(out["residual"], again, rtol=0, atol=1e-14)


def test_wavelet_clean_of_empty_sky_finds_nothing(track):
    u, v, w = track
    out = oc.wavelet_clean(u, v, w, np.zeros(u.size, np.complex128), 8, 8, 4e-3, 10, RA, DEC,
                           0.1, 0.0, 10, 2)
    assert out["pix"].size == 0 and out["cycles"] == []
    assert np.all(out["residual"] == 0.0)


def test_clean_workload_recipes():
    for S in (configs.CLEAN7, configs.CLEAN_SMALL):
        l, m, f = S.sources()
        assert l.size == S.n_sources and np.all(f == 1.0)
        assert np.all(np.abs(l) < S.n_pix * S.cell / 2) and np.all(np.abs(m) < S.n_pix * S.cell / 2)
    assert configs.CLEAN7.track.n_vis == 351 * 2016
    assert models.half_width(configs.CLEAN7.fov_deg) < 1.0


def test_clean_predictors_agree_where_they_should(track):
    """Direct, degridding (W = 12) and tree (J = 22) clean of pixel-centred
    sources find the same components: the three predictors agree to the
    degridder's kernel error and the tree's 0.1" snapping."""
    u, v, w = track
    nx = ny = 20
    cell = 4e-3
    l, m, _, _ = oc.image_grid(nx, ny, cell)
    src = np.array([4 * nx + 5, 11 * nx + 14, 15 * nx + 6])
    vis = ov.predict_direct(u, v, w, l[src], m[src], np.array([1.0, 0.5, 0.7]))
    runs = {p: oc.wavelet_clean(u, v, w, vis, nx, ny, cell, 22, RA, DEC, 0.2, 0.0, 40, 3,
                                predictor=p, support=12) for p in ("direct", "degrid", "tree")}
    d = runs["direct"]
    for p in ("degrid", "tree"):
        assert np.array_equal(runs[p]["pix"], d["pix"])
        np.testing.assert_allclose(runs[p]["val"], d["val"], rtol=0, atol=1e-6)
    np.testing.assert_allclose(runs["degrid"]["val"], d["val"], rtol=0, atol=1e-9)
    assert [c["leaves"] for c in d["cycles"]] == [c["leaves"] for c in runs["tree"]["cycles"]]
