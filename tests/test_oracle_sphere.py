"""Pins of the oracle's frames (Eq. 18) and nested equal-area pixelisation
(section 3.2), including the values the paper prints (tests/golden)."""
import math

import numpy as np
import pytest

from oracle import sphere as sp


def _random_xyz(n, seed):
    rng = np.random.default_rng(seed)
    z = rng.uniform(-1, 1, n)
    phi = rng.uniform(0, 2 * np.pi, n)
    s = np.sqrt(1 - z * z)
    # xyz frame: y is the pole
    return np.stack([s * np.sin(phi), z, s * np.cos(phi)]).astype(sp.LD)


def test_pixel_count_formula():
    for j in range(1, 8):
        assert sp.n_pixels(j) == 12 * 4 ** (j - 1)
        pix = sp.ang2pix_xyz(j, _random_xyz(20000, j))
        assert pix.min() >= 0 and pix.max() < sp.n_pixels(j)


def test_base_pixel_centres_closed_form():
    c = sp.pix2xyz(1, np.arange(12))
    z = np.asarray(c[1], float)
    phi = np.mod(np.arctan2(np.asarray(c[0], float), np.asarray(c[2], float)), 2 * np.pi)
    for f in range(4):
        assert z[f] == pytest.approx(2 / 3, abs=1e-15)
        assert phi[f] == pytest.approx(np.pi / 4 + f * np.pi / 2, abs=1e-15)
        assert z[4 + f] == pytest.approx(0.0, abs=1e-15)
        assert phi[4 + f] == pytest.approx(f * np.pi / 2, abs=1e-15)
        assert z[8 + f] == pytest.approx(-2 / 3, abs=1e-15)
        assert phi[8 + f] == pytest.approx(np.pi / 4 + f * np.pi / 2, abs=1e-15)


@pytest.mark.parametrize("j", [1, 2, 3, 4, 5, 6])
def test_round_trip_every_pixel(j):
    pix = np.arange(sp.n_pixels(j), dtype=np.int64)
    assert np.array_equal(sp.ang2pix_xyz(j, sp.pix2xyz(j, pix)), pix)


@pytest.mark.parametrize("j", [9, 12, 20, 29])
def test_round_trip_sample(j):
    rng = np.random.default_rng(j)
    pix = np.unique(rng.integers(0, sp.n_pixels(j), 20000, dtype=np.int64))
    assert np.array_equal(sp.ang2pix_xyz(j, sp.pix2xyz(j, pix)), pix)


@pytest.mark.parametrize("j", [1, 2, 3, 5])
def test_children_centres_inside_parent(j):
    # the four children 4k + c of pixel k lie inside k (section 3.5's k >> 2)
    ch = np.arange(sp.n_pixels(j + 1), dtype=np.int64)
    assert np.array_equal(sp.ang2pix_xyz(j, sp.pix2xyz(j + 1, ch)), ch >> 2)


def test_nested_parent_rule_random_points():
    xyz = _random_xyz(50000, 11)
    J = 29
    kJ = sp.ang2pix_xyz(J, xyz)
    for j in (1, 2, 7, 15, 28):
        assert np.array_equal(kJ >> (2 * (J - j)), sp.ang2pix_xyz(j, xyz))


def test_equal_area_monte_carlo():
    j = 3
    n = 1_536_000
    counts = np.bincount(sp.ang2pix_xyz(j, _random_xyz(n, 12)), minlength=sp.n_pixels(j))
    exp = n / sp.n_pixels(j)
    chi2 = np.sum((counts - exp) ** 2 / exp)
    dof = sp.n_pixels(j) - 1
    # 6-sigma band of a chi^2 with `dof` degrees of freedom
    assert abs(chi2 - dof) < 6 * math.sqrt(2 * dof), chi2


def _ring_centres(nside):
    """Pixel centres (z, phi) of the HEALPix ring scheme (Gorski et al. 2005),
    ring by ring from the north pole: polar ring i < nside holds 4 i centres
    at z = 1 - i^2 / (3 nside^2), phi = (pi / (2 i)) (k - 1/2); the rings
    nside <= i <= 3 nside hold 4 nside centres at z = 4/3 - 2 i / (3 nside),
    phi = (pi / (2 nside)) (k - s/2) with s = (i - nside + 1) mod 2; the
    southern polar rings mirror the northern ones."""
    out = []
    for i in range(1, nside):
        k = np.arange(1, 4 * i + 1)
        z = 1 - i * i / (3 * nside * nside)
        for zz in (z, -z):
            out += [(zz, p) for p in np.pi / (2 * i) * (k - 0.5)]
    for i in range(nside, 3 * nside + 1):
        k = np.arange(1, 4 * nside + 1)
        s_ = (i - nside + 1) % 2
        z = 4 / 3 - 2 * i / (3 * nside)
        out += [(z, p) for p in np.pi / (2 * nside) * (k - s_ / 2)]
    return np.array(out)


@pytest.mark.parametrize("j", [1, 2, 3, 4, 5])
def test_centres_are_the_ring_scheme_centres(j):
    # the set of nested centres equals the ring scheme's closed-form centres
    nside = 1 << (j - 1)
    c = sp.pix2xyz(j, np.arange(sp.n_pixels(j)))
    z = np.asarray(c[1], float)
    phi = np.mod(np.arctan2(np.asarray(c[0], float), np.asarray(c[2], float)), 2 * np.pi)
    ref = _ring_centres(nside)
    assert ref.shape[0] == sp.n_pixels(j)
    got = np.stack([z, phi], 1)
    # phi within 1e-12 of 2 pi is the same direction as phi = 0
    got[:, 1] = np.where(got[:, 1] > 2 * np.pi - 1e-12, 0.0, got[:, 1])
    ref[:, 1] = np.mod(ref[:, 1], 2 * np.pi)
    key = lambda a: np.lexsort((np.round(a[:, 1], 9), np.round(a[:, 0], 9)))  # noqa: E731
    g, r = got[key(got)], ref[key(ref)]
    assert np.max(np.abs(g - r)) < 1e-13


@pytest.mark.parametrize("j", [2, 3])
def test_iso_latitude_rings(j):
    # HEALPix centres lie on 4 nside - 1 rings; polar ring i (1..nside-1
    # from each pole) holds 4 i pixels, every other ring 4 nside.
    nside = 1 << (j - 1)
    z = np.asarray(sp.pix2xyz(j, np.arange(sp.n_pixels(j)))[1], float)
    rings, counts = np.unique(np.round(z, 12), return_counts=True)
    assert len(rings) == 4 * nside - 1
    expect = sorted([4 * i for i in range(1, nside)] * 2 + [4 * nside] * (2 * nside + 1))
    assert sorted(counts.tolist()) == expect


def test_point_to_centre_distance():
    j = 7
    xyz = _random_xyz(100000, 13)
    c = sp.pix2xyz(j, sp.ang2pix_xyz(j, xyz))
    dot = np.clip(np.sum(np.asarray(xyz, float) * np.asarray(c, float), axis=0), -1, 1)
    assert np.max(np.arccos(dot)) < 1.2 * sp.angular_size(j)


def test_frame_axes():
    # Eq. 18: the phase centre maps to (alpha_P, delta_P); u points east
    # (increasing RA), v north (increasing declination).
    ra_p, dec_p = 1.234, 0.567
    R = np.asarray(sp.rotation_uvw_to_xyz(ra_p, dec_p), float)
    assert np.allclose(R @ R.T, np.eye(3), atol=1e-15)
    assert np.linalg.det(R) == pytest.approx(1.0, abs=1e-15)
    ra, dec = sp.xyz_to_radec(sp.lm_to_xyz([0.0], [0.0], ra_p, dec_p))
    assert float(ra[0]) == pytest.approx(ra_p, abs=1e-15)
    assert float(dec[0]) == pytest.approx(dec_p, abs=1e-15)
    eps = 1e-6
    ra_e, dec_e = sp.xyz_to_radec(sp.lm_to_xyz([eps], [0.0], ra_p, dec_p))
    ra_n, dec_n = sp.xyz_to_radec(sp.lm_to_xyz([0.0], [eps], ra_p, dec_p))
    assert float(ra_e[0] - ra_p) * math.cos(dec_p) == pytest.approx(eps, rel=1e-5)
    assert float(dec_e[0]) == pytest.approx(dec_p, abs=1e-11)
    assert float(dec_n[0] - dec_p) == pytest.approx(eps, rel=1e-5)
    assert float(ra_n[0]) == pytest.approx(ra_p, abs=1e-11)


def test_pixel_centre_lmn_of_phase_centre_pixel():
    # a component at the phase centre snaps to a pixel whose centre is within
    # one pixel size; n - 1 agrees with the SIN relation
    J = 10
    ra_p, dec_p = 3.0, 0.5
    k = sp.ang2pix_xyz(J, sp.lm_to_xyz([0.0], [0.0], ra_p, dec_p))
    l, m, nm1 = sp.pixel_centres_lmn(J, k, ra_p, dec_p)
    assert math.hypot(l[0], m[0]) < sp.angular_size(J)
    r2 = l[0] ** 2 + m[0] ** 2
    assert nm1[0] == pytest.approx(-r2 / (1 + math.sqrt(1 - r2)), rel=1e-14)


def test_recommended_resolution_table(golden):
    mas = math.pi / 180 / 3600 / 1000
    for name, res_mas, J, wav_mas in golden["recommended_resolutions"]["rows"]:
        assert sp.recommended_level(res_mas * mas) == J, name
        got = sp.angular_size(J) / mas
        digits = len(str(wav_mas).replace(".", "").lstrip("0"))
        # printed value is got rounded to its printed significant digits
        # (the table prints 400 for 402.6 and 50 for 50.3: two digits)
        sig = max(1, min(digits, 2))
        assert float(f"{got:.{sig}g}") == pytest.approx(wav_mas, rel=1e-9), (name, got)


def test_printed_pixel_counts(golden):
    for J, count in golden["pixel_counts"]["rows"]:
        assert float(f"{sp.n_pixels(J):.2g}") == count


def test_ngc628_level(golden):
    g = golden["ngc628_resolution"]
    arcsec = sp.angular_size(g["J"]) * 180 / math.pi * 3600
    assert round(arcsec, 1) == g["arcsec"]


def test_runtime_scaling_arithmetic(golden):
    g = golden["runtime_scaling"]
    d = g["J_to"] - g["J_from"]
    assert round(g["base"] ** d, 1) == g["time_ratio"]
    assert abs(2 ** d - g["resolution_ratio"]) / g["resolution_ratio"] < 0.01
    n_bl = g["jvla_antennas"] * (g["jvla_antennas"] - 1) // 2
    assert float(f"{n_bl * g['jvla_seconds']:.3g}") == g["jvla_visibilities"]


def test_disk_pixels_are_exactly_those_within_radius():
    J, ra_p, dec_p, rad = 6, 2.0, 0.3, math.radians(8.0)
    pix, l, m, nm1 = sp.pixels_in_disk(J, ra_p, dec_p, rad)
    allpix = np.arange(sp.n_pixels(J))
    _, _, nm1_all = sp.pixel_centres_lmn(J, allpix, ra_p, dec_p)
    inside = allpix[(1 + nm1_all) >= math.cos(rad) - 1e-15]
    assert np.array_equal(pix, inside)
    # the disk holds ~ (disk area) / A_J pixels
    expect = 2 * math.pi * (1 - math.cos(rad)) / sp.pixel_area(J)
    assert abs(len(pix) - expect) < 0.25 * expect


def _child_layout_violations(j, parents):
    """Parents at level j whose children 4k + c break the nested layout:
    child 0 at the southern corner (lowest z), 1 the eastern and 2 the
    western (equal z, 1 east of 2), 3 the northern (highest z)."""
    ch = (np.asarray(parents, np.int64)[:, None] * 4 + np.arange(4)).ravel()
    c = sp.pix2xyz(j + 1, ch)
    z = np.asarray(c[1], float).reshape(-1, 4)
    phi = np.arctan2(np.asarray(c[0], float), np.asarray(c[2], float)).reshape(-1, 4)
    east = np.angle(np.exp(1j * (phi[:, 1] - phi[:, 2])))      # phi_1 - phi_2 in (-pi, pi]
    ok = (z[:, 0] < z[:, 1]) & (z[:, 1] == z[:, 2]) & (z[:, 2] < z[:, 3]) & (east > 0)
    return np.asarray(parents)[~ok]


def test_nested_child_layout():
    # HEALPix NESTED (Gorski et al. 2005): inside a base pixel the x index
    # grows towards the north-east edge and y towards the north-west edge, so
    # child 0 is the southern corner, 1 the eastern, 2 the western, 3 the
    # northern one -- in every base pixel: north row (0-3), equatorial row
    # (4-7) and south row (8-11).
    assert _child_layout_violations(1, np.arange(12)).size == 0
    for face in (0, 4, 8):          # one base pixel per row, spelt out
        c = sp.pix2xyz(2, 4 * face + np.arange(4))
        z = np.asarray(c[1], float)
        phi = np.arctan2(np.asarray(c[0], float), np.asarray(c[2], float))
        assert z[0] < z[1] and z[0] < z[2] and z[3] > z[1] and z[3] > z[2], face
        assert np.angle(np.exp(1j * (phi[1] - phi[0]))) > 0, face
        assert np.angle(np.exp(1j * (phi[0] - phi[2]))) > 0, face
        assert z[1] == pytest.approx(z[2], abs=1e-15)


def test_level2_children_closed_form():
    # The children of base pixels 0, 4 and 8 at level 2 (nside = 2), from the
    # ring scheme: north face 0 (centre z = 2/3, phi = pi/4) has its children
    # at z = 1/3 (south), 2/3 (east, west), 11/12 (north); equatorial face 4
    # (z = 0, phi = 0) at -1/3, 0, 0, 1/3; south face 8 at -11/12, -2/3, -2/3,
    # -1/3.  East and west sit pi/8 either side of the face centre's phi.
    q = np.pi / 8
    expect = {
        0: [(1 / 3, 2 * q), (2 / 3, 3 * q), (2 / 3, q), (11 / 12, 2 * q)],
        4: [(-1 / 3, 0.0), (0.0, q), (0.0, -q), (1 / 3, 0.0)],
        8: [(-11 / 12, 2 * q), (-2 / 3, 3 * q), (-2 / 3, q), (-1 / 3, 2 * q)],
    }
    for face, rows in expect.items():
        c = sp.pix2xyz(2, 4 * face + np.arange(4))
        z = np.asarray(c[1], float)
        phi = np.arctan2(np.asarray(c[0], float), np.asarray(c[2], float))
        for cc, (ze, pe) in enumerate(rows):
            assert z[cc] == pytest.approx(ze, abs=1e-15), (face, cc)
            assert phi[cc] == pytest.approx(pe, abs=1e-15), (face, cc)


@pytest.mark.parametrize("j", [1, 2, 3, 4, 5])
def test_child_layout_every_pixel(j):
    assert _child_layout_violations(j, np.arange(sp.n_pixels(j))).size == 0


@pytest.mark.parametrize("j", [9, 17, 28])
def test_child_layout_deep_levels(j):
    rng = np.random.default_rng(j)
    parents = rng.integers(0, sp.n_pixels(j), 3000, dtype=np.int64)
    assert _child_layout_violations(j, parents).size == 0
