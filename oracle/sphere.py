"""Oracle: coordinate frames and the hierarchical equal-area sphere pixelisation.

Frames (section 3.4, Eq. 18).  uvw: w towards the phase centre P, u east,
v north.  xyz: y towards the north celestial pole, x towards RA 6h, z
towards RA 0h, so a direction (alpha, delta) is
[cos d sin a, sin d, cos d cos a].  The rotation is
R_uvw->xyz = R_y(alpha_P) R_x(-delta_P) with the standard right-handed
active matrices.

Pixelisation (section 3.2).  Twelve equal-area base pixels at level j = 1,
each split into four equal-area children per level, N_j = 12 * 4^(j-1),
nested indices so that the parent of k is k >> 2 (section 3.5).  The paper
bases this on HEALPix (Gorski et al. 2005) with its own software; this is
the HEALPix NESTED scheme at nside = 2^(j-1), written here from the
geometry of the HEALPix projection:

* equatorial zone |z| <= 2/3 (z = cos theta): X = phi/(pi/2), Y = 3z/4;
* polar caps: sigma = sqrt(3 (1 - |z|)), X = Xc + (X0 - Xc) sigma with
  Xc the centre of the quarter-turn containing phi, Y = +-(1 - sigma/2).

In the (X, Y) plane every base pixel is a square rotated by 45 degrees;
A = X + Y + 1/2 and B = Y + 1/2 - X are coordinates along its two edges,
floor(A) and floor(B) identify the base pixel (north: floor A + floor B = 1,
equatorial 0, south -1) and their fractional parts times nside are the
in-face indices (ix, iy).  The nested index interleaves the bits of ix (even
positions) and iy (odd positions) under the face number.  Base pixels 0-3
are centred at z = 2/3, phi = pi/4 + f pi/2; 4-7 at z = 0, phi = f pi/2;
8-11 at z = -2/3, phi = pi/4 + f pi/2.

All geometry is evaluated in numpy.longdouble (x86 extended precision) and
rounded to FP64 once, so a pixel centre is the FP64 rounding of the exact
centre up to ~1e-19.
"""
from __future__ import annotations

import numpy as np

LD = np.longdouble
PI_LD = LD(4) * np.arctan(LD(1))


def n_pixels(j: int) -> int:
    """N_j = 12 * 4^(j-1) (section 3.2)."""
    return 12 * 4 ** (j - 1)


def pixel_area(j: int) -> float:
    """A_j = 4 pi / N_j steradians."""
    return 4.0 * np.pi / n_pixels(j)


def angular_size(j: int) -> float:
    """Delta theta_j ~ sqrt(A_j) = 2^(1-j) sqrt(pi/3) radians (section 3.3)."""
    return 2.0 ** (1 - j) * np.sqrt(np.pi / 3.0)


def recommended_level(resolution_rad: float, oversample: float = 2.0) -> int:
    """Smallest J whose pixel size oversamples an image cell of the given size
    by at least `oversample` (the rule of the recommended-resolution table)."""
    j = 1
    while resolution_rad / angular_size(j) < oversample:
        j += 1
    return j


# ------------------------------------------------------------------ frames --
def rot_x(t):
    c, s = np.cos(LD(t)), np.sin(LD(t))
    return np.array([[1, 0, 0], [0, c, -s], [0, s, c]], dtype=LD)


def rot_y(t):
    c, s = np.cos(LD(t)), np.sin(LD(t))
    return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]], dtype=LD)


def rotation_uvw_to_xyz(ra_p: float, dec_p: float):
    """R_uvw->xyz = R_y(alpha_P) R_x(-delta_P) (Eq. 18), longdouble 3x3."""
    return rot_y(ra_p) @ rot_x(-dec_p)


def lm_to_xyz(l, m, ra_p, dec_p):
    """SIN projection [l, m, sqrt(1 - l^2 - m^2)] (section 3.3) rotated to xyz.
    Returns a (3, K) longdouble array."""
    l = np.asarray(l, dtype=LD)
    m = np.asarray(m, dtype=LD)
    n = np.sqrt(LD(1) - l * l - m * m)
    return rotation_uvw_to_xyz(ra_p, dec_p) @ np.stack([l, m, n])


def xyz_to_radec(xyz):
    """(alpha in [0, 2 pi), delta) of xyz unit vectors."""
    x, y, z = xyz
    ra = np.arctan2(x, z)
    ra = np.where(ra < 0, ra + 2 * PI_LD, ra)
    dec = np.arctan2(y, np.sqrt(x * x + z * z))
    return ra, dec


def radec_to_xyz(ra, dec):
    ra = np.asarray(ra, dtype=LD)
    dec = np.asarray(dec, dtype=LD)
    return np.stack([np.cos(dec) * np.sin(ra), np.sin(dec), np.cos(dec) * np.cos(ra)])


# -------------------------------------------------------- nested pixels ----
def _interleave(ix, iy, bits):
    out = np.zeros_like(ix)
    for b in range(bits):
        out |= ((ix >> b) & 1) << (2 * b)
        out |= ((iy >> b) & 1) << (2 * b + 1)
    return out


def _deinterleave(p, bits):
    ix = np.zeros_like(p)
    iy = np.zeros_like(p)
    for b in range(bits):
        ix |= ((p >> (2 * b)) & 1) << b
        iy |= ((p >> (2 * b + 1)) & 1) << b
    return ix, iy


def ang2pix_xyz(j: int, xyz) -> np.ndarray:
    """Level-j nested pixel index of xyz unit vectors (3, K)."""
    nside = 1 << (j - 1)
    x, y, zx = (np.asarray(c, dtype=LD) for c in xyz)
    z = y                                   # cos(theta) = sin(dec)
    s2 = x * x + zx * zx                    # sin^2(theta)
    phi = np.arctan2(x, zx)
    phi = np.where(phi < 0, phi + 2 * PI_LD, phi)
    tt = phi / (PI_LD / 2)                  # quarter turns in [0, 4]
    tt = np.where(tt >= 4, tt - 4, tt)
    ns = LD(nside)

    # equatorial zone
    A = tt + LD(0.75) * z + LD(0.5)
    B = LD(0.75) * z + LD(0.5) - tt
    Na = np.floor(ns * A).astype(np.int64)
    Nb = np.floor(ns * B).astype(np.int64)
    p = np.floor_divide(Na, nside)
    q = np.floor_divide(Nb, nside)
    ix_e = Na - p * nside
    iy_e = Nb - q * nside
    sgn = p + q
    face_e = np.where(sgn == 0, 4 + np.mod(p, 4),
                      np.where(sgn > 0, np.mod(p - 1, 4), 8 + np.mod(p, 4)))

    # polar caps: 1 - |z| = sin^2(theta) / (1 + |z|)
    az = np.abs(z)
    sig = np.sqrt(LD(3) * s2 / (LD(1) + az))
    f = np.minimum(np.floor(tt).astype(np.int64), 3)
    tp = tt - f
    north = z > 0
    a_n = LD(1) - sig * (LD(1) - tp)
    b_n = LD(1) - sig * tp
    a_s = sig * tp
    b_s = sig * (LD(1) - tp)
    a = np.where(north, a_n, a_s)
    b = np.where(north, b_n, b_s)
    ix_p = np.clip(np.floor(ns * a).astype(np.int64), 0, nside - 1)
    iy_p = np.clip(np.floor(ns * b).astype(np.int64), 0, nside - 1)
    face_p = np.where(north, f, 8 + f)

    polar = az > LD(2) / LD(3)
    face = np.where(polar, face_p, face_e)
    ix = np.where(polar, ix_p, ix_e)
    iy = np.where(polar, iy_p, iy_e)
    return face * (nside * nside) + _interleave(ix, iy, j - 1)


def pix2xyz(j: int, pix) -> np.ndarray:
    """Centre of level-j nested pixels as longdouble xyz unit vectors (3, K)."""
    nside = 1 << (j - 1)
    pix = np.asarray(pix, dtype=np.int64)
    face = pix // (nside * nside)
    ix, iy = _deinterleave(pix % (nside * nside), j - 1)
    a = (ix.astype(LD) + LD(0.5)) / LD(nside)
    b = (iy.astype(LD) + LD(0.5)) / LD(nside)
    f = np.mod(face, 4).astype(LD)
    ring = face // 4                         # 0 north, 1 equatorial, 2 south

    # (X, Y) of the centre in the projection plane
    X = np.where(ring == 1, (a - b) / 2 + f, (a - b) / 2 + f + LD(0.5))
    Y = np.where(ring == 0, (a + b) / 2,
                 np.where(ring == 1, (a + b - 1) / 2, (a + b - 2) / 2))
    polar = np.abs(Y) > LD(0.5)
    sig = np.where(Y > 0, 2 - (a + b), a + b)          # only used where polar
    sig = np.where(polar, sig, LD(1))
    omz = sig * sig / 3                                  # 1 - |z| in the caps
    z = np.where(polar, np.sign(Y) * (1 - omz), LD(4) * Y / 3)
    # sin(theta) = sqrt((1 - z)(1 + z)), using 1 - |z| directly in the caps
    s_pol = np.sqrt(omz * (2 - omz))
    s_eq = np.sqrt((1 - z) * (1 + z))
    st = np.where(polar, s_pol, s_eq)
    tt = np.where(polar, f + LD(0.5) + (a - b) / (2 * sig), X)
    phi = tt * (PI_LD / 2)
    return np.stack([st * np.sin(phi), z, st * np.cos(phi)])


def xyz_to_uvw_lmn(xyz, ra_p, dec_p):
    """Rotate xyz unit vectors to uvw and return FP64 (l, m, n - 1), each the
    rounding of a longdouble value; n - 1 = -(l^2 + m^2)/(1 + n) for n > 0."""
    s = rotation_uvw_to_xyz(ra_p, dec_p).T @ np.asarray(xyz, dtype=LD)
    l, m, n = s
    nm1 = np.where(n > 0, -(l * l + m * m) / (1 + np.abs(n)), n - 1)
    return l.astype(np.float64), m.astype(np.float64), nm1.astype(np.float64)


def pixel_centres_lmn(j: int, pix, ra_p: float, dec_p: float):
    """(l, m, n - 1) in the uvw frame of the centres of level-j pixels."""
    return xyz_to_uvw_lmn(pix2xyz(j, pix), ra_p, dec_p)


def pixels_in_disk(j: int, ra_p: float, dec_p: float, radius_rad: float):
    """Sorted level-j pixels whose centres lie within `radius_rad` of the phase
    centre, with their (l, m, n - 1).  Brute force over every pixel."""
    out_pix = []
    cosr = np.cos(LD(radius_rad))
    pc = radec_to_xyz(ra_p, dec_p)
    npix = n_pixels(j)
    step = 1 << 18
    for s in range(0, npix, step):
        pix = np.arange(s, min(npix, s + step), dtype=np.int64)
        c = pix2xyz(j, pix)
        dot = pc[0] * c[0] + pc[1] * c[1] + pc[2] * c[2]
        out_pix.append(pix[dot >= cosr])
    pix = np.concatenate(out_pix)
    l, m, nm1 = pixel_centres_lmn(j, pix, ra_p, dec_p)
    return pix, l, m, nm1
