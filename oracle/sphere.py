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
the HEALPix NESTED scheme at nside = 2^(j-1), written from the HEALPix
projection of the sphere onto a plane (Calabretta & Roukema 2007), in units
of a quarter turn:

* equatorial zone |z| <= 2/3 (z = cos theta): X = phi/(pi/2), Y = 3z/4;
* polar caps: sigma = sqrt(3 (1 - |z|)), X = Xc + (phi/(pi/2) - Xc) sigma
  with Xc the centre of the quarter turn containing phi, Y = +-(1 - sigma/2).

In that plane every base pixel is a square rotated by 45 degrees (a diamond)
and the four children of a pixel are the quarters of its diamond at its
south, east, west and north corners, numbered 0, 1, 2, 3.  A point's pixel
is found as the paper's section 3.5 builds its tree, from the top: the base
pixel whose diamond holds it, then level by level the quarter that holds it,
k <- 4k + c.  A pixel's centre is found the same way, moving from the base
centre towards corner c of every enclosing diamond.  Base pixels 0-3 are
centred at z = 2/3, phi = pi/4 + f pi/2; 4-7 at z = 0, phi = f pi/2; 8-11 at
z = -2/3, phi = pi/4 + f pi/2.

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
# Centres (X, Y) of the twelve base pixels in the projection plane, in
# quarter turns: 0-3 the north row, 4-7 the equatorial row, 8-11 the south row.
BASE_X = np.array([0.5, 1.5, 2.5, 3.5, 0.0, 1.0, 2.0, 3.0, 0.5, 1.5, 2.5, 3.5], dtype=LD)
BASE_Y = np.array([0.5] * 4 + [0.0] * 4 + [-0.5] * 4, dtype=LD)

# Child c of a pixel is the quarter of its diamond at its c-th corner:
# 0 south, 1 east, 2 west, 3 north.  Offsets of the child's centre from the
# parent's, in units of half the parent's half-diagonal.
CHILD_DX = np.array([0, 1, -1, 0], dtype=LD)
CHILD_DY = np.array([-1, 0, 0, 1], dtype=LD)


def _wrap(dX):
    """An X difference brought into [-2, 2) (X is periodic with period 4)."""
    return dX - 4 * np.floor((dX + 2) / 4)


def project(xyz):
    """HEALPix projection of unit vectors (3, K) to the plane (X, Y), in units
    of a quarter turn, and the quarter q of the polar triangle (-1 in the
    equatorial zone).  Returns (X, Y, q)."""
    x, z, zx = (np.asarray(c, dtype=LD) for c in xyz)     # z = cos(theta)
    t = np.arctan2(x, zx) / (PI_LD / 2)                     # phi in quarter turns
    t = np.where(t < 0, t + 4, t)
    t = np.where(t >= 4, t - 4, t)
    polar = np.abs(z) > LD(2) / LD(3)
    # sigma^2 = 3 (1 - |z|), with 1 - |z| = sin^2(theta) / (1 + |z|)
    sig = np.sqrt(LD(3) * (x * x + zx * zx) / (LD(1) + np.abs(z)))
    q = np.minimum(np.floor(t), 3)
    X = np.where(polar, q + LD(0.5) + (t - q - LD(0.5)) * sig, t)
    Y = np.where(polar, np.sign(z) * (LD(1) - sig / 2), LD(0.75) * z)
    return X, Y, np.where(polar, q, -1).astype(np.int64)


def _base_pixel(X, Y, q):
    """The base pixel holding each plane point.  A polar point lies in the
    triangle of its quarter.  In the equatorial strip the diamonds tile the
    plane: a diamond holds the points with edge coordinates a = dX + dY and
    b = dY - dX in [-1/2, 1/2), so a point on an edge goes to the pixel on
    its northern side."""
    face = np.full(X.shape, -1, dtype=np.int64)
    for f in range(12):
        dX = _wrap(X - BASE_X[f])
        dY = Y - BASE_Y[f]
        a, b = dX + dY, dY - dX
        inside = (a >= -0.5) & (a < 0.5) & (b >= -0.5) & (b < 0.5)
        face = np.where((face < 0) & inside, f, face)
    face = np.where(q >= 0, np.where(Y > 0, q, 8 + q), face)
    assert np.all(face >= 0), "a point outside every base pixel"
    return face


def ang2pix_xyz(j: int, xyz) -> np.ndarray:
    """Level-j nested pixel index of xyz unit vectors (3, K), by descent: the
    base pixel holding the point, then j - 1 times the child (k <- 4k + c)
    whose quarter of the current diamond holds it (sections 3.2, 3.5)."""
    X, Y, q = project(xyz)
    face = _base_pixel(X, Y, q)
    dX = _wrap(X - BASE_X[face])          # offset from the current centre
    dY = Y - BASE_Y[face]
    pix = face.copy()
    h = LD(0.5)                           # half-diagonal of the current diamond
    for _ in range(j - 1):
        ne = (dX + dY) >= 0               # north-east half of the diamond
        nw = (dY - dX) >= 0               # north-west half
        c = ne.astype(np.int64) + 2 * nw.astype(np.int64)
        pix = 4 * pix + c
        dX = dX - CHILD_DX[c] * (h / 2)
        dY = dY - CHILD_DY[c] * (h / 2)
        h = h / 2
    return pix


def pixel_plane_centre(j: int, pix):
    """(X, Y) of the centre of level-j nested pixels: the base centre moved
    towards corner c of each enclosing diamond, level by level."""
    pix = np.asarray(pix, dtype=np.int64)
    face = pix >> (2 * (j - 1))
    X = BASE_X[face].copy()
    Y = BASE_Y[face].copy()
    h = LD(0.5)
    for lev in range(1, j):
        c = (pix >> (2 * (j - 1 - lev))) & 3
        X = X + CHILD_DX[c] * (h / 2)
        Y = Y + CHILD_DY[c] * (h / 2)
        h = h / 2
    return X, Y


def unproject(X, Y):
    """Inverse of `project` for points inside the base pixels: longdouble xyz
    unit vectors (3, K)."""
    X = np.asarray(X, dtype=LD)
    Y = np.asarray(Y, dtype=LD)
    polar = np.abs(Y) > LD(0.5)
    sig = np.where(polar, 2 - 2 * np.abs(Y), LD(1))
    omz = sig * sig / 3                                   # 1 - |z| in the caps
    z = np.where(polar, np.sign(Y) * (1 - omz), LD(4) * Y / 3)
    st = np.where(polar, np.sqrt(omz * (2 - omz)), np.sqrt((1 - z) * (1 + z)))
    xc = np.floor(X) + LD(0.5)                            # centre of the quarter
    t = np.where(polar, xc + (X - xc) / sig, X)
    phi = t * (PI_LD / 2)
    return np.stack([st * np.sin(phi), z, st * np.cos(phi)])


def pix2xyz(j: int, pix) -> np.ndarray:
    """Centre of level-j nested pixels as longdouble xyz unit vectors (3, K)."""
    return unproject(*pixel_plane_centre(j, pix))


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
