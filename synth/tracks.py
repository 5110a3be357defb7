"""Seeded synthetic interferometer (u, v, w) tracks.

This module only manufactures inputs. It holds none of the visibility
arithmetic of the method (no phase, no plane wave, no sum over components):
it places antennas, forms baselines and rotates them with the Earth, using
the textbook relations of aperture synthesis (Thompson, Moran & Swenson,
"Interferometry and Synthesis in Radio Astronomy", ch. 4).  Both the GPU
path and the CPU oracle are fed from here, and neither is imported here.

Conventions
-----------
* Antenna positions are local east/north/up (ENU) metres at a site of
  geodetic latitude ``lat`` (radians).
* Baseline ``b = x_q - x_p`` for every antenna pair ``p < q``.
* Equatorial baseline components (X towards hour angle 0 / declination 0,
  Y towards hour angle -6h, Z towards the celestial pole)::

      X = -N sin(lat) + U cos(lat),  Y = E,  Z = N cos(lat) + U sin(lat)

* (u, v, w) towards a source at hour angle H, declination dec::

      u =  sin H X + cos H Y
      v = -sin dec cos H X + sin dec sin H Y + cos dec Z
      w =  cos dec cos H X - cos dec sin H Y + sin dec Z

  divided by the wavelength, so (u, v, w) are in wavelengths (FP64).
* Rows are time-major: row = t * n_baselines + baseline.
"""
from __future__ import annotations

import numpy as np

C_LIGHT = 299_792_458.0          # m/s
SIDEREAL_DAY_S = 86_164.0905     # s
SITE_LAT_DEG = 34.08             # a JVLA-like site latitude


def antennas_in_disk(n_ant: int, radius_m: float, rng: np.random.Generator) -> np.ndarray:
    """Antennas uniform in a disk of the given radius: r = R sqrt(U), theta = 2 pi U'.

    Returns an (n_ant, 3) array of ENU metres (up = 0)."""
    r = radius_m * np.sqrt(rng.random(n_ant))
    th = 2.0 * np.pi * rng.random(n_ant)
    enu = np.zeros((n_ant, 3))
    enu[:, 0] = r * np.cos(th)
    enu[:, 1] = r * np.sin(th)
    return enu


def baseline_pairs(n_ant: int) -> tuple[np.ndarray, np.ndarray]:
    """Index arrays (p, q) of all pairs p < q, in row-major order."""
    p, q = np.triu_indices(n_ant, k=1)
    return p.astype(np.int64), q.astype(np.int64)


def enu_to_equatorial(enu: np.ndarray, lat: float) -> np.ndarray:
    """Local ENU vectors -> equatorial (X, Y, Z) vectors (same units)."""
    e, n, up = enu[..., 0], enu[..., 1], enu[..., 2]
    out = np.empty_like(enu)
    out[..., 0] = -n * np.sin(lat) + up * np.cos(lat)
    out[..., 1] = e
    out[..., 2] = n * np.cos(lat) + up * np.sin(lat)
    return out


def hour_angles(duration_s: float, n_t: int) -> np.ndarray:
    """Hour angles (radians) at the midpoints of n_t equal bins, symmetric about transit."""
    t = (np.arange(n_t) + 0.5) * (duration_s / n_t) - 0.5 * duration_s
    return 2.0 * np.pi * t / SIDEREAL_DAY_S


def uvw_from_baselines(bxyz: np.ndarray, H: np.ndarray, dec: float, freq_hz: float):
    """(u, v, w) in wavelengths for every (time, baseline), time-major, as three
    contiguous FP64 arrays of length len(H) * len(bxyz)."""
    lam = C_LIGHT / freq_hz
    X = bxyz[:, 0][None, :]
    Y = bxyz[:, 1][None, :]
    Z = bxyz[:, 2][None, :]
    sH = np.sin(H)[:, None]
    cH = np.cos(H)[:, None]
    sd, cd = np.sin(dec), np.cos(dec)
    u = (sH * X + cH * Y) / lam
    v = (-sd * cH * X + sd * sH * Y + cd * Z) / lam
    w = (cd * cH * X - cd * sH * Y + sd * Z) / lam
    return (np.ascontiguousarray(u.ravel()), np.ascontiguousarray(v.ravel()),
            np.ascontiguousarray(w.ravel()))


def array_tracks(n_ant: int, radius_m: float, dec_deg: float, duration_s: float,
                 n_t: int, freq_hz: float, seed: int, lat_deg: float = SITE_LAT_DEG):
    """Full Earth-rotation tracks of a seeded random array. Returns (u, v, w)."""
    rng = np.random.default_rng(seed)
    enu = antennas_in_disk(n_ant, radius_m, rng)
    p, q = baseline_pairs(n_ant)
    bxyz = enu_to_equatorial(enu[q] - enu[p], np.deg2rad(lat_deg))
    H = hour_angles(duration_s, n_t)
    return uvw_from_baselines(bxyz, H, np.deg2rad(dec_deg), freq_hz)


def array_baselines_xyz(n_ant: int, radius_m: float, seed: int,
                        lat_deg: float = SITE_LAT_DEG) -> np.ndarray:
    """Equatorial baseline vectors (metres) of the seeded array, shape (n_bl, 3)."""
    rng = np.random.default_rng(seed)
    enu = antennas_in_disk(n_ant, radius_m, rng)
    p, q = baseline_pairs(n_ant)
    return enu_to_equatorial(enu[q] - enu[p], np.deg2rad(lat_deg))


def uvw_rows(bxyz: np.ndarray, n_t: int, duration_s: float, dec_deg: float,
             freq_hz: float, rows: np.ndarray):
    """(u, v, w) of selected time-major rows only (row = t * n_bl + b).

    Evaluates the same expressions as uvw_from_baselines, element by element,
    so a sampled row equals the corresponding row of the full track."""
    n_bl = bxyz.shape[0]
    rows = np.asarray(rows, dtype=np.int64)
    t = rows // n_bl
    b = rows % n_bl
    H = hour_angles(duration_s, n_t)[t]
    lam = C_LIGHT / freq_hz
    X, Y, Z = bxyz[b, 0], bxyz[b, 1], bxyz[b, 2]
    sH, cH = np.sin(H), np.cos(H)
    dec = np.deg2rad(dec_deg)
    sd, cd = np.sin(dec), np.cos(dec)
    u = (sH * X + cH * Y) / lam
    v = (-sd * cH * X + sd * sH * Y + cd * Z) / lam
    w = (cd * cH * X - cd * sH * Y + sd * Z) / lam
    return u, v, w
