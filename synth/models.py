"""Seeded synthetic clean-component models, residuals and noise.

Inputs only: positions are direction cosines (l, m) in a square field
|l|, |m| <= sin(F/2) around the phase centre, fluxes are lognormal Jy.
No part of the method's arithmetic lives here.
"""
from __future__ import annotations

import numpy as np


def half_width(field_deg: float) -> float:
    """Half-width in direction cosines of a square field of full width ``field_deg``."""
    return float(np.sin(np.deg2rad(field_deg) / 2.0))


def lognormal_fluxes(n: int, rng: np.random.Generator, mu: float = -3.0, sigma: float = 1.0):
    return rng.lognormal(mean=mu, sigma=sigma, size=n)


def uniform_components(n: int, field_deg: float, rng: np.random.Generator):
    """(l, m, flux): n components uniform in a square field of full width field_deg."""
    h = half_width(field_deg)
    l = rng.uniform(-h, h, n)
    m = rng.uniform(-h, h, n)
    return l, m, lognormal_fluxes(n, rng)


def blob_mixture_components(n_total: int, frac_clustered: float, n_blobs: int,
                            blob_sigma_deg: float, blob_centre_field_deg: float,
                            uniform_field_deg: float, rng: np.random.Generator):
    """A mixture: round(frac * n) components in n_blobs Gaussian blobs (sigma per
    axis blob_sigma_deg, blob centres uniform in a field of full width
    blob_centre_field_deg), the rest uniform over uniform_field_deg."""
    n_cl = int(round(frac_clustered * n_total))
    n_un = n_total - n_cl
    hc = half_width(blob_centre_field_deg)
    centres = rng.uniform(-hc, hc, size=(n_blobs, 2))
    which = rng.integers(0, n_blobs, n_cl)
    sig = np.sin(np.deg2rad(blob_sigma_deg))
    lc = centres[which, 0] + sig * rng.standard_normal(n_cl)
    mc = centres[which, 1] + sig * rng.standard_normal(n_cl)
    hu = half_width(uniform_field_deg)
    lu = rng.uniform(-hu, hu, n_un)
    mu = rng.uniform(-hu, hu, n_un)
    l = np.concatenate([lc, lu])
    m = np.concatenate([mc, mu])
    return l, m, lognormal_fluxes(n_total, rng)


def perturb_model(l, m, flux, rng: np.random.Generator, flux_frac_sigma: float = 0.05,
                  pos_sigma_rad: float = np.deg2rad(1.0 / 3600.0)):
    """Fluxes x (1 + N(0, flux_frac_sigma)), positions + N(0, pos_sigma) per axis."""
    n = len(flux)
    f2 = flux * (1.0 + flux_frac_sigma * rng.standard_normal(n))
    l2 = l + pos_sigma_rad * rng.standard_normal(n)
    m2 = m + pos_sigma_rad * rng.standard_normal(n)
    return l2, m2, f2


def complex_noise(n: int, sigma: float, rng: np.random.Generator) -> np.ndarray:
    """Complex Gaussian noise, real and imaginary parts each N(0, sigma^2)."""
    return sigma * rng.standard_normal(n) + 1j * sigma * rng.standard_normal(n)


def random_complex(n: int, rng: np.random.Generator, scale: float = 1.0) -> np.ndarray:
    return scale * (rng.standard_normal(n) + 1j * rng.standard_normal(n))
