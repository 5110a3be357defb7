"""Oracle: the conventional model-visibility predictor the paper compares the
wavelet route against (section 2.2, first step of the major cycle: a forward
FFT of the model image, then degridding with an anti-aliasing kernel and a
correction for the w-term).

TEST INFRASTRUCTURE (see oracle/__init__.py): plain NumPy, FP64.

The predictor is written here as a type-2 non-uniform FFT in (u, v, w) with
the "exponential of semicircle" kernel phi(z) = exp(beta (sqrt(1 - z^2) - 1)),
|z| <= 1 (Barnett, Magland & af Klinteberg 2019), and w handled by stacking
planes that are themselves interpolated with the same kernel (the improved
w-stacking of Ye et al. 2021).  For an image I_p on the grid of
oracle.clean.image_grid (pixel offsets t_x, t_y from the phase centre, cell
Delta, direction cosine n_p):

  uv grid:   N_x = 2 n_x, N_y = 2 n_y cells; grid units xi = u N_x Delta,
             zeta = v N_y Delta.
  w planes:  spacing dw = 1 / (2 E), E = the extent of n - 1 over the image;
             c = the midpoint of that range; plane q at w_q = w_0 + q dw,
             w_0 = min w - (W / 2) dw; eta = (w - w_0) / dw.
  kernel:    phi_W(x) = phi(2 x / W) over W cells (the same W in u, v, w),
             beta = 2.3 W; phi_hat(f) = int phi_W(x) cos(2 pi f x) dx.
  plane q:   G_q[k] = sum_p I_p e^{s 2 pi i w_q (n_p - 1 - c)}
                      / (phi_hat(t_x / N_x) phi_hat(t_y / N_y) phi_hat(dw (n_p - 1 - c)))
                      e^{s 2 pi i (k_x t_x / N_x + k_y t_y / N_y)}   (an FFT of the
             zero-padded image, pixel t at index t mod N)
  visibility: V_j = e^{s 2 pi i w_j c} sum_q phi_W(eta_j - q)
                    sum_k phi_W(xi_j - k_x) phi_W(zeta_j - k_y) G_q[k mod N]

By Poisson summation each kernel sum equals the exact phase factor times the
correction it is divided by, up to the kernel's aliasing error (about
10^(1 - W) at twofold padding), so V_j approximates the direct sum
sum_p I_p e^{s 2 pi i (u l_p + v m_p + w (n_p - 1))}.  What pins it: the
error against that direct sum falls with W and stays under the bound; a
source at the phase centre gives a smooth V; the quadrature converges.
"""
from __future__ import annotations

import numpy as np

from . import clean

BETA_PER_W = 2.3
N_QUAD = 100


def es_kernel(z, beta):
    """phi(z) = exp(beta (sqrt(1 - z^2) - 1)) on |z| <= 1, else 0."""
    z = np.asarray(z, np.float64)
    out = np.zeros_like(z)
    inside = np.abs(z) <= 1.0
    out[inside] = np.exp(beta * (np.sqrt(1.0 - z[inside] ** 2) - 1.0))
    return out


def es_hat(f, W: int, n_quad: int = N_QUAD):
    """phi_hat(f) = int_{-W/2}^{W/2} phi(2 x / W) cos(2 pi f x) dx.  With
    x = (W / 2) sin(theta) the integrand exp(beta (cos theta - 1))
    cos(2 pi f (W / 2) sin theta) cos theta is smooth on [-pi/2, pi/2], where
    Gauss-Legendre quadrature converges fast."""
    beta = BETA_PER_W * W
    t, wq = np.polynomial.legendre.leggauss(n_quad)        # nodes on [-1, 1]
    theta = 0.5 * np.pi * t
    f = np.asarray(f, np.float64)
    vals = (np.exp(beta * (np.cos(theta) - 1.0)) * np.cos(theta))[None, :] * np.cos(
        2 * np.pi * f.reshape(-1, 1) * (W / 2) * np.sin(theta)[None, :])
    return (vals @ wq).reshape(f.shape) * (0.5 * np.pi) * (W / 2)


def plan(nx: int, ny: int, cell: float, w, W: int):
    """Grid sizes and w planes for an (ny, nx) image and the rows' w."""
    l, m, nm1, inside = clean.image_grid(nx, ny, cell)
    if not inside.all():
        raise ValueError("image grid leaves the unit disk")
    lo, hi = float(nm1.min()), float(nm1.max())
    extent = max(hi - lo, 1e-300)
    c = 0.5 * (lo + hi)
    dw = 1.0 / (2.0 * extent)
    w = np.asarray(w, np.float64)
    w0 = float(w.min()) - (W / 2) * dw
    n_planes = int(np.floor((float(w.max()) - w0) / dw + W / 2)) + 1
    return {"Nx": 2 * nx, "Ny": 2 * ny, "dw": dw, "c": c, "w0": w0, "n_planes": n_planes,
            "l": l, "m": m, "nm1": nm1}


def predict_degrid(image, cell: float, u, v, w, W: int = 10, sign: int = -1):
    """Model visibilities of an (ny, nx) image by FFT + degridding (see the
    module docstring).  Returns complex128 [n_vis]."""
    I = np.asarray(image, np.float64)
    ny, nx = I.shape
    u, v, w = (np.asarray(a, np.float64) for a in (u, v, w))
    P = plan(nx, ny, cell, w, W)
    Nx, Ny, dw, c, w0, nq = P["Nx"], P["Ny"], P["dw"], P["c"], P["w0"], P["n_planes"]
    beta = BETA_PER_W * W
    cx, cy = nx // 2, ny // 2
    tx = np.arange(nx) - cx
    ty = np.arange(ny) - cy
    corr = (es_hat(ty / Ny, W)[:, None] * es_hat(tx / Nx, W)[None, :]
            * es_hat(dw * (P["nm1"].reshape(ny, nx) - c), W))
    base = I / corr
    shifted_n = P["nm1"].reshape(ny, nx) - c
    grids = np.empty((nq, Ny, Nx), np.complex128)
    for q in range(nq):
        wq = w0 + q * dw
        img = base * np.exp(sign * 2j * np.pi * wq * shifted_n)
        pad = np.zeros((Ny, Nx), np.complex128)
        pad[np.ix_(ty % Ny, tx % Nx)] = img
        # sum_t pad[t] e^{s 2 pi i k t / N}
        grids[q] = np.fft.fft2(pad) if sign < 0 else np.fft.ifft2(pad) * (Nx * Ny)
    xi = u * Nx * cell
    zeta = v * Ny * cell
    eta = (w - w0) / dw
    out = np.zeros(u.shape[0], np.complex128)
    half = W / 2
    for j in range(u.shape[0]):
        kx = np.arange(int(np.ceil(xi[j] - half)), int(np.floor(xi[j] + half)) + 1)
        ky = np.arange(int(np.ceil(zeta[j] - half)), int(np.floor(zeta[j] + half)) + 1)
        kq = np.arange(int(np.ceil(eta[j] - half)), int(np.floor(eta[j] + half)) + 1)
        fx = es_kernel((xi[j] - kx) / half, beta)
        fy = es_kernel((zeta[j] - ky) / half, beta)
        fq = es_kernel((eta[j] - kq) / half, beta)
        sub = grids[np.ix_(kq, ky % Ny, kx % Nx)]
        out[j] = np.einsum("q,y,x,qyx->", fq, fy, fx, sub)
    return out * np.exp(sign * 2j * np.pi * w * c)
