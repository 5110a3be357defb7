"""Oracle: direct model-visibility sum, its adjoint, chi^2 gradients, residual.

Plain, slow NumPy FP64.  Each function states the passage it follows.

Phase convention.  For a baseline B = (u, v, w) in wavelengths and a
component at direction cosines (l, m) the paper's direct sum (section 3.3,
Eq. 12 with the phase centre at [0, 0, 1]) has the phase, in cycles,

    phi = u l + v m + w (n - 1),   n = sqrt(1 - l^2 - m^2),

and the visibility V = sum_k I_k exp(s 2 pi i phi_k).  The paper prints
s = +1; the library takes s as an argument (default -1).  Point components
on the sphere carry no 1/n factor (Eq. 12 has none; the 1/n of Eq. 1 is the
Jacobian of dl dm, absorbed by a point measure on the sphere).

Exactness.  phi reaches ~10^4 cycles, where one FP64 ulp is ~2e-12 cycles.
The oracle therefore evaluates phi mod 1 without rounding the large
products: every product a*b is split exactly into p + e (Dekker's
TwoProduct on a Veltkamp split, Dekker 1971), the integer part of each p is
removed exactly (p - rint(p) is exact by Sterbenz' lemma), and only the
small remainders are added.  The reduced phase r in [-1/2, 1/2] is then
accurate to a few 1e-16 cycles, far below the GPU path's own rounding, so a
GPU/oracle difference measures the GPU path.
"""
from __future__ import annotations

import numpy as np

_VELTKAMP = 134217729.0   # 2**27 + 1


def n_minus_1(l, m):
    """n - 1 for the SIN-projected direction [l, m, n] (section 3.3), in the
    cancellation-free form -(l^2 + m^2) / (1 + sqrt(1 - l^2 - m^2))."""
    l = np.asarray(l, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    r2 = l * l + m * m
    return -r2 / (1.0 + np.sqrt(1.0 - r2))


def _split(a):
    c = _VELTKAMP * a
    hi = c - (c - a)
    return hi, a - hi


def _two_prod(a, b):
    """a*b = p + e exactly (Dekker's TwoProduct)."""
    p = a * b
    ah, al = _split(a)
    bh, bl = _split(b)
    e = ((ah * bh - p) + ah * bl + al * bh) + al * bl
    return p, e


def reduced_phase(u, v, w, l, m, nm1):
    """phi mod 1 in [-1/2, 1/2] for every (row, component) pair (Eq. 12's
    dot product B . (C - P) with P = [0, 0, 1]).  Shapes broadcast; pass
    rows as (R, 1) and components as (1, K)."""
    p1, e1 = _two_prod(u, l)
    p2, e2 = _two_prod(v, m)
    p3, e3 = _two_prod(w, nm1)
    r = (p1 - np.rint(p1)) + (p2 - np.rint(p2)) + (p3 - np.rint(p3)) + ((e1 + e2) + e3)
    return r - np.rint(r)


def phasors(u, v, w, l, m, nm1, sign=-1):
    """e_jk = exp(s 2 pi i phi_jk) as a complex (R, K) array."""
    r = reduced_phase(np.asarray(u)[:, None], np.asarray(v)[:, None], np.asarray(w)[:, None],
                      np.asarray(l)[None, :], np.asarray(m)[None, :], np.asarray(nm1)[None, :])
    ang = 2.0 * np.pi * r
    return np.cos(ang) + 1j * (sign * np.sin(ang))


def _check_sign(sign):
    if sign not in (-1, 1):
        raise ValueError("sign must be +1 or -1")


def predict_direct(u, v, w, l, m, flux, sign=-1, nm1=None, chunk=2048):
    """Direct component sum, Eq. 12 (section 3.3):

        V_j = sum_k I_k exp(s 2 pi i (u_j l_k + v_j m_k + w_j (n_k - 1))).

    ``flux`` may be complex (a general linear map, used for the adjoint
    identity).  ``nm1`` overrides n - 1 (pixel centres on the far side of the
    sphere have n < 0, which (l, m) alone cannot express).  Returns complex128."""
    _check_sign(sign)
    u = np.asarray(u, np.float64)
    v = np.asarray(v, np.float64)
    w = np.asarray(w, np.float64)
    l = np.asarray(l, np.float64)
    m = np.asarray(m, np.float64)
    nm1 = n_minus_1(l, m) if nm1 is None else np.asarray(nm1, np.float64)
    a = np.asarray(flux).astype(np.complex128)
    out = np.empty(u.shape[0], np.complex128)
    for s in range(0, u.shape[0], chunk):
        e = phasors(u[s:s + chunk], v[s:s + chunk], w[s:s + chunk], l, m, nm1, sign)
        out[s:s + chunk] = e @ a
    return out


def predict_direct_fp64(u, v, w, l, m, flux, sign=-1, nm1=None, chunk=1024):
    """Eq. 12 as predict_direct, with the phase u l + v m + w (n - 1) formed in
    plain FP64 arithmetic (then reduced by rint) instead of error-free
    products: its error is a few units in the last place of the phase, about
    2 pi 3 2^-53 |phi| per term, and it runs several times faster, for inputs
    of full workload size (the observed visibilities of a perturbed model)."""
    _check_sign(sign)
    u = np.asarray(u, np.float64)
    v = np.asarray(v, np.float64)
    w = np.asarray(w, np.float64)
    l = np.asarray(l, np.float64)
    m = np.asarray(m, np.float64)
    nm1 = n_minus_1(l, m) if nm1 is None else np.asarray(nm1, np.float64)
    a = np.asarray(flux, np.float64)
    out = np.empty(u.shape[0], np.complex128)
    for s in range(0, u.shape[0], chunk):
        sl = slice(s, s + chunk)
        ph = np.outer(u[sl], l) + np.outer(v[sl], m) + np.outer(w[sl], nm1)
        ang = 2.0 * np.pi * (ph - np.rint(ph))
        out[sl] = np.cos(ang) @ a + 1j * (sign * (np.sin(ang) @ a))
    return out


def adjoint(u, v, w, y, l, m, nm1, sign=-1, chunk=2048):
    """Adjoint of predict_direct on a pixel set p = (l, m, n-1):

        x_p = sum_j conj(e_jp) y_j.

    With y the residual visibilities this is the residual (dirty) image on
    the sphere pixels, the step the major cycle performs after the subtract
    (section 2.2, third step) written as the exact transpose of Eq. 12
    instead of gridding and an FFT."""
    _check_sign(sign)
    y = np.asarray(y, np.complex128)
    out = np.zeros(np.asarray(l).shape[0], np.complex128)
    for s in range(0, y.shape[0], chunk):
        e = phasors(u[s:s + chunk], v[s:s + chunk], w[s:s + chunk], l, m, nm1, sign)
        out += np.conj(e).T @ y[s:s + chunk]
    return out


def grad_direct(u, v, w, y, l, m, flux, sign=-1, alpha=1.0, chunk=2048):
    """Real gradient of alpha * Re sum_j conj(y_j) V_j(theta) with respect to the
    real component parameters theta = (I_k, l_k, m_k), V from Eq. 12:

        dV_j/dI_k = e_jk
        dV_j/dl_k = I_k s 2 pi i (u_j - w_j l_k / n_k) e_jk     (dn/dl = -l/n)
        dV_j/dm_k = I_k s 2 pi i (v_j - w_j m_k / n_k) e_jk

    With y = r (residuals) and alpha = -2/sigma^2 this is the gradient of
    chi^2 = sum |V_obs - V|^2 / sigma^2; with y = dL/dV* and alpha = 1 it is
    the backward of a real loss L.  Returns (d_flux, d_l, d_m)."""
    _check_sign(sign)
    u = np.asarray(u, np.float64)
    v = np.asarray(v, np.float64)
    w = np.asarray(w, np.float64)
    l = np.asarray(l, np.float64)
    m = np.asarray(m, np.float64)
    flux = np.asarray(flux, np.float64)
    nm1 = n_minus_1(l, m)
    n = 1.0 + nm1
    y = np.asarray(y, np.complex128)
    gI = np.zeros(l.shape[0])
    gl = np.zeros(l.shape[0])
    gm = np.zeros(l.shape[0])
    for s in range(0, u.shape[0], chunk):
        sl = slice(s, s + chunk)
        e = phasors(u[sl], v[sl], w[sl], l, m, nm1, sign)
        cy = np.conj(y[sl])[:, None]
        dVdI = e
        dVdl = flux[None, :] * (sign * 2j * np.pi) * (u[sl][:, None] - w[sl][:, None] * (l / n)[None, :]) * e
        dVdm = flux[None, :] * (sign * 2j * np.pi) * (v[sl][:, None] - w[sl][:, None] * (m / n)[None, :]) * e
        gI += np.real(np.sum(cy * dVdI, axis=0))
        gl += np.real(np.sum(cy * dVdl, axis=0))
        gm += np.real(np.sum(cy * dVdm, axis=0))
    return alpha * gI, alpha * gl, alpha * gm


def residual_chi2(vis_obs, vis_model, inv_sigma2):
    """Subtract step of the major cycle (section 2.2): r = V_obs - V_model,
    and chi^2 = sum_j |r_j|^2 / sigma^2."""
    r = np.asarray(vis_obs, np.complex128) - np.asarray(vis_model, np.complex128)
    chi2 = float(np.sum(r.real * r.real + r.imag * r.imag) * inv_sigma2)
    return r, chi2
