"""Oracle: the clean loop around the predictor (sections 2.1, 2.2, 3.5).

TEST INFRASTRUCTURE (see oracle/__init__.py): plain NumPy, FP64, written
from the paper's description of Hogbom clean, the Cotton-Schwab major and
minor cycles and the wavelet-clean cross-reference table.

image_grid       the SIN-projected image pixels [l, m] of a regular grid.
dirty_image      (1/N_vis) Re sum_j conj(e_jp) y_j: the exact adjoint of the
                 direct sum in place of gridding and the inverse FFT (the
                 first two steps of section 2.1, third step of section 2.2).
dirty_beam       the dirty image of a unit source at the phase centre, on the
                 grid of pixel offsets (-(n-1) .. n-1) that Eq. 4 shifts.
hogbom           Eqs. 4 and 5: repeatedly take the peak pixel C_n, record the
                 clean component g C_n and subtract g C_n times the beam
                 shifted to it.
cross_reference  image pixel -> level-J sphere pixel (section 3.5).
tree_from_pixels the coefficient tree of clean components given by their
                 level-J pixels (section 3.5: k_j = k_J >> 2(J - j)).
fit_clean_beam   the clean beam B_C: a rotated 2-D Gaussian fitted to the
                 dirty beam's main lobe (section 2.1, third step).
restore          Eq. 6: the components convolved with B_C.
wavelet_clean    the whole loop: minor cycles of hogbom, major cycles that
                 predict the model visibilities by the wavelet tree, subtract
                 them and form the new residual image.

Readings of the paper where it leaves a choice (each also fixed by the GPU
library): the peak is the largest pixel value (or the largest magnitude with
absolute=True), the first such pixel in row-major order on ties; the minor
cycle stops when that peak is not above the threshold or after max_iter
components; beam pixels whose direction lies off the unit disk are zero; the
main lobe is the 8-connected region of beam >= 1/2 around the centre, and
the Gaussian is the least-squares fit of ln B over it.
"""
from __future__ import annotations

from collections import deque

import numpy as np

from . import sphere, tree, visibility


def image_grid(nx: int, ny: int, cell: float, cx: int | None = None, cy: int | None = None):
    """Pixel p = iy * nx + ix sits at l = (ix - cx) cell, m = (iy - cy) cell
    (default centre (nx // 2, ny // 2)); n - 1 from the SIN projection.
    Returns (l, m, nm1, inside) with inside = l^2 + m^2 < 1; nm1 is 0 where
    the direction is off the disk."""
    cx = nx // 2 if cx is None else cx
    cy = ny // 2 if cy is None else cy
    iy, ix = np.divmod(np.arange(nx * ny, dtype=np.int64), nx)
    l = (ix - cx).astype(np.float64) * cell
    m = (iy - cy).astype(np.float64) * cell
    r2 = l * l + m * m
    inside = r2 < 1.0
    nm1 = np.zeros_like(l)
    nm1[inside] = visibility.n_minus_1(l[inside], m[inside])
    return l, m, nm1, inside


def dirty_image(u, v, w, y, l, m, nm1, sign=-1):
    """Real image (1/N_vis) Re sum_j conj(e_jp) y_j on the pixels (l, m, n-1):
    a unit source at a pixel gives 1 there."""
    n = np.asarray(u).shape[0]
    x = visibility.adjoint(u, v, w, y, l, m, nm1, sign)
    return x.real / n


def dirty_beam(u, v, w, nx: int, ny: int, cell: float, sign=-1):
    """Beam on the (2 ny - 1) x (2 nx - 1) grid of pixel offsets, centre at
    (ny - 1, nx - 1): the dirty image of unit visibilities, i.e. of a unit
    source at the phase centre.  Zero where the offset direction is off the
    unit disk."""
    bl, bm, bnm1, inside = image_grid(2 * nx - 1, 2 * ny - 1, cell, nx - 1, ny - 1)
    n = np.asarray(u).shape[0]
    beam = np.zeros(bl.shape[0])
    ones = np.ones(n, np.complex128)
    beam[inside] = dirty_image(u, v, w, ones, bl[inside], bm[inside], bnm1[inside], sign)
    return beam.reshape(2 * ny - 1, 2 * nx - 1)


def hogbom(image, beam, gain: float, threshold: float, max_iter: int, absolute=False):
    """Eqs. 4-5 on a (ny, nx) image with a (2 ny - 1, 2 nx - 1) beam.

    Each iteration takes the peak pixel p_n (value C_n), stops if the peak is
    not above `threshold`, records (p_n, g C_n) and subtracts g C_n times the
    beam centred on p_n.  Returns (residual image, pixel ids, component
    values g C_n) in the order found."""
    I = np.array(image, dtype=np.float64, copy=True)
    ny, nx = I.shape
    B = np.asarray(beam, np.float64)
    if B.shape != (2 * ny - 1, 2 * nx - 1):
        raise ValueError("beam must be (2 ny - 1, 2 nx - 1)")
    pix, val = [], []
    for _ in range(int(max_iter)):
        key = np.abs(I) if absolute else I
        p = int(np.argmax(key))            # first maximum in row-major order
        if not key.flat[p] > threshold:
            break
        py, px = divmod(p, nx)
        gC = gain * I.flat[p]
        I -= gC * B[ny - 1 - py:2 * ny - 1 - py, nx - 1 - px:2 * nx - 1 - px]
        pix.append(p)
        val.append(gC)
    return I, np.asarray(pix, np.int64), np.asarray(val, np.float64)


def cross_reference(J: int, ra_p: float, dec_p: float, l, m):
    """Level-J sphere pixel of every image pixel (section 3.5): [l, m, n] is
    rotated to the equatorial frame and located in the nested pixelisation."""
    xyz = sphere.lm_to_xyz(np.asarray(l, np.float64), np.asarray(m, np.float64), ra_p, dec_p)
    return sphere.ang2pix_xyz(J, xyz)


def tree_from_pixels(J: int, ra_p: float, dec_p: float, kJ, flux) -> tree.Tree:
    """Coefficient tree of components given by their level-J pixels: components
    sharing a pixel are summed into one leaf at the pixel centre."""
    leaf, inv = np.unique(np.asarray(kJ, np.int64), return_inverse=True)
    F = np.bincount(inv, weights=np.asarray(flux, np.float64), minlength=leaf.shape[0])
    ll, mm, nm1 = sphere.pixel_centres_lmn(J, leaf, ra_p, dec_p)
    return tree.Tree(J, ra_p, dec_p, leaf, F, ll, mm, nm1, tree.build_levels(J, leaf, F))


def main_lobe(beam):
    """(dy, dx) offsets of the 8-connected region of beam >= 1/2 that holds
    the centre pixel."""
    B = np.asarray(beam, np.float64)
    nby, nbx = B.shape
    cy, cx = nby // 2, nbx // 2
    if not B[cy, cx] >= 0.5:
        raise ValueError("beam centre below 1/2")
    seen = np.zeros(B.shape, bool)
    seen[cy, cx] = True
    todo = deque([(cy, cx)])
    cells = []
    while todo:
        y, x = todo.popleft()
        cells.append((y - cy, x - cx))
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                yy, xx = y + dy, x + dx
                if 0 <= yy < nby and 0 <= xx < nbx and not seen[yy, xx] and B[yy, xx] >= 0.5:
                    seen[yy, xx] = True
                    todo.append((yy, xx))
    return np.asarray(cells, np.int64)


def fit_clean_beam(beam):
    """Clean beam B_C(dx, dy) = exp(-(a dx^2 + 2 b dx dy + c dy^2)), offsets in
    pixels: the least-squares fit of -ln B over the main lobe.  Returns
    (a, b, c); raises if the lobe does not determine the three parameters or
    the fit is not a peaked Gaussian."""
    B = np.asarray(beam, np.float64)
    cells = main_lobe(B)
    if cells.shape[0] < 4:
        raise ValueError("main lobe narrower than the pixel grid resolves")
    dy = cells[:, 0].astype(np.float64)
    dx = cells[:, 1].astype(np.float64)
    vals = B[cells[:, 0] + B.shape[0] // 2, cells[:, 1] + B.shape[1] // 2]
    A = np.stack([dx * dx, 2.0 * dx * dy, dy * dy], axis=1)
    coef, _, rank, _ = np.linalg.lstsq(A, -np.log(vals), rcond=None)
    if rank < 3:
        raise ValueError("main lobe does not determine the three parameters")
    a, b, c = (float(t) for t in coef)
    if not (a > 0 and c > 0 and a * c - b * b > 0):
        raise ValueError("fitted clean beam is not a peaked Gaussian")
    return a, b, c


def restore(nx: int, ny: int, comp_pix, comp_val, abc, residual=None):
    """Eq. 6: I_C = sum_i g C_i B_C(. - p_i), term by term in list order, plus
    the residual image if one is given.  Returns a (ny, nx) image."""
    a, b, c = abc
    iy, ix = np.divmod(np.arange(nx * ny, dtype=np.int64), nx)
    out = np.zeros(nx * ny)
    for p, g in zip(np.asarray(comp_pix, np.int64), np.asarray(comp_val, np.float64)):
        qy, qx = divmod(int(p), nx)
        dx = (ix - qx).astype(np.float64)
        dy = (iy - qy).astype(np.float64)
        out += g * np.exp(-(a * dx * dx + 2.0 * b * dx * dy + c * dy * dy))
    out = out.reshape(ny, nx)
    if residual is not None:
        out = out + np.asarray(residual, np.float64).reshape(ny, nx)
    return out


def wavelet_clean(u, v, w, vis_obs, nx: int, ny: int, cell: float, J: int, ra_p: float,
                  dec_p: float, gain: float, threshold: float, minor_iter: int, n_major: int,
                  absolute=False, sign=-1, predictor="tree", support=10):
    """Cotton-Schwab cleaning with the wavelet predictor (sections 2.2, 3.5).

    Before the loop: the image grid, the dirty beam, the cross-reference table
    and the dirty image.  Each major cycle runs up to minor_iter Hogbom
    iterations on the residual image, then builds the tree of every component
    found so far, predicts the model visibilities by Eq. 17, subtracts them
    from the observed ones and forms the new residual image.  Stops after
    n_major cycles or when a minor cycle finds no component.

    predictor "degrid" or "direct" runs the same loop with the model image
    (components summed per pixel in list order) predicted by FFT + degridding
    (oracle.degrid, kernel width `support`) or by the direct sum over its
    non-zero pixels: the conventional clean and the exact one.

    Returns a dict: pix, val (all components, in order), residual (ny, nx),
    beam, vis_model, kJ (cross-reference), cycles (per cycle: components
    found, distinct leaves or model pixels, chi^2 = sum |residual visibility|^2)."""
    from . import degrid
    if predictor not in ("tree", "degrid", "direct"):
        raise ValueError("predictor must be tree, degrid or direct")
    l, m, nm1, inside = image_grid(nx, ny, cell)
    if not inside.all():
        raise ValueError("image grid leaves the unit disk")
    beam = dirty_beam(u, v, w, nx, ny, cell, sign)
    kJ = cross_reference(J, ra_p, dec_p, l, m)
    vis_obs = np.asarray(vis_obs, np.complex128)
    resid = dirty_image(u, v, w, vis_obs, l, m, nm1, sign).reshape(ny, nx)
    pix = np.zeros(0, np.int64)
    val = np.zeros(0)
    vis_model = np.zeros_like(vis_obs)
    cycles = []
    for _ in range(int(n_major)):
        resid, p_new, v_new = hogbom(resid, beam, gain, threshold, minor_iter, absolute)
        if p_new.shape[0] == 0:
            break
        pix = np.concatenate([pix, p_new])
        val = np.concatenate([val, v_new])
        if predictor == "tree":
            t = tree_from_pixels(J, ra_p, dec_p, kJ[pix], val)
            vis_model = tree.predict_tree(t, u, v, w, sign)
            leaves = t.n_leaves
        else:
            model = np.zeros(nx * ny)
            for p, g in zip(pix, val):          # list order
                model[p] += g
            nz = np.nonzero(model)[0]
            leaves = int(nz.shape[0])
            if predictor == "degrid":
                vis_model = degrid.predict_degrid(model.reshape(ny, nx), cell, u, v, w, support,
                                                  sign)
            else:
                vis_model = visibility.predict_direct(u, v, w, l[nz], m[nz], model[nz], sign)
        r = vis_obs - vis_model
        resid = dirty_image(u, v, w, r, l, m, nm1, sign).reshape(ny, nx)
        cycles.append({"found": int(p_new.shape[0]), "leaves": leaves,
                       "chi2": float(np.sum(np.abs(r) ** 2))})
    return {"pix": pix, "val": val, "residual": resid, "beam": beam, "vis_model": vis_model,
            "kJ": kJ, "cycles": cycles}
