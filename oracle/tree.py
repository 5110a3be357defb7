"""Oracle: the spherical-Haar wavelet tree route (sections 3.2-3.5).

Steps, in the paper's order and notation:

1. Each component [l, m, n] (SIN projection, section 3.3) is rotated to xyz
   (Eq. 18) and assigned to its level-J pixel k_J (section 3.5); components
   in the same pixel are summed (the "distinct" components, section 3.3).
2. The level-J model scaling coefficient of each occupied pixel is its flux
   density, lambda_{J,k} = F_k / A_J (reading of the garbled Eq. 17
   normalisation: lambda as a mean value over the pixel, consistent with
   Eq. 9's 1/4 average and Eq. 10's orthonormal sqrt(A_j)/4 factor).
3. Coarser coefficients of existing nodes, j = J-1 ... 1 (Eqs. 9, 10):
       lambda_{j,k}   = 1/4 sum_c lambda_{j+1,4k+c}
       gamma^m_{j,k}  = sqrt(A_j)/4 sum_c s^m_c lambda_{j+1,4k+c}
   with the sign patterns of Eq. 10 (rows m = 0, 1, 2; columns c = 0..3).
   Node ids of ancestors are k_j = k_J >> 2 (J - j) (section 3.5).  Absent
   children are zero and are skipped (the tree stores no zero branch).
4. Per visibility, the plane wave F^P(s, B) = exp(s 2 pi i B . (s - P))
   (Eq. 14) at the leaf pixel centres gives eta_{J,k}; the same two formulas
   applied to eta give eta_{j,k} and sigma^m_{j,k} (section 3.3, last
   paragraphs; section 3.5).
5. Reconstruction (Eq. 17 with the normalisation of step 2):
       V = A_1 sum_k lambda_{1,k} eta_{1,k} + sum_{j<J} sum_k sum_m gamma^m sigma^m.

Because the 4x4 sign matrix H (rows: all-plus and the three patterns) has
H H^T = 4 I, step 5 equals sum_k F_k eta_{J,k} exactly: the tree route is the
direct sum over pixel-snapped components (Eq. 16).  `predict_snapped`
evaluates that plain definition; `predict_tree` evaluates steps 4-5.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import sphere
from .visibility import phasors, predict_direct

# Eq. 10 sign patterns s^m_c: row m = wavelet type, column c = child 4k + c.
WAVELET_SIGNS = np.array([[+1, -1, +1, -1],
                          [+1, +1, -1, -1],
                          [+1, -1, -1, +1]], dtype=np.float64)


@dataclass
class Level:
    j: int
    pix: np.ndarray                  # sorted nested ids of existing nodes
    lam: np.ndarray                  # lambda_{j,k}
    gamma: np.ndarray | None = None  # (n, 3) gamma^m_{j,k}, j < J
    child: np.ndarray | None = None  # (n, 4) index into level j+1 or -1, j < J


@dataclass
class Tree:
    J: int
    ra_p: float
    dec_p: float
    leaf_pix: np.ndarray
    leaf_flux: np.ndarray
    leaf_l: np.ndarray
    leaf_m: np.ndarray
    leaf_nm1: np.ndarray
    levels: list = field(default_factory=list)   # levels[j-1] is level j

    @property
    def n_leaves(self) -> int:
        return int(self.leaf_pix.shape[0])

    @property
    def n_internal(self) -> int:
        return int(sum(lv.pix.shape[0] for lv in self.levels[:-1]))


def snap_components(J, ra_p, dec_p, l, m, flux):
    """Steps 1: level-J pixel of every component and the merged leaves.
    Returns (k_J per component, sorted leaf ids, summed leaf flux)."""
    xyz = sphere.lm_to_xyz(l, m, ra_p, dec_p)
    kJ = sphere.ang2pix_xyz(J, xyz)
    leaf, inv = np.unique(kJ, return_inverse=True)
    F = np.bincount(inv, weights=np.asarray(flux, np.float64), minlength=leaf.shape[0])
    return kJ, leaf, F


def build_levels(J, leaf_pix, leaf_flux):
    """Steps 2-3: model coefficients of every existing node, levels J..1."""
    levels = [None] * J
    levels[J - 1] = Level(J, leaf_pix, leaf_flux / sphere.pixel_area(J))
    for j in range(J - 1, 0, -1):
        below = levels[j]                       # level j + 1
        parent = below.pix >> 2
        c = (below.pix & 3).astype(np.int64)
        pix, inv = np.unique(parent, return_inverse=True)
        child = -np.ones((pix.shape[0], 4), dtype=np.int64)
        child[inv, c] = np.arange(below.pix.shape[0])
        lam = np.zeros(pix.shape[0])
        gamma = np.zeros((pix.shape[0], 3))
        a = np.sqrt(sphere.pixel_area(j)) / 4.0
        for cc in range(4):
            has = child[:, cc] >= 0
            vals = below.lam[child[has, cc]]
            lam[has] += vals
            gamma[has] += WAVELET_SIGNS[:, cc][None, :] * vals[:, None]
        levels[j - 1] = Level(j, pix, 0.25 * lam, a * gamma, child)
    return levels


def build_tree(J, ra_p, dec_p, l, m, flux) -> Tree:
    """The sparse coefficient tree of a component list (section 3.5)."""
    if not 1 <= J <= 29:
        raise ValueError("J must be in [1, 29]")
    _, leaf, F = snap_components(J, ra_p, dec_p, l, m, flux)
    ll, mm, nm1 = sphere.pixel_centres_lmn(J, leaf, ra_p, dec_p)
    return Tree(J, ra_p, dec_p, leaf, F, ll, mm, nm1, build_levels(J, leaf, F))


def build_full_tree(J, ra_p, dec_p, l, m, flux) -> Tree:
    """Like build_tree but with every one of the N_J pixels as a leaf (zero flux
    where empty): the unmasked transform, for small J only."""
    _, leaf, F = snap_components(J, ra_p, dec_p, l, m, flux)
    allpix = np.arange(sphere.n_pixels(J), dtype=np.int64)
    Fall = np.zeros(allpix.shape[0])
    Fall[leaf] = F
    ll, mm, nm1 = sphere.pixel_centres_lmn(J, allpix, ra_p, dec_p)
    return Tree(J, ra_p, dec_p, allpix, Fall, ll, mm, nm1, build_levels(J, allpix, Fall))


def plane_wave_coefficients(tree: Tree, u, v, w, sign=-1):
    """Step 4 for a block of visibilities: per level j, eta_j (R, n_j) and, for
    j < J, sigma_j (R, n_j, 3)."""
    J = tree.J
    eta = [None] * J
    sig = [None] * J
    eta[J - 1] = phasors(u, v, w, tree.leaf_l, tree.leaf_m, tree.leaf_nm1, sign)
    for j in range(J - 1, 0, -1):
        lv = tree.levels[j - 1]
        below = eta[j]
        R = below.shape[0]
        e = np.zeros((R, lv.pix.shape[0]), np.complex128)
        s = np.zeros((R, lv.pix.shape[0], 3), np.complex128)
        a = np.sqrt(sphere.pixel_area(j)) / 4.0
        for cc in range(4):
            has = lv.child[:, cc] >= 0
            vals = below[:, lv.child[has, cc]]
            e[:, has] += vals
            s[:, has, :] += WAVELET_SIGNS[:, cc][None, None, :] * vals[:, :, None]
        eta[j - 1] = 0.25 * e
        sig[j - 1] = a * s
    return eta, sig


def reconstruct(tree: Tree, eta, sig):
    """Step 5: Eq. 17 with the A_1 factor on the scaling term."""
    V = sphere.pixel_area(1) * (eta[0] @ tree.levels[0].lam)
    for j in range(1, tree.J):
        lv = tree.levels[j - 1]
        V = V + np.einsum("rkm,km->r", sig[j - 1], lv.gamma)
    return V


def predict_tree(tree: Tree, u, v, w, sign=-1, chunk=1024):
    """Model visibilities by the wavelet route (steps 4-5), chunked over rows."""
    u = np.asarray(u, np.float64)
    v = np.asarray(v, np.float64)
    w = np.asarray(w, np.float64)
    out = np.empty(u.shape[0], np.complex128)
    for s in range(0, u.shape[0], chunk):
        sl = slice(s, s + chunk)
        eta, sig = plane_wave_coefficients(tree, u[sl], v[sl], w[sl], sign)
        out[sl] = reconstruct(tree, eta, sig)
    return out


def predict_snapped(tree: Tree, u, v, w, sign=-1):
    """Eq. 16's plain form: the direct sum over the merged leaves at their pixel
    centres, V = sum_k F_k exp(s 2 pi i B . (s_k - P))."""
    return predict_direct(u, v, w, tree.leaf_l, tree.leaf_m, tree.leaf_flux, sign,
                          nm1=tree.leaf_nm1)


def synthesise(tree: Tree):
    """Inverse of steps 2-3 (from Eqs. 9, 10): every child of an existing node is
    lambda_{j+1,4k+c} = lambda_{j,k} + (1/sqrt(A_j)) sum_m s^m_c gamma^m_{j,k}.
    Returns the level-J coefficients over the full 4^(J-1)-fold refinement of
    the existing level-1 nodes as a dict {pixel id: lambda}."""
    cur = dict(zip(tree.levels[0].pix.tolist(), tree.levels[0].lam.tolist()))
    for j in range(1, tree.J):
        lv = tree.levels[j - 1]
        g = dict(zip(lv.pix.tolist(), lv.gamma.tolist()))
        inv = 1.0 / np.sqrt(sphere.pixel_area(j))
        nxt = {}
        for k, lam in cur.items():
            gam = g.get(k, [0.0, 0.0, 0.0])
            for cc in range(4):
                nxt[4 * k + cc] = lam + inv * sum(WAVELET_SIGNS[mm, cc] * gam[mm] for mm in range(3))
        cur = nxt
    return cur
