"""Oracle: hard thresholding of the wavelet coefficients (the retention of a
fixed proportion of coefficients that section 1 attributes to McEwen 2008; the
paper itself keeps every non-zero coefficient).  TEST INFRASTRUCTURE, like the
rest of oracle/.

The paper describes the variant in words only; the reading taken, step by
step:

1. Ranked are the wavelet coefficients gamma^m_{j,k} of the sky, m = 0, 1, 2,
   of every existing node at levels j = 1 .. J-1.  Eq. 10 gives them in the
   orthonormal normalisation (sqrt(A_j)/4), so magnitudes compare across
   levels.  The level-1 scaling coefficients are always kept.
2. A fixed proportion p is retained: the round(p N) coefficients of largest
   |gamma| (N = 3 x internal nodes; ties go to the lower level, then the lower
   node index in pixel order, then the lower m).  The others are set to zero.
3. A node none of whose own or descendants' coefficients is retained is a leaf
   of the thresholded tree at its own level: the plane wave is sampled at its
   pixel centre, as the tree samples it at the level-J leaves (section 3.5),
   and nothing below it is visited.
4. V_p = A_1 sum_k lambda_{1,k} eta_{1,k} + sum over retained (j, k, m) of
   gamma^m_{j,k} sigma^m_{j,k}, with eta and sigma from Eqs. 9 and 10 applied
   to the plane wave over the children that remain (Eq. 17 over the
   thresholded tree).

With p = 1 nothing is dropped and V_p is the exact tree route.
"""
from __future__ import annotations

import numpy as np

from . import sphere
from .tree import WAVELET_SIGNS, Tree
from .visibility import phasors


def coefficient_ranking(tree: Tree) -> np.ndarray:
    """Flat indices of all wavelet coefficients, largest |gamma| first (step 2's
    order).  Flat index of gamma^m_{j,k}: 3 (number of nodes at levels < j) +
    3 k + m, k the node's index in its level's pixel order."""
    mags = np.concatenate([np.abs(lv.gamma).ravel() for lv in tree.levels[:-1]]) \
        if tree.J > 1 else np.zeros(0)
    # stable sort on -|gamma| keeps the flat order (level, node, m) among ties
    return np.argsort(-mags, kind="stable")


def retained(tree: Tree, fraction: float) -> np.ndarray:
    """Flat indices of the retained coefficients for proportion `fraction`."""
    order = coefficient_ranking(tree)
    n_keep = int(np.floor(fraction * order.size + 0.5))
    return np.sort(order[:max(0, min(order.size, n_keep))])


def keep_masks(tree: Tree, flat) -> list:
    """Per level j < J, a (n_j, 3) boolean array of retained coefficients."""
    flat = np.asarray(flat, np.int64)
    out, off = [], 0
    for lv in tree.levels[:-1]:
        n = lv.pix.shape[0]
        k = np.zeros(3 * n, bool)
        sel = flat[(flat >= off) & (flat < off + 3 * n)] - off
        k[sel] = True
        out.append(k.reshape(n, 3))
        off += 3 * n
    return out


def alive_nodes(tree: Tree, keep) -> list:
    """Step 3: per level j < J, whether the node keeps a coefficient of its own
    or below (it stays an internal node of the thresholded tree)."""
    J = tree.J
    alive = [None] * (J - 1)
    for j in range(J - 1, 0, -1):
        lv = tree.levels[j - 1]
        a = keep[j - 1].any(axis=1)
        if j + 1 < J:
            below = alive[j]
            for cc in range(4):
                has = lv.child[:, cc] >= 0
                a[has] |= below[lv.child[has, cc]]
        alive[j - 1] = a
    return alive


def predict_thresholded(tree: Tree, flat, u, v, w, sign=-1, chunk=1024):
    """Steps 3-4 for the retained coefficients `flat` (flat indices)."""
    J = tree.J
    keep = keep_masks(tree, flat)
    alive = alive_nodes(tree, keep)
    u = np.asarray(u, np.float64)
    v = np.asarray(v, np.float64)
    w = np.asarray(w, np.float64)
    # pixel centres of every internal node (used where a node is a leaf)
    centres = [sphere.pixel_centres_lmn(j, tree.levels[j - 1].pix, tree.ra_p, tree.dec_p)
               for j in range(1, J)]
    out = np.empty(u.shape[0], np.complex128)
    for s in range(0, u.shape[0], chunk):
        sl = slice(s, s + chunk)
        ub, vb, wb = u[sl], v[sl], w[sl]
        # eta of level J: the leaves
        below = phasors(ub, vb, wb, tree.leaf_l, tree.leaf_m, tree.leaf_nm1, sign)
        V = np.zeros(ub.shape[0], np.complex128)
        for j in range(J - 1, 0, -1):
            lv = tree.levels[j - 1]
            a = np.sqrt(sphere.pixel_area(j)) / 4.0
            e = np.zeros((ub.shape[0], lv.pix.shape[0]), np.complex128)
            sg = np.zeros((ub.shape[0], lv.pix.shape[0], 3), np.complex128)
            for cc in range(4):
                has = lv.child[:, cc] >= 0
                vals = below[:, lv.child[has, cc]]
                e[:, has] += vals
                sg[:, has, :] += WAVELET_SIGNS[:, cc][None, None, :] * vals[:, :, None]
            eta = 0.25 * e
            sig = a * sg
            V = V + np.einsum("rkm,km->r", sig, np.where(keep[j - 1], lv.gamma, 0.0))
            # a node without a retained coefficient below it is a leaf at its
            # own level: the plane wave at its pixel centre
            dead = ~alive[j - 1]
            if dead.any():
                cl, cm, cn = (c[dead] for c in centres[j - 1])
                eta[:, dead] = phasors(ub, vb, wb, cl, cm, cn, sign)
            below = eta
        # below now holds eta at level 1 (the leaves themselves when J = 1)
        out[sl] = V + sphere.pixel_area(1) * (below @ tree.levels[0].lam)
    return out
