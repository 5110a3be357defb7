"""Pins of the thresholding oracle (coefficient retention, read from section 1;
oracle/threshold.py states the reading): the exact tree at p = 1, plain
direct sums when whole levels are kept or dropped, and a hand-derived two-leaf
tree."""
import math

import numpy as np
import pytest

from oracle import sphere as sp
from oracle import threshold as oth
from oracle import tree as ot
from oracle import visibility as ov
from synth import configs


def _tracks(n, seed, scale=2e4):
    rng = np.random.default_rng(seed)
    return tuple(rng.uniform(-scale, scale, n) for _ in range(3))


def _model(n, seed, spread=0.03):
    rng = np.random.default_rng(seed)
    return rng.uniform(-spread, spread, n), rng.uniform(-spread, spread, n), \
        rng.lognormal(-3, 1, n)


RA, DEC = 1.1, 0.4


@pytest.mark.parametrize("J", [1, 3, 7, 10])
def test_full_retention_is_the_exact_tree(J):
    l, m, f = _model(150, J)
    t = ot.build_tree(J, RA, DEC, l, m, f)
    u, v, w = _tracks(300, J)
    keep = oth.retained(t, 1.0)
    assert keep.size == 3 * t.n_internal
    got = oth.predict_thresholded(t, keep, u, v, w)
    ref = ot.predict_snapped(t, u, v, w)
    assert np.max(np.abs(got - ref)) <= (J + 2) * 4e-16 * f.sum() * 8


def test_no_retention_is_the_level1_sum():
    # everything collapses into the level-1 nodes: their total flux at their
    # pixel centres (a plain direct sum)
    J = 8
    l, m, f = _model(200, 4, spread=0.4)
    t = ot.build_tree(J, RA, DEC, l, m, f)
    u, v, w = _tracks(200, 5)
    got = oth.predict_thresholded(t, oth.retained(t, 0.0), u, v, w)
    base = t.leaf_pix >> (2 * (J - 1))
    pix, inv = np.unique(base, return_inverse=True)
    F = np.bincount(inv, weights=t.leaf_flux)
    cl, cm, cn = sp.pixel_centres_lmn(1, pix, RA, DEC)
    ref = ov.predict_direct(u, v, w, cl, cm, F, nm1=cn)
    assert len(pix) >= 2
    assert np.max(np.abs(got - ref)) <= 1e-13 * f.sum()


@pytest.mark.parametrize("L", [1, 4, 8])
def test_levels_kept_whole_give_the_direct_sum_one_level_down(L):
    # every coefficient of levels <= L kept, none below: every node of level
    # L + 1 collapses, and V is the direct sum over those nodes at their pixel
    # centres with the flux of the leaves below them (Eq. 16 at level L + 1)
    J = 11
    l, m, f = _model(300, 7 + L)
    t = ot.build_tree(J, RA, DEC, l, m, f)
    u, v, w = _tracks(250, 8)
    n_upto = sum(t.levels[j - 1].pix.size for j in range(1, L + 1))
    got = oth.predict_thresholded(t, np.arange(3 * n_upto), u, v, w)
    node = t.leaf_pix >> (2 * (J - L - 1))
    pix, inv = np.unique(node, return_inverse=True)
    F = np.bincount(inv, weights=t.leaf_flux)
    cl, cm, cn = sp.pixel_centres_lmn(L + 1, pix, RA, DEC)
    ref = ov.predict_direct(u, v, w, cl, cm, F, nm1=cn)
    assert np.max(np.abs(got - ref)) <= 1e-13 * f.sum()


def _two_leaf_tree():
    """J = 2: flux F0 in child 0 and F3 in child 3 of base pixel 5."""
    J, F0, F3 = 2, 0.3, 0.5
    pix = np.array([4 * 5 + 0, 4 * 5 + 3])
    flux = np.array([F0, F3])
    ll, mm, nn = sp.pixel_centres_lmn(J, pix, RA, DEC)
    t = ot.Tree(J, RA, DEC, pix, flux, ll, mm, nn, ot.build_levels(J, pix, flux))
    return t, F0, F3


def test_two_leaf_tree_by_hand():
    # One node (level 1) with children c = 0, 3 of densities lambda_0, lambda_3
    # = F / A_2, lambda_1 = (lambda_0 + lambda_3) / 4, A_1 = 4 A_2, and
    # gamma^m = (sqrt(A_1) / 4) (s^m_0 lambda_0 + s^m_3 lambda_3): the Eq. 10
    # signs of children 0, 3 are (+, -) for m = 0, 1 and (+, +) for m = 2.
    # With e_c the plane wave at child c, eta_1 = (e_0 + e_3) / 4 and
    # sigma^m = (sqrt(A_1) / 4) (s^m_0 e_0 + s^m_3 e_3), so
    #   keep all:      V = F0 e0 + F3 e3 (the exact tree);
    #   keep gamma^2:  V = (F0 + F3)(e0 + e3) / 2;
    #   keep gamma^0:  V = [(F0 + F3)(e0 + e3) + (F0 - F3)(e0 - e3)] / 4
    #                    = (F0 e0 + F3 e3) / 2;
    #   keep nothing:  the node collapses: V = (F0 + F3) e_parent.
    t, F0, F3 = _two_leaf_tree()
    u, v, w = _tracks(64, 11, scale=300.0)
    e = ov.phasors(u, v, w, t.leaf_l, t.leaf_m, t.leaf_nm1)
    e0, e3 = e[:, 0], e[:, 1]
    pl, pm, pn = sp.pixel_centres_lmn(1, np.array([5]), RA, DEC)
    ep = ov.phasors(u, v, w, pl, pm, pn)[:, 0]
    cases = {
        (0, 1, 2): F0 * e0 + F3 * e3,
        (2,): (F0 + F3) * (e0 + e3) / 2,
        (0,): ((F0 + F3) * (e0 + e3) + (F0 - F3) * (e0 - e3)) / 4,
        (): (F0 + F3) * ep,
    }
    for kept, ref in cases.items():
        got = oth.predict_thresholded(t, np.array(kept, np.int64), u, v, w)
        assert np.max(np.abs(got - ref)) <= 1e-15, kept


def test_ranking_order_and_count():
    l, m, f = _model(400, 13)
    t = ot.build_tree(10, RA, DEC, l, m, f)
    mags = np.concatenate([np.abs(lv.gamma).ravel() for lv in t.levels[:-1]])
    for p in (0.0, 0.013, 0.1, 0.5, 0.999, 1.0):
        keep = oth.retained(t, p)
        assert keep.size == int(math.floor(p * mags.size + 0.5))
        dropped = np.setdiff1d(np.arange(mags.size), keep)
        if keep.size and dropped.size:
            assert mags[keep].min() >= mags[dropped].max()
    # ties go to the lower flat index (level, node, m): the two-leaf tree has
    # |gamma^0| = |gamma^1| < |gamma^2|
    t2, _, _ = _two_leaf_tree()
    g = np.abs(t2.levels[0].gamma[0])
    assert g[0] == g[1] < g[2]
    assert list(oth.retained(t2, 2 / 3)) == [0, 2]


def test_error_falls_to_zero_as_retention_grows():
    # not a proof, but the variant must approach the exact route: on cfg2's
    # clustered model the error at 50 % retention is below the error at 1 %
    W = configs.CFG2
    l, m, f = W.components()
    t = ot.build_tree(9, W.ra_p, W.dec_p, l, m, f)
    u, v, w = (a[:2000] for a in W.track.uvw())
    exact = ot.predict_snapped(t, u, v, w)
    errs = [np.max(np.abs(oth.predict_thresholded(t, oth.retained(t, p), u, v, w) - exact))
            for p in (0.01, 0.5, 1.0)]
    assert errs[0] > errs[1] > errs[2] and errs[2] <= 1e-12 * f.sum()
