"""GPU parity of coefficient thresholding (the retained-proportion variant of
section 1; reading in oracle/threshold.py): the thresholded tree's route
against the oracle's literal evaluation, driven by the oracle's own choice of
retained coefficients; full retention gives the exact route bit for bit; both
traversals and the batched form agree."""
import numpy as np
import pytest

from oracle import sphere as sp
from oracle import threshold as oth
from oracle import tree as ot
from oracle import visibility as ov
from synth import configs

from .gpu_util import dev, errors, fp64_row_bound, host, note, require_gpu
from .test_gpu_tree import _with_walker

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    return require_gpu()


@pytest.fixture(scope="module")
def cfg2():
    W = configs.CFG2
    u, v, w = W.track.uvw()
    return W, u, v, w, configs.sample_rows(u.size, 1536, seed=77)


def _bound(rt, u, v, w, f, J):
    return fp64_row_bound(u, v, w, rt.leaf_l, rt.leaf_m, rt.leaf_nm1, rt.leaf_flux) + \
        (J + 2) * 4e-16 * np.abs(f).sum() * 4


@pytest.mark.parametrize("J,frac", [(10, 0.01), (10, 0.1), (10, 0.5), (9, 0.2), (8, 0.03)])
def test_thresholded_cfg2_vs_oracle(env, cfg2, J, frac):
    torch, swv = env
    W, u, v, w, rows = cfg2
    l, m, f = W.components()
    rt = ot.build_tree(J, W.ra_p, W.dec_p, l, m, f)
    keep = oth.retained(rt, frac)
    tp = swv.Tree(J, W.ra_p, W.dec_p, l, m, f).prune(keep)
    U, V, Wt = dev(u, torch), dev(v, torch), dev(w, torch)
    got = host(tp.predict(U, V, Wt))[rows]
    swv.synchronize()
    ref = oth.predict_thresholded(rt, keep, u[rows], v[rows], w[rows])
    bound = _bound(rt, u[rows], v[rows], w[rows], f, J)
    e_max, _ = errors(got, ref, f.sum())
    exact = ot.predict_snapped(rt, u[rows], v[rows], w[rows])
    st = tp.stats()
    note(f"cfg2 J={J} keep {frac:.0%} ({keep.size} of {3 * rt.n_internal}): "
         f"{st['n_leaves']} leaves, {st['n_internal']} internal; E_max vs oracle {e_max:.2e}, "
         f"vs exact V {errors(ref, exact, f.sum())[0]:.2e}")
    # the gate is the derived per-row bound (reading C-T1): thresholding leaves
    # fewer, heavier leaves, whose phase rounding cancels less than over the
    # exact tree's many light ones, so the summed-flux figure is reported only
    assert np.all(np.abs(got - ref) <= bound)


def test_full_retention_is_the_exact_route_bitwise(env, cfg2):
    torch, swv = env
    W, u, v, w, _ = cfg2
    l, m, f = W.components()
    U, V, Wt = (dev(a[:200000], torch) for a in (u, v, w))
    for J in (8, 10, 13):
        t = swv.Tree(J, W.ra_p, W.dec_p, l, m, f)
        a = t.predict(U, V, Wt)
        b = t.threshold(1.0).predict(U, V, Wt)
        swv.synchronize()
        assert torch.equal(a, b), J


@pytest.mark.parametrize("J,frac", [(10, 0.05), (14, 0.1), (20, 0.02)])
def test_thresholded_walkers_bitwise_and_f32c(env, J, frac):
    # the branch walker on the same thresholded tree, same bits; the FP32
    # leaf phasors within their bound
    torch, swv = env
    T = configs.SWEEP_TRACK
    u, v, w = (a[:60000] for a in T.uvw())
    l, m, f = configs.sweep_components(140)
    ra, dec = np.radians(T.ra_deg), np.radians(T.dec_deg)
    rt = ot.build_tree(J, ra, dec, l, m, f)
    keep = oth.retained(rt, frac)
    tp = swv.Tree(J, ra, dec, l, m, f).prune(keep)
    U, V, Wt = dev(u, torch), dev(v, torch), dev(w, torch)
    a = _with_walker(swv, 2, lambda: tp.predict(U, V, Wt))
    if J <= 16:
        b = _with_walker(swv, 4, lambda: tp.predict(U, V, Wt))
        swv.synchronize()
        assert torch.equal(a, b)
    rows = configs.sample_rows(u.size, 512, seed=J)
    ref = oth.predict_thresholded(rt, keep, u[rows], v[rows], w[rows])
    got = host(a)[rows]
    assert np.all(np.abs(got - ref) <= _bound(rt, u[rows], v[rows], w[rows], f, J))
    g32 = host(tp.predict(U, V, Wt, prec="f32c"))[rows].astype(np.complex128)
    assert errors(g32, ref, f.sum())[0] <= 1e-6


def test_two_leaf_tree_on_the_gpu(env):
    # the hand-derived case of the oracle's pins, through the library:
    # keeping only gamma^2 of a node with fluxes F0, F3 in children 0, 3 gives
    # V = (F0 + F3)(e0 + e3) / 2; keeping nothing, (F0 + F3) e_parent
    torch, swv = env
    J, ra, dec = 2, 1.1, 0.4
    pix, flux = np.array([20, 23]), np.array([0.3, 0.5])
    t = swv.Tree.from_pixels(J, ra, dec, pix, flux)
    rng = np.random.default_rng(4)
    u, v, w = (rng.uniform(-300, 300, 256) for _ in range(3))
    U, V, Wt = dev(u, torch), dev(v, torch), dev(w, torch)
    cl, cm, cn = sp.pixel_centres_lmn(J, pix, ra, dec)
    e = ov.phasors(u, v, w, cl, cm, cn)
    pl, pm, pn = sp.pixel_centres_lmn(1, np.array([5]), ra, dec)
    ep = ov.phasors(u, v, w, pl, pm, pn)[:, 0]
    # phase rounding of the GPU's phasors: the per-row bound at both the leaf
    # and the parent centre
    bound = fp64_row_bound(u, v, w, np.r_[cl, pl], np.r_[cm, pm], np.r_[cn, pn],
                           np.r_[flux, flux.sum()])
    for kept, ref in (([2], flux.sum() * (e[:, 0] + e[:, 1]) / 2), ([], flux.sum() * ep),
                      ([0, 1, 2], flux[0] * e[:, 0] + flux[1] * e[:, 1])):
        got = host(t.prune(kept).predict(U, V, Wt))
        assert np.all(np.abs(got - ref) <= bound), kept


def test_thresholded_tree_in_a_batched_plan(env):
    torch, swv = env
    rng = np.random.default_rng(12)
    insts, refs = [], []
    for J, frac, n in ((9, 0.05, 30011), (10, 0.3, 4097), (7, 0.0, 65)):
        l, m, f = rng.uniform(-0.03, 0.03, 200), rng.uniform(-0.03, 0.03, 200), \
            rng.lognormal(-3, 1, 200)
        tp = swv.Tree(J, 0.7, 0.3, l, m, f).threshold(frac)
        u, v, w = (dev(rng.uniform(-3e4, 3e4, n), torch) for _ in range(3))
        out = torch.full((n,), 7.0, dtype=torch.complex128, device="cuda")
        insts.append(dict(route="tree", tree=tp, u=u, v=v, w=w, out=out))
        refs.append(tp.predict(u, v, w))
    plan = swv.BatchPlan(insts)
    plan.run()
    swv.synchronize()
    assert all(torch.equal(d["out"], r) for d, r in zip(insts, refs))
    plan.close()
