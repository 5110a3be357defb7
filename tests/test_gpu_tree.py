"""GPU parity of the wavelet-tree route (Eqs. 14-17) against the oracle.

The oracle builds its own tree (its own pixelisation and centres) and
evaluates Eq. 17 step by step; the GPU path builds the tree in the library's
host code and walks it on the device.  Tolerance: E_max <= 1e-12 relative to
sum |F| (see test_gpu_direct).  A further property test compares the tree
route with the direct route of the library on the tree's own leaves (Eq. 16
= Eq. 17) at the full measured size."""
import numpy as np
import pytest

from oracle import tree as ot
from synth import configs

from .gpu_util import dev, errors, fp64_row_bound, host, note, require_gpu

pytestmark = pytest.mark.gpu
TOL64 = 1e-12


@pytest.fixture(scope="module")
def env():
    return require_gpu()


def _tree_run(env, J, ra, dec, l, m, f, u, v, w, sign=-1):
    torch, swv = env
    t = swv.Tree(J, ra, dec, l, m, f)
    out = t.predict(dev(u, torch), dev(v, torch), dev(w, torch), sign=sign)
    swv.synchronize()
    return t, host(out)


@pytest.mark.parametrize("sign", [-1, 1])
def test_cfg1_tree_full(env, sign):
    W = configs.CFG1
    u, v, w = W.track.uvw()
    l, m, f = W.components()
    J = W.J[0]
    t, got = _tree_run(env, J, W.ra_p, W.dec_p, l, m, f, u, v, w, sign)
    ref_t = ot.build_tree(J, W.ra_p, W.dec_p, l, m, f)
    rows = np.arange(u.size)
    ref = ot.predict_tree(ref_t, u[rows], v[rows], w[rows], sign)
    e_max, e_rms = errors(got, ref, f.sum())
    note(f"cfg1 tree J={J} ({t.stats()['n_leaves']} leaves): E_max={e_max:.3e} E_rms={e_rms:.3e}")
    assert e_max <= TOL64
    snapped = ot.predict_snapped(ref_t, u, v, w, sign)
    assert errors(got, snapped, f.sum())[0] <= TOL64


@pytest.mark.parametrize("J", [8, 9, 10])
def test_cfg2_tree_sampled(env, J):
    torch, swv = env
    W = configs.CFG2
    u, v, w = W.track.uvw()
    l, m, f = W.components()
    t = swv.Tree(J, W.ra_p, W.dec_p, l, m, f)
    out = t.predict(dev(u, torch), dev(v, torch), dev(w, torch))
    swv.synchronize()
    rows = configs.sample_rows(u.size, 2048, seed=J)
    got = host(out[torch.as_tensor(rows, device="cuda")])
    ref_t = ot.build_tree(J, W.ra_p, W.dec_p, l, m, f)
    ref = ot.predict_tree(ref_t, u[rows], v[rows], w[rows])
    e_max, e_rms = errors(got, ref, f.sum())
    st = t.stats()
    note(f"cfg2 tree J={J}: leaves={st['n_leaves']} internal={st['n_internal']} "
         f"sparsity={st['sparsity']:.3e} E_max={e_max:.3e} E_rms={e_rms:.3e}")
    assert e_max <= TOL64


@pytest.mark.parametrize("J", [8, 10])
def test_tree_equals_direct_on_its_leaves_full_size(env, J):
    # Eq. 17 == Eq. 16 at every one of the 8.36M rows (library only)
    torch, swv = env
    W = configs.CFG2
    u, v, w = (dev(a, torch) for a in W.track.uvw())
    l, m, f = W.components()
    t = swv.Tree(J, W.ra_p, W.dec_p, l, m, f)
    lv = t.leaves()
    # the direct kernel takes (l, m) and forms n - 1 itself; leaves lie on the
    # near hemisphere, so the same centre is described
    vt = t.predict(u, v, w)
    vd = swv.predict_direct(u, v, w, dev(lv["l"], torch), dev(lv["m"], torch),
                            dev(lv["flux"], torch))
    swv.synchronize()
    d = (vt - vd).abs().max().item() / float(np.abs(f).sum())
    note(f"cfg2 J={J}: max |V_tree - V_direct(leaves)| / sum|F| over {u.numel()} rows = {d:.3e}")
    assert d <= TOL64


@pytest.mark.parametrize("J", list(range(1, 13)))
def test_small_trees_every_depth(env, J):
    rng = np.random.default_rng(100 + J)
    n = 37
    half = 0.5 if J < 5 else 0.05
    l, m = rng.uniform(-half, half, n), rng.uniform(-half, half, n)
    f = rng.lognormal(-3, 1, n)
    nv = 333
    scale = 200.0 if J < 5 else 2e4
    u, v, w = (rng.uniform(-scale, scale, nv) for _ in range(3))
    ra, dec = 1.0, 0.3
    _, got = _tree_run(env, J, ra, dec, l, m, f, u, v, w)
    rt = ot.build_tree(J, ra, dec, l, m, f)
    ref = ot.predict_tree(rt, u, v, w)
    # few leaves: per-row bound of the FP64 leaf phases, plus J levels of sums
    bound = fp64_row_bound(u, v, w, rt.leaf_l, rt.leaf_m, rt.leaf_nm1, rt.leaf_flux)
    assert np.all(np.abs(got - ref) <= bound + (J + 2) * 4e-16 * np.abs(f).sum())


def _spine_pixels(J, base, counts, rng):
    """Level-J pixel ids of a tree whose spine node at level j has counts[j-1]
    children (a random subset of the four), one of which continues the spine;
    the others end in one-child chains down to level J."""
    pix, node = [], base                     # level-1 pixel: the base pixel
    for j in range(1, J):
        cs = rng.choice(4, counts[j - 1], replace=False)
        for c in cs[1:]:
            p = 4 * node + int(c)
            for _ in range(J - j - 1):
                p = 4 * p + int(rng.integers(4))
            pix.append(p)
        node = 4 * node + int(cs[0])
    pix.append(node)
    return pix


@pytest.mark.parametrize("J,walker", [(10, 1), (10, 2), (12, 2), (15, 2), (12, 4), (15, 4)])
def test_every_child_count_on_the_lds_levels(env, J, walker):
    """The top levels (segments) of a deep traversal keep their finished
    children in LDS and form the sums when the last child returns; spines
    whose nodes have 1, 2, 3 and 4 children at every depth cover every count
    of kept children, with both walkers, against the oracle."""
    torch, swv = env
    rng = np.random.default_rng(7 * J + walker)
    pix = []
    for base, shift in ((4, 0), (5, 1), (6, 2), (7, 3)):
        counts = [1 + (j + shift) % 4 for j in range(J - 1)]
        pix += _spine_pixels(J, base, counts, rng)
    flux = rng.normal(size=len(pix))
    ra, dec = 1.0, 0.3
    t = swv.Tree.from_pixels(J, ra, dec, pix, flux)
    st = t.stats()
    nv = 333
    u, v, w = (rng.uniform(-2e4, 2e4, nv) for _ in range(3))
    got = host(_with_walker(swv, walker, lambda: t.predict(dev(u, torch), dev(v, torch),
                                                           dev(w, torch))))
    swv.synchronize()
    from oracle import clean as oc
    rt = oc.tree_from_pixels(J, ra, dec, pix, flux)
    ref = ot.predict_tree(rt, u, v, w)
    kids = {}
    for j in range(1, 5):                    # children per node on the top four levels
        parents = t.level(j + 1)["pix"] // 4
        kids[j] = sorted(set(np.unique(parents, return_counts=True)[1].tolist()))
    note(f"J={J} walker={walker}: {st['n_leaves']} leaves, max_branching="
         f"{st['max_branching']}, children per node on levels 1-4: {kids}")
    assert all(kids[j] == [1, 2, 3, 4] for j in (1, 2, 3, 4))
    bound = fp64_row_bound(u, v, w, rt.leaf_l, rt.leaf_m, rt.leaf_nm1, rt.leaf_flux)
    assert np.all(np.abs(got - ref) <= bound + (J + 2) * 4e-16 * np.abs(flux).sum())


def test_empty_tree_gives_zero(env):
    _, got = _tree_run(env, 7, 0.0, 0.5, np.zeros(0), np.zeros(0), np.zeros(0),
                       np.ones(100), np.ones(100), np.ones(100))
    assert np.all(got == 0)


def _nested_components(j0, J=29, ra=0.3, dec=0.4, l0=0.01, m0=0.003):
    """One component plus, for every level j0..J, one at the centre of a sibling
    of its level-j pixel: every ancestor from level j0-1 down branches."""
    from paper_1909_03956_amd.api import ang2pix, pixel_centres
    k = int(ang2pix(J, ra, dec, np.array([l0]), np.array([m0]))[0])
    ls, ms = [l0], [m0]
    for j in range(j0, J + 1):
        cl, cm, _ = pixel_centres(j, ra, dec, np.array([(k >> 2 * (J - j)) ^ 1], np.int64))
        ls.append(cl[0])
        ms.append(cm[0])
    return np.array(ls), np.array(ms)


def _oracle_tree_on_library_pixels(J, ra, dec, l, m, f):
    """The oracle's tree of components that sit on pixel edges (the centre of
    a level-j pixel is a corner of its descendants), built on the library's
    choice of pixel for each: where the two pixelisations part, the point must
    lie within 1e-12 rad of an edge, i.e. a nudge of 1e-12 rad towards the
    library's pixel centre puts it there for the oracle too (reading C-T7)."""
    from oracle import clean as oc
    from oracle import sphere as sp
    from paper_1909_03956_amd.api import ang2pix
    lib = ang2pix(J, ra, dec, l, m)
    ora = sp.ang2pix_xyz(J, sp.lm_to_xyz(l, m, ra, dec))
    bad = np.nonzero(lib != ora)[0]
    if bad.size:
        P = sp.lm_to_xyz(l[bad], m[bad], ra, dec)
        d = sp.pix2xyz(J, lib[bad]) - P
        Q = P + sp.LD(1e-12) * d / np.sqrt((d * d).sum(0))
        Q = Q / np.sqrt((Q * Q).sum(0))
        assert np.array_equal(sp.ang2pix_xyz(J, Q), lib[bad]), "not an edge tie"
    note(f"components on edges: {bad.size} of {l.size} assigned across an edge")
    return oc.tree_from_pixels(J, ra, dec, lib, f)


def _with_walker(swv, walker, fn):
    """Runs fn() with the tree traversal chosen by `walker` (1 by depth and
    shape, 2 branch walker, 4 level walker wherever it is compiled)."""
    from paper_1909_03956_amd._lib import FAM_TREE
    ctx = swv.context()
    saved = [ctx.tune_get(FAM_TREE, c) for c in (0, 1)]
    try:
        for c in (0, 1):
            ctx.tune_set(FAM_TREE, c, walker, saved[c][1])
        return fn()
    finally:
        for c in (0, 1):
            ctx.tune_set(FAM_TREE, c, *saved[c])


@pytest.mark.parametrize("name,J", [("cfg1", 6), ("cfg2", 8), ("cfg2", 9), ("cfg2", 10),
                                    ("cfg1", 12), ("cfg1", 16)])
def test_walkers_bitwise_equal(env, name, J):
    # both traversals perform the same operations in the same order
    torch, swv = env
    W = configs.WORKLOADS[name]
    u, v, w = (dev(a, torch) for a in W.track.uvw())
    l, m, f = W.components()
    t = swv.Tree(J, W.ra_p, W.dec_p, l, m, f)
    a = _with_walker(swv, 4, lambda: t.predict(u, v, w))
    b = _with_walker(swv, 2, lambda: t.predict(u, v, w))
    c = _with_walker(swv, 1, lambda: t.predict(u, v, w))
    swv.synchronize()
    st = t.stats()
    note(f"{name} J={J}: max_branching={st['max_branching']} rows={u.numel()}")
    assert torch.equal(a, b) and torch.equal(a, c)


@pytest.mark.parametrize("J", list(range(1, 17)))
def test_walkers_bitwise_equal_small_trees(env, J):
    torch, swv = env
    rng = np.random.default_rng(200 + J)
    n = 61
    half = 0.5 if J < 5 else 0.05
    l, m = rng.uniform(-half, half, n), rng.uniform(-half, half, n)
    f = rng.lognormal(-3, 1, n)
    u, v, w = (dev(rng.uniform(-2e4, 2e4, 1000), torch) for _ in range(3))
    t = swv.Tree(J, 1.0, 0.3, l, m, f)
    a = _with_walker(swv, 4, lambda: t.predict(u, v, w))
    b = _with_walker(swv, 2, lambda: t.predict(u, v, w))
    swv.synchronize()
    assert torch.equal(a, b)


def _deep_case(env, J, l, m, f, nv, seed, scale, on_edges=False):
    torch, swv = env
    ra, dec = 0.3, 0.4
    rng = np.random.default_rng(seed)
    u, v, w = (rng.uniform(-scale, scale, nv) for _ in range(3))
    t = swv.Tree(J, ra, dec, l, m, f)
    got = host(t.predict(dev(u, torch), dev(v, torch), dev(w, torch)))
    swv.synchronize()
    rt = (_oracle_tree_on_library_pixels(J, ra, dec, l, m, f) if on_edges
          else ot.build_tree(J, ra, dec, l, m, f))
    assert t.stats()["n_leaves"] == rt.n_leaves
    ref = ot.predict_tree(rt, u, v, w)
    snapped = ot.predict_snapped(rt, u, v, w)
    bound = fp64_row_bound(u, v, w, rt.leaf_l, rt.leaf_m, rt.leaf_nm1, rt.leaf_flux)
    slack = (J + 2) * 4e-16 * np.abs(f).sum()
    note(f"deep J={J}: leaves={rt.n_leaves} internal={rt.n_internal} "
         f"max_branching={t.stats()['max_branching']} "
         f"max|d|/bound={np.max(np.abs(got - ref) / (bound + slack)):.3f}")
    assert np.all(np.abs(got - ref) <= bound + slack)
    assert np.all(np.abs(got - snapped) <= bound + slack)


@pytest.mark.parametrize("J,n", [(13, 140), (16, 40), (20, 140), (25, 10), (25, 140), (29, 140)])
def test_deep_trees_vs_oracle(env, J, n):
    # the run-time sweep's regime: tens to ~140 leaves, J = 12 .. 29
    rng = np.random.default_rng(J * 1000 + n)
    l, m = rng.uniform(-0.02, 0.02, n), rng.uniform(-0.02, 0.02, n)
    f = rng.lognormal(-3, 1, n)
    _deep_case(env, J, l, m, f, 500, J, 4.6e5)


def test_deepest_supported_branching(env):
    # 15 nested branchings: the largest the branch walker is compiled for
    l, m = _nested_components(15)
    f = np.random.default_rng(5).lognormal(-3, 1, l.size)
    torch, swv = env
    assert swv.Tree(29, 0.3, 0.4, l, m, f).stats()["max_branching"] == 15
    _deep_case(env, 29, l, m, f, 300, 7, 4.6e5, on_edges=True)


def test_too_many_branchings_not_supported(env):
    torch, swv = env
    from paper_1909_03956_amd._lib import SWV_ENOTSUP, SwvError
    l, m = _nested_components(14)
    t = swv.Tree(29, 0.3, 0.4, l, m, np.ones(l.size))
    assert t.stats()["max_branching"] == 16
    x = dev(np.ones(4), torch)
    with pytest.raises(SwvError) as e:
        t.predict(x, x, x)
    assert e.value.code == SWV_ENOTSUP


def test_tree_bitwise_reproducible(env):
    W = configs.CFG1
    u, v, w = W.track.uvw()
    l, m, f = W.components()
    _, a = _tree_run(env, 6, W.ra_p, W.dec_p, l, m, f, u, v, w)
    _, b = _tree_run(env, 6, W.ra_p, W.dec_p, l, m, f, u, v, w)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("J,n", [(20, 140), (25, 15)])
def test_sweep_workload_vs_oracle(env, J, n):
    # the run-time sweep's own inputs: a one-hour, one-second 27-antenna track
    torch, swv = env
    T = configs.SWEEP_TRACK
    u, v, w = T.uvw()
    l, m, f = configs.sweep_components(n)
    ra, dec = np.radians(T.ra_deg), np.radians(T.dec_deg)
    t = swv.Tree(J, ra, dec, l, m, f)
    out = t.predict(dev(u, torch), dev(v, torch), dev(w, torch))
    swv.synchronize()
    rows = configs.sample_rows(u.size, 1024, seed=J)
    got = host(out[torch.as_tensor(rows, device="cuda")])
    rt = ot.build_tree(J, ra, dec, l, m, f)
    ref = ot.predict_tree(rt, u[rows], v[rows], w[rows])
    e_max, e_rms = errors(got, ref, f.sum())
    note(f"sweep J={J} N~_C={rt.n_leaves}: E_max={e_max:.3e} E_rms={e_rms:.3e}")
    assert e_max <= TOL64


# Precision form of the tree route: FP64 phase reduced exactly, FP32 hardware
# sine/cosine at the leaves, FP64 node arithmetic.  Per leaf the phasor is off
# by at most 2 pi 2^-25 (the FP32 rounding of the reduced phase) plus the
# hardware sincos error (<= 2.5e-7, test_gpu_direct): < 4.4e-7, so
# |V - V_exact| < 4.4e-7 sum |F|; gate E_max <= 1e-6 as for the direct form.
TOL32 = 1e-6


@pytest.mark.parametrize("J", [8, 9, 10])
def test_tree_f32c_cfg2_sampled(env, J):
    torch, swv = env
    W = configs.CFG2
    u, v, w = W.track.uvw()
    l, m, f = W.components()
    t = swv.Tree(J, W.ra_p, W.dec_p, l, m, f)
    out = t.predict(dev(u, torch), dev(v, torch), dev(w, torch), prec="f32c")
    swv.synchronize()
    assert out.dtype == torch.complex64
    rows = configs.sample_rows(u.size, 2048, seed=J + 40)
    got = host(out[torch.as_tensor(rows, device="cuda")]).astype(np.complex128)
    ref = ot.predict_tree(ot.build_tree(J, W.ra_p, W.dec_p, l, m, f), u[rows], v[rows], w[rows])
    e_max, e_rms = errors(got, ref, f.sum())
    note(f"cfg2 tree f32c J={J}: E_max={e_max:.3e} E_rms={e_rms:.3e}")
    assert e_max <= TOL32


def test_tree_f32c_deep_and_walkers(env):
    torch, swv = env
    T = configs.SWEEP_TRACK
    u, v, w = T.uvw()
    rows = configs.sample_rows(u.size, 1024, seed=3)
    l, m, f = configs.sweep_components(140)
    ra, dec = np.radians(T.ra_deg), np.radians(T.dec_deg)
    U, V, W = (dev(a[rows], torch) for a in (u, v, w))
    for J in (10, 20):
        t = swv.Tree(J, ra, dec, l, m, f)
        a = _with_walker(swv, 1, lambda: t.predict(U, V, W, prec="f32c"))
        b = _with_walker(swv, 2, lambda: t.predict(U, V, W, prec="f32c"))
        swv.synchronize()
        assert torch.equal(a, b)
        ref = ot.predict_tree(ot.build_tree(J, ra, dec, l, m, f), u[rows], v[rows], w[rows])
        e_max, _ = errors(host(a).astype(np.complex128), ref, f.sum())
        note(f"sweep tree f32c J={J}: E_max={e_max:.3e}")
        assert e_max <= TOL32


def test_tree_f32c_out_dtype_checked(env):
    torch, swv = env
    t = swv.Tree(6, 0.0, 0.5, [0.01], [0.0], [1.0])
    x = dev(np.ones(4), torch)
    with pytest.raises(ValueError):
        t.predict(x, x, x, prec="f32c", out=torch.empty(4, dtype=torch.complex128, device="cuda"))


# ------------------------------------------------ Eq. 16 form (leaf sum) --
@pytest.mark.parametrize("J", [8, 10])
def test_leaf_sum_equals_tree_and_oracle(env, J):
    """swv_predict_tree_leaves (Eq. 16) against the traversal at every cfg2
    row and against the oracle's snapped direct sum on sampled rows."""
    torch, swv = env
    W = configs.CFG2
    u, v, w = W.track.uvw()
    U, V, Wt = dev(u, torch), dev(v, torch), dev(w, torch)
    l, m, f = W.components()
    t = swv.Tree(J, W.ra_p, W.dec_p, l, m, f)
    vt = t.predict(U, V, Wt)
    vl = t.predict_leaves(U, V, Wt)
    swv.synchronize()
    d = (vt - vl).abs().max().item() / float(np.abs(f).sum())
    rows = configs.sample_rows(u.size, 2048, seed=J + 50)
    ref_t = ot.build_tree(J, W.ra_p, W.dec_p, l, m, f)
    ref = ot.predict_snapped(ref_t, u[rows], v[rows], w[rows])
    e_max, _ = errors(host(vl[torch.as_tensor(rows, device="cuda")]), ref, f.sum())
    note(f"cfg2 J={J} leaf sum: vs traversal {d:.3e}, vs oracle {e_max:.3e}")
    assert d <= TOL64 and e_max <= TOL64
    v32 = host(t.predict_leaves(U, V, Wt, prec="f32c"))
    assert v32.dtype == np.complex64
    assert errors(v32[rows], ref, f.sum())[0] <= 1e-6


def test_leaf_sum_follows_set_flux_and_needs_no_walker(env):
    torch, swv = env
    # a tree the traversals do not support (16 nested branchings) still sums
    l, m = _nested_components(14)
    rng = np.random.default_rng(8)
    f = rng.lognormal(-3, 1, l.size)
    t = swv.Tree(29, 0.3, 0.4, l, m, f)
    assert t.stats()["max_branching"] == 16
    u, v, w = (rng.uniform(-4.6e5, 4.6e5, 700) for _ in range(3))
    U, V, Wt = dev(u, torch), dev(v, torch), dev(w, torch)
    got = host(t.predict_leaves(U, V, Wt))
    rt = _oracle_tree_on_library_pixels(29, 0.3, 0.4, l, m, f)
    bound = fp64_row_bound(u, v, w, rt.leaf_l, rt.leaf_m, rt.leaf_nm1, rt.leaf_flux)
    assert np.all(np.abs(got - ot.predict_snapped(rt, u, v, w)) <= bound)
    # new leaf fluxes reach the device copy of the leaves
    f2 = rng.lognormal(-3, 1, t.stats()["n_leaves"])
    t.set_leaf_flux(f2)
    rt.leaf_flux = f2
    got2 = host(t.predict_leaves(U, V, Wt))
    bound2 = fp64_row_bound(u, v, w, rt.leaf_l, rt.leaf_m, rt.leaf_nm1, f2)
    assert np.all(np.abs(got2 - ot.predict_snapped(rt, u, v, w)) <= bound2)
