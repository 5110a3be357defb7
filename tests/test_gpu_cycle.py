"""GPU tests of the captured major cycle (section 2.2: predict, subtract,
image; the chi^2 gradients beside them): a graph replay equals the eager
cycle bit for bit, a new model each cycle (new component lists, new trees of
another depth) replays without a new capture, and every output agrees with
the oracle."""
import numpy as np
import pytest

from oracle import tree as ot
from oracle import visibility as ov
from synth import models

from .gpu_util import dev, dev_c, errors, fp64_row_bound, host, note, require_gpu
from .test_gpu_image import _grad_scales

pytestmark = pytest.mark.gpu
TOL64 = 1e-12
RA, DEC = 1.1, 0.4


@pytest.fixture(scope="module")
def env():
    return require_gpu()


SPECS = [  # route, rows, comp_cap, tree_level_cap, pixels, grads
    ("direct", 50_000, 300, 1, 40, True),
    ("direct", 7_001, 64, 1, 0, True),
    ("tree", 30_011, 300, 9, 25, False),
    ("tree", 65, 50, 10, 0, False),
]


def _make(torch, swv, rng):
    inst, host_in = [], []
    for route, n, cap, jcap, npix, grads in SPECS:
        u, v, w = (rng.uniform(-3e4, 3e4, n) for _ in range(3))
        obs = models.random_complex(n, rng)
        d = dict(route=route, u=dev(u, torch), v=dev(v, torch), w=dev(w, torch),
                 vis_obs=dev_c(obs, torch), inv_sigma2=1e4, comp_cap=cap, tree_level_cap=jcap,
                 grads=grads)
        pix = None
        if npix:
            pix = tuple(rng.uniform(-0.04, 0.04, npix) for _ in range(2))
            pix = pix + (ov.n_minus_1(*pix),)
            d["pixels"] = tuple(dev(a, torch) for a in pix)
        inst.append(d)
        host_in.append((u, v, w, obs, pix))
    return inst, host_in


def _model(rng, counts, levels):
    """Per instance: (l, m, flux) for a direct one, a tree for a tree one."""
    out = []
    for (route, *_), k, J in zip(SPECS, counts, levels):
        l, m = rng.uniform(-0.03, 0.03, k), rng.uniform(-0.03, 0.03, k)
        f = rng.lognormal(-3, 1, k)
        out.append((route, J, l, m, f))
    return out


def _set(torch, swv, cy, model):
    keep = []
    for k, (route, J, l, m, f) in enumerate(model):
        if route == "direct":
            cy.set_components(k, dev(l, torch), dev(m, torch), dev(f, torch))
        else:
            t = swv.Tree(J, RA, DEC, l, m, f)
            cy.set_tree(k, t)
            keep.append(t)
    for t in keep:
        t.close()           # the cycle copied the records


def _snapshot(cy):
    snap = []
    for o in cy.out:
        s = {k: v.clone() for k, v in o.items() if k != "grads"}
        if "grads" in o:
            s["grads"] = [g.clone() for g in o["grads"]]
        snap.append(s)
    return snap


def _equal(torch, a, b):
    bad = []
    for k, (x, y) in enumerate(zip(a, b)):
        for key in x:
            xs = x[key] if key == "grads" else [x[key]]
            ys = y[key] if key == "grads" else [y[key]]
            if not all(torch.equal(p, q) for p, q in zip(xs, ys)):
                bad.append((k, key))
    return bad


def _oracle_checks(cy, host_in, model):
    for k, ((u, v, w, obs, pix), (route, J, l, m, f), o) in enumerate(zip(host_in, model, cy.out)):
        vm = host(o["vis_model"])
        if route == "direct":
            ref = ov.predict_direct(u, v, w, l, m, f) if l.size else np.zeros(u.size, complex)
            bound = fp64_row_bound(u, v, w, l, m, ov.n_minus_1(l, m), f) if l.size else 0
        else:
            rt = ot.build_tree(J, RA, DEC, l, m, f)
            ref = ot.predict_tree(rt, u, v, w)
            bound = fp64_row_bound(u, v, w, rt.leaf_l, rt.leaf_m, rt.leaf_nm1, rt.leaf_flux) + \
                (J + 2) * 4e-16 * np.abs(f).sum()
        assert np.all(np.abs(vm - ref) <= bound), (k, "vis_model")
        r = host(o["resid"])
        assert np.array_equal(r, obs - vm), (k, "resid")      # one subtraction per part
        chi2 = float(host(o["chi2"])[0])
        assert chi2 == pytest.approx(1e4 * np.sum(np.abs(r) ** 2), rel=1e-13), (k, "chi2")
        if pix is not None:
            img = host(o["image"])
            rimg = ov.adjoint(u, v, w, r, *pix)
            b = fp64_row_bound(*pix, u, v, w, np.abs(r))
            assert np.all(np.abs(img - rimg) <= b), (k, "image")
        if "grads" in o and l.size:
            got = [host(g)[: l.size] for g in o["grads"]]
            refg = ov.grad_direct(u, v, w, r, l, m, f, alpha=-2e4)
            for g, rg, s in zip(got, refg, _grad_scales(u, v, w, l, m, f, r)):
                assert np.all(np.abs(g - rg) <= 2e4 * s), (k, "grads")
        e, _ = errors(vm, ref, max(np.abs(f).sum(), 1e-300))
        note(f"cycle instance {k} ({route}, {l.size} components): E_max {e:.2e}")


def test_cycle_graph_replays_new_models(env):
    torch, swv = env
    rng = np.random.default_rng(2025)
    inst, host_in = _make(torch, swv, rng)
    cy = swv.MajorCycle(inst)
    # cycle 1
    mA = _model(rng, (200, 40, 150, 30), (1, 1, 8, 10))
    _set(torch, swv, cy, mA)
    cy.run()
    swv.synchronize()
    eager_a = _snapshot(cy)
    _oracle_checks(cy, host_in, mA)
    cy.capture()
    for rep in range(3):
        for o in cy.out:                       # eager work between the replays
            o["vis_model"].zero_()
            o["image"].zero_() if "image" in o else None
        torch.cuda.synchronize()
        cy.launch()
        swv.synchronize()
        assert not _equal(torch, eager_a, _snapshot(cy)), rep
    # cycle 2: other component counts (the full capacity and none), other trees
    # and depths, replayed without a new capture
    mB = _model(rng, (300, 0, 260, 12), (1, 1, 9, 6))
    _set(torch, swv, cy, mB)
    cy.launch()
    swv.synchronize()
    graph_b = _snapshot(cy)
    # the empty component list predicts zero and leaves the gradients alone
    assert torch.count_nonzero(cy.out[1]["vis_model"]) == 0
    assert torch.equal(cy.out[1]["grads"][0], eager_a[1]["grads"][0])
    cy.run()
    swv.synchronize()
    assert not _equal(torch, graph_b, _snapshot(cy))
    _oracle_checks(cy, host_in, mB)
    cy.close()


def test_cycle_argument_errors(env):
    torch, swv = env
    from paper_1909_03956_amd._lib import SWV_EINVAL, SwvError
    rng = np.random.default_rng(7)
    inst, _ = _make(torch, swv, rng)
    cy = swv.MajorCycle(inst)
    with pytest.raises(SwvError) as e:
        cy.launch()                            # nothing captured yet
    assert e.value.code == SWV_EINVAL
    x = dev(np.zeros(301), torch)
    with pytest.raises(SwvError) as e:
        cy.set_components(0, x, x, x)          # above comp_cap
    assert e.value.code == SWV_EINVAL
    with pytest.raises(SwvError) as e:
        cy.set_components(2, x[:3], x[:3], x[:3])   # a tree instance
    assert e.value.code == SWV_EINVAL
    t = swv.Tree(10, RA, DEC, np.zeros(1), np.zeros(1), np.ones(1))
    with pytest.raises(SwvError) as e:
        cy.set_tree(2, t)                      # J = 10 above the cap of 9
    assert e.value.code == SWV_EINVAL
    t.close()
    cy.run()                                   # no model anywhere: zeros
    swv.synchronize()
    assert all(torch.count_nonzero(o["vis_model"]) == 0 for o in cy.out)
    cy.close()
