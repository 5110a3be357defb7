"""GPU tests of the autograd Functions: torch.autograd.gradcheck (FP64), the
backward of a torch chi^2 against the gradient kernel and the oracle, and the
tree route's leaf-flux gradient against the oracle adjoint."""
import numpy as np
import pytest

from oracle import tree as ot
from oracle import visibility as ov
from synth import configs, models

from .gpu_util import dev, dev_c, host, note, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    return require_gpu()


def test_gradcheck_direct(env):
    torch, swv = env
    from paper_1909_03956_amd.autograd import DirectPredict
    rng = np.random.default_rng(1)
    u, v, w = (dev(rng.uniform(-30, 30, 9), torch) for _ in range(3))
    f = dev(rng.uniform(0.5, 2.0, 4), torch).requires_grad_()
    l = dev(rng.uniform(-0.2, 0.2, 4), torch).requires_grad_()
    m = dev(rng.uniform(-0.2, 0.2, 4), torch).requires_grad_()
    for sign in (-1, 1):
        assert torch.autograd.gradcheck(
            lambda a, b, c: DirectPredict.apply(a, b, c, u, v, w, sign), (f, l, m),
            eps=1e-6, atol=1e-6, rtol=1e-5)


def test_gradcheck_tree_leaf_flux(env):
    torch, swv = env
    from paper_1909_03956_amd.autograd import TreePredict
    rng = np.random.default_rng(2)
    t = swv.Tree(5, 1.0, 0.4, rng.uniform(-0.3, 0.3, 12), rng.uniform(-0.3, 0.3, 12),
                 rng.uniform(0.5, 1.5, 12))
    nl = t.stats()["n_leaves"]
    u, v, w = (dev(rng.uniform(-20, 20, 11), torch) for _ in range(3))
    F = dev(rng.uniform(0.5, 2.0, nl), torch).requires_grad_()
    assert torch.autograd.gradcheck(lambda x: TreePredict.apply(x, t, u, v, w, -1), (F,),
                                    eps=1e-6, atol=1e-6, rtol=1e-5)


def test_torch_chi2_backward_matches_kernel_and_oracle(env):
    torch, swv = env
    from paper_1909_03956_amd.autograd import predict_direct
    W = configs.CFG1
    u, v, w = (a[:20000] for a in W.track.uvw())
    l, m, f = W.components()
    rng = np.random.default_rng(3)
    l2, m2, f2 = models.perturb_model(l, m, f, rng)
    obs = ov.predict_direct(u, v, w, l2, m2, f2) + models.complex_noise(u.size, 0.01, rng)
    U, V, Wt = dev(u, torch), dev(v, torch), dev(w, torch)
    F = dev(f, torch).requires_grad_()
    L = dev(l, torch).requires_grad_()
    M = dev(m, torch).requires_grad_()
    inv_s2 = 1e4
    Vm = predict_direct(U, V, Wt, L, M, F)
    r = dev_c(obs, torch) - Vm
    chi2 = (r.real ** 2 + r.imag ** 2).sum() * inv_s2
    chi2.backward()
    ker = swv.grad_direct(U, V, Wt, r.detach().contiguous(), L.detach(), M.detach(),
                          F.detach(), alpha=-2 * inv_s2)
    # same kernel; torch scales y by -2/sigma^2 before the sums, the direct call after
    for g, k in zip((F.grad, L.grad, M.grad), ker):
        assert ((g - k).abs().max() <= 1e-13 * k.abs().max()).item()
    rr = obs - ov.predict_direct(u, v, w, l, m, f)
    ref = ov.grad_direct(u, v, w, rr, l, m, f, alpha=-2 * inv_s2)
    for name, g, r_ in zip(("flux", "l", "m"), (F.grad, L.grad, M.grad), ref):
        rel = np.max(np.abs(host(g) - r_)) / np.max(np.abs(r_))
        note(f"torch chi^2 backward d/d{name}: max relative difference to the oracle {rel:.2e}")
        assert rel <= 1e-8


def test_conjugate_views_are_materialised(env):
    # torch may hand a lazily conjugated gradient to backward
    torch, swv = env
    rng = np.random.default_rng(6)
    u, v, w = (dev(rng.uniform(-1e3, 1e3, 500), torch) for _ in range(3))
    y = dev_c(models.random_complex(500, rng), torch)
    l, m, nm1 = (dev(x, torch) for x in (rng.uniform(-0.05, 0.05, 9), rng.uniform(-0.05, 0.05, 9),
                                          np.full(9, -1e-3)))
    a = swv.adjoint(u, v, w, y.conj(), l, m, nm1)
    b = swv.adjoint(u, v, w, y.conj().resolve_conj(), l, m, nm1)
    assert y.conj().is_conj() and torch.equal(a, b)


def test_tree_leaf_flux_gradient_vs_oracle(env):
    torch, swv = env
    from paper_1909_03956_amd.autograd import predict_tree
    W = configs.CFG2
    rows = configs.sample_rows(W.track.n_vis, 1 << 15, seed=4, tile=0)
    u, v, w = W.track.uvw_rows(rows)
    l, m, f = W.components()
    t = swv.Tree(9, W.ra_p, W.dec_p, l, m, f)
    lv = t.leaves()
    F = dev(lv["flux"], torch).requires_grad_()
    rng = np.random.default_rng(5)
    y = models.random_complex(u.size, rng)
    Vt = predict_tree(t, F, dev(u, torch), dev(v, torch), dev(w, torch))
    (Vt.conj() * dev_c(y, torch)).real.sum().backward()    # L = Re <V, y>
    rt = ot.build_tree(9, W.ra_p, W.dec_p, l, m, f)
    ref = np.real(ov.adjoint(u, v, w, y, rt.leaf_l, rt.leaf_m, rt.leaf_nm1))
    rel = np.max(np.abs(host(F.grad) - ref)) / np.abs(y).sum()
    note(f"tree J=9 leaf-flux gradient ({lv['flux'].size} leaves, {u.size} rows): "
         f"max |d| / sum|y| = {rel:.2e}")
    assert rel <= 1e-12
