"""GPU test of swv_adjoint_noalloc, the adjoint whose partial sums live in the
library's fixed device array: called through the C ABI, it gives the same
image as swv_adjoint (the same tiling and summation order, so the same bits,
and within the FP64 bar of the oracle), on two calls in a row, the second
smaller, and refuses a problem whose partial sums exceed the array."""
import ctypes as C
import math

import numpy as np
import pytest

from oracle import sphere as sp
from oracle import visibility as ov
from synth import configs, models

from .gpu_util import dev, dev_c, errors, host, note, require_gpu

pytestmark = pytest.mark.gpu
TOL64 = 1e-12
TOL32 = 1e-6


@pytest.fixture(scope="module")
def env():
    return require_gpu()


def _call(swv, fn, ctx, u, v, w, y, l, m, nm1, sign, prec, out):
    p = lambda t: C.c_void_p(t.data_ptr())  # noqa: E731
    return getattr(swv.lib(), fn)(ctx.handle, u.numel(), p(u), p(v), p(w), p(y), l.numel(),
                                  p(l), p(m), p(nm1), sign, prec, p(out))


def _case(rng, n_vis, n_pix):
    W = configs.CFG2
    u, v, w = (a[:n_vis] for a in W.track.uvw())
    y = models.complex_noise(n_vis, configs.CFG5_NOISE_SIGMA, rng)
    pix, pl, pm, pn = sp.pixels_in_disk(configs.CFG5_J, W.ra_p, W.dec_p,
                                        math.radians(configs.CFG5_DISK_RADIUS_DEG))
    sel = np.sort(rng.choice(pix.size, n_pix, replace=False))
    return u, v, w, y, pl[sel], pm[sel], pn[sel]


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_equals_adjoint_twice(env, prec):
    torch, swv = env
    from paper_1909_03956_amd._lib import SWV_OK
    ctx = swv.context()
    rng = np.random.default_rng(7100 + prec)
    # two calls in a row: the second, smaller one finds the first one's
    # partial sums in the array and must not read them
    for n_vis, n_pix in ((2_000_000, 955), (300_001, 123)):
        u, v, w, y, l, m, nm1 = _case(rng, n_vis, n_pix)
        U, V, Wd, L, M, N = (dev(a, torch) for a in (u, v, w, l, m, nm1))
        Y = dev_c(y, torch)
        ref = torch.full((n_pix,), complex("nan"), dtype=torch.complex128, device="cuda")
        got = torch.full((n_pix,), complex("nan"), dtype=torch.complex128, device="cuda")
        note(f"noalloc prec={prec} n_vis={n_vis} n_pix={n_pix}")
        assert _call(swv, "swv_adjoint", ctx, U, V, Wd, Y, L, M, N, -1, prec, ref) == SWV_OK
        assert _call(swv, "swv_adjoint_noalloc", ctx, U, V, Wd, Y, L, M, N, -1, prec,
                     got) == SWV_OK
        ctx.synchronize()
        g, r = host(got), host(ref)
        assert np.all(np.isfinite(g))
        scale = np.abs(y).sum()
        e_max, _ = errors(g, r, scale)
        assert e_max <= (TOL64 if prec == 0 else TOL32)
        assert np.array_equal(g.view(np.float64), r.view(np.float64))   # same bits
        # and against the oracle on a few pixels
        k = np.unique(np.r_[0, n_pix - 1, rng.choice(n_pix, 3, replace=False)])
        o = ov.adjoint(u, v, w, y, l[k], m[k], nm1[k], chunk=65536)
        e_o, _ = errors(g[k], o, scale)
        note(f"  E_max vs swv_adjoint {e_max:.3e}, vs oracle {e_o:.3e}")
        assert e_o <= (TOL64 if prec == 0 else TOL32)


def test_noalloc_refuses_oversize_and_bad_arguments(env):
    torch, swv = env
    from paper_1909_03956_amd._lib import SWV_EINVAL, SWV_ENOMEM
    ctx = swv.context()
    # 400,000 pixels need at least 8 row chunks x 16 B = 51 MB of partial sums;
    # the check happens on the host before anything is enqueued, so the
    # buffers are never read (small stand-ins suffice)
    t = torch.zeros(4, dtype=torch.float64, device="cuda")
    tc = torch.zeros(4, dtype=torch.complex128, device="cuda")
    p = C.c_void_p(t.data_ptr())
    pc = C.c_void_p(tc.data_ptr())
    rc = swv.lib().swv_adjoint_noalloc(ctx.handle, 4_000_000, p, p, p, pc, 400_000, p, p, p,
                                       -1, 0, pc)
    assert rc == SWV_ENOMEM
    assert b"fixed scratch" in swv.lib().swv_last_error()
    rc = swv.lib().swv_adjoint_noalloc(ctx.handle, 4, None, p, p, pc, 4, p, p, p, -1, 0, pc)
    assert rc == SWV_EINVAL
    rc = swv.lib().swv_adjoint_noalloc(None, 4, p, p, p, pc, 4, p, p, p, -1, 0, pc)
    assert rc == SWV_EINVAL
    ctx.synchronize()
