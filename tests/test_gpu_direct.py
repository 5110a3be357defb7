"""GPU parity of the direct sum (Eq. 12) against the oracle, through the C ABI.

Tolerance (FP64): E_max = max_j |V_gpu - V_oracle| / sum_k |I_k| <= 1e-12.
The oracle reduces the phase exactly; the GPU rounds phi ~ 1e4 cycles in
FP64 (one ulp ~ 2e-12 cycles), so per-term phase errors are ~1e-12 rad and
average down over components.
Tolerance (FP32-compensated): E_max <= 1e-6, the bound of the form's per-term
rounding: FP32 rounding of r in [0, 1) (2 pi 2^-25), FP32 sincos (measured below),
the FP32 flux (2^-24), the two FMAs through which a pair of components' products
enters the sums (at most 2 x 2^-24 of a term), and the Kahan sums (2 x 2^-24).
"""
import numpy as np
import pytest

from oracle import visibility as ov
from synth import configs

from .gpu_util import dev, errors, fp64_row_bound, host, note, require_gpu

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-6


@pytest.fixture(scope="module")
def env():
    return require_gpu()


def _run(env, u, v, w, l, m, f, sign=-1, prec="fp64"):
    torch, swv = env
    out = swv.predict_direct(dev(u, torch), dev(v, torch), dev(w, torch), dev(l, torch),
                             dev(m, torch), dev(f, torch), sign=sign, prec=prec)
    swv.synchronize()
    return host(out)


@pytest.mark.parametrize("sign", [-1, 1])
def test_cfg1_full(env, sign):
    W = configs.CFG1
    u, v, w = W.track.uvw()
    l, m, f = W.components()
    got = _run(env, u, v, w, l, m, f, sign)
    ref = ov.predict_direct(u, v, w, l, m, f, sign)
    e_max, e_rms = errors(got, ref, f.sum())
    note(f"cfg1 direct fp64 sign={sign}: E_max={e_max:.3e} E_rms={e_rms:.3e}")
    assert e_max <= TOL64


@pytest.mark.parametrize("n_vis", [1, 5, 63, 64, 65, 257, 511, 1000, 4099])
@pytest.mark.parametrize("n_comp", [1, 3, 17])
def test_small_and_ragged(env, n_vis, n_comp):
    rng = np.random.default_rng(n_vis * 100 + n_comp)
    u, v, w = (rng.uniform(-2e5, 2e5, n_vis) for _ in range(3))
    l, m = rng.uniform(-0.03, 0.03, n_comp), rng.uniform(-0.03, 0.03, n_comp)
    f = rng.lognormal(-3, 1, n_comp)
    got = _run(env, u, v, w, l, m, f)
    ref = ov.predict_direct(u, v, w, l, m, f)
    # few components do not average the per-term phase rounding: every row
    # is held to the bound derived from the FP64 evaluation of the phase
    bound = fp64_row_bound(u, v, w, l, m, ov.n_minus_1(l, m), f)
    assert np.all(np.abs(got - ref) <= bound)


def test_no_components_gives_zero(env):
    got = _run(env, np.ones(300), np.ones(300), np.ones(300), np.zeros(0), np.zeros(0),
               np.zeros(0))
    assert np.all(got == 0)


def test_unit_source_at_phase_centre_is_exactly_one(env):
    rng = np.random.default_rng(1)
    u, v, w = (rng.uniform(-4e5, 4e5, 1000) for _ in range(3))
    got = _run(env, u, v, w, [0.0], [0.0], [1.0])
    assert np.all(got == 1.0 + 0j)


def test_sign_flip_is_exact_conjugate(env):
    W = configs.CFG1
    u, v, w = W.track.uvw()
    l, m, f = W.components()
    a = _run(env, u[:5000], v[:5000], w[:5000], l, m, f, -1)
    b = _run(env, u[:5000], v[:5000], w[:5000], l, m, f, +1)
    assert np.array_equal(a, np.conj(b))


@pytest.mark.parametrize("name", ["cfg2", "cfg3"])
def test_full_size_sampled_rows(env, name):
    torch, swv = env
    W = configs.WORKLOADS[name]
    u, v, w = W.track.uvw()
    l, m, f = W.components()
    out = swv.predict_direct(dev(u, torch), dev(v, torch), dev(w, torch), dev(l, torch),
                             dev(m, torch), dev(f, torch))
    swv.synchronize()
    rows = configs.sample_rows(u.size, 2048 if name == "cfg3" else 4096, seed=7)
    got = host(out[torch.as_tensor(rows, device="cuda")])
    ref = ov.predict_direct(u[rows], v[rows], w[rows], l, m, f)
    e_max, e_rms = errors(got, ref, f.sum())
    note(f"{name} direct fp64 ({rows.size} sampled rows of {u.size}): "
         f"E_max={e_max:.3e} E_rms={e_rms:.3e}")
    assert e_max <= TOL64
    bound = fp64_row_bound(u[rows], v[rows], w[rows], l, m, ov.n_minus_1(l, m), f)
    assert np.all(np.abs(got - ref) <= bound)


@pytest.mark.parametrize("prec", ["f32c"])
def test_precision_form_cfg3(env, prec):
    torch, swv = env
    W = configs.CFG3
    u, v, w = W.track.uvw()
    l, m, f = W.components()
    out = swv.predict_direct(dev(u, torch), dev(v, torch), dev(w, torch), dev(l, torch),
                             dev(m, torch), dev(f, torch), prec=prec)
    swv.synchronize()
    assert out.dtype == torch.complex64
    rows = configs.sample_rows(u.size, 2048, seed=8)
    got = host(out[torch.as_tensor(rows, device="cuda")]).astype(np.complex128)
    ref = ov.predict_direct(u[rows], v[rows], w[rows], l, m, f)
    e_max, e_rms = errors(got, ref, f.sum())
    note(f"cfg3 direct {prec}: E_max={e_max:.3e} E_rms={e_rms:.3e}")
    assert e_max <= TOL32


@pytest.mark.parametrize("n_comp", [1, 2, 3, 16, 17, 1000, 1001])
@pytest.mark.parametrize("sign", [-1, 1])
def test_f32c_component_pairs(env, n_comp, sign):
    """The FP32-compensated form sums components in pairs with an odd last
    one alone: even and odd counts, both signs, against the oracle at the
    form's bound, on 8,195 rows of cfg1 (a multiple of no block size)."""
    rng = np.random.default_rng(n_comp * 10 + (sign > 0))
    u, v, w = configs.CFG1.track.uvw()
    u, v, w = u[:8195], v[:8195], w[:8195]
    l, m = rng.uniform(-0.03, 0.03, n_comp), rng.uniform(-0.03, 0.03, n_comp)
    f = rng.lognormal(-3, 1, n_comp)
    got = _run(env, u, v, w, l, m, f, sign, "f32c").astype(np.complex128)
    ref = ov.predict_direct(u, v, w, l, m, f, sign)
    e_max, e_rms = errors(got, ref, f.sum())
    note(f"direct f32c {n_comp} components sign={sign}: E_max={e_max:.3e} E_rms={e_rms:.3e}")
    assert e_max <= TOL32


@pytest.mark.parametrize("prec", ["fp64", "f32c"])
def test_phasor_accuracy_dense(env, prec):
    # one unit component at l = 1/2, u = 2 r (exact): V = exp(-2 pi i r)
    n = 1 << 16
    r = (np.arange(n) - n // 2) / n
    u = 2.0 * r
    got = _run(env, u, np.zeros(n), np.zeros(n), [0.5], [0.0], [1.0], -1, prec).astype(
        np.complex128)
    ref = np.exp(-2j * np.pi * r)
    err = np.abs(got - ref).max()
    note(f"phasor {prec}: max |error| over {n} phases = {err:.3e}")
    assert err <= (2e-15 if prec == "fp64" else 2.5e-7)


@pytest.mark.parametrize("prec", ["fp64", "f32c"])
def test_every_tile_shape_same_bits(env, prec):
    """A row's arithmetic does not depend on the tile shape (rows per lane,
    threads per block): all nine shapes give the same bits, on a row count
    that is a multiple of no tile, with an odd component count."""
    torch, swv = env
    ctx = swv.context()
    fam, small = (0 if prec == "fp64" else 1), 0
    saved = ctx.tune_get(fam, small)
    rng = np.random.default_rng(77)
    n_vis, n_comp = 5003, 101
    u, v, w = (rng.uniform(-2e5, 2e5, n_vis) for _ in range(3))
    l, m = rng.uniform(-0.03, 0.03, n_comp), rng.uniform(-0.03, 0.03, n_comp)
    f = rng.lognormal(-3, 1, n_comp)
    outs = {}
    try:
        for vpl in (1, 2, 4):
            for block in (64, 128, 256):
                ctx.tune_set(fam, small, vpl, block)
                outs[(vpl, block)] = _run(env, u, v, w, l, m, f, -1, prec)
    finally:
        ctx.tune_set(fam, small, *saved)
    first = outs[(1, 64)]
    for shape, got in outs.items():
        assert np.array_equal(got, first), shape
    ref = ov.predict_direct(u, v, w, l, m, f)
    if prec == "fp64":
        # few components do not average the per-term phase rounding
        assert np.all(np.abs(first - ref) <= fp64_row_bound(u, v, w, l, m, ov.n_minus_1(l, m), f))
    else:
        e_max, _ = errors(first.astype(np.complex128), ref, f.sum())
        assert e_max <= TOL32


def test_run_to_run_bitwise(env):
    W = configs.CFG1
    u, v, w = W.track.uvw()
    l, m, f = W.components()
    a = _run(env, u, v, w, l, m, f)
    b = _run(env, u, v, w, l, m, f)
    assert np.array_equal(a, b)


def test_deferred_domain_errors(env):
    torch, swv = env
    from paper_1909_03956_amd._lib import SWV_EDOMAIN, SwvError
    ones = dev(np.ones(100), torch)
    bad = dev(np.array([0.8, 0.0]), torch)
    mm = dev(np.array([0.7, 0.0]), torch)
    f = dev(np.array([1.0, 1.0]), torch)
    swv.predict_direct(ones, ones, ones, bad, mm, f)
    with pytest.raises(SwvError) as e:
        swv.synchronize()
    assert e.value.code == SWV_EDOMAIN
    swv.synchronize()   # the flag is cleared
    nanu = dev(np.full(100, np.nan), torch)
    swv.predict_direct(nanu, ones, ones, dev([0.01], torch), dev([0.0], torch),
                       dev([1.0], torch))
    with pytest.raises(SwvError) as e:
        swv.synchronize()
    assert e.value.code == SWV_EDOMAIN


def test_argument_errors(env):
    torch, swv = env
    from paper_1909_03956_amd._lib import SWV_EDOMAIN, SWV_EINVAL, SwvError
    x = dev(np.ones(10), torch)
    with pytest.raises(SwvError) as e:
        swv.predict_direct(x, x, x, x[:2] * 0, x[:2] * 0, x[:2], sign=2)
    assert e.value.code == SWV_EDOMAIN
    with pytest.raises(SwvError) as e:
        swv.predict_direct(x, x, x, x[:2] * 0, x[:2] * 0, x[:2], prec=9)
    assert e.value.code == SWV_EINVAL
    with pytest.raises(ValueError):
        swv.predict_direct(x, x[:5], x, x[:2], x[:2], x[:2])
