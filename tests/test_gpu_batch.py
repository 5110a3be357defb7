"""GPU tests of the batched persistent form, its HIP-graph capture and the
autotuner.  Per-row arithmetic does not depend on the tiling, so batched and
single-instance predictions must agree bit for bit; the batched workload
(64 channels x 4 pointings) is also checked against the oracle."""
import json
import os
import time

import numpy as np
import pytest

from oracle import tree as ot
from oracle import visibility as ov
from synth import configs

from .gpu_util import dev, errors, host, note, require_gpu

pytestmark = pytest.mark.gpu
TOL64 = 1e-12


@pytest.fixture(scope="module")
def env():
    return require_gpu()


def _instances(torch, swv, rng):
    """Mixed direct (FP64, FP32c) and tree instances of ragged sizes."""
    specs = [("direct", "fp64", 0, 5), ("direct", "fp64", 1, 0), ("direct", "fp64", 4097, 33),
             ("direct", "f32c", 100003, 17), ("tree", 1, 63, 40), ("tree", 6, 777, 200),
             ("tree", 9, 30011, 300), ("tree", 12, 2048, 60), ("direct", "fp64", 65, 1),
             ("direct", "fp64", 200000, 300)]
    insts, refs = [], []
    for route, p, n, k in specs:
        u, v, w = (dev(rng.uniform(-3e4, 3e4, n), torch) for _ in range(3))
        l, m = rng.uniform(-0.04, 0.04, k), rng.uniform(-0.04, 0.04, k)
        f = rng.lognormal(-3, 1, k)
        if route == "direct":
            L, M, F = dev(l, torch), dev(m, torch), dev(f, torch)
            dt = torch.complex128 if p == "fp64" else torch.complex64
            out = torch.full((n,), 7.0, dtype=dt, device="cuda")
            insts.append(dict(route="direct", prec=p, u=u, v=v, w=w, l=L, m=M, flux=F, out=out))
            refs.append(lambda u=u, v=v, w=w, L=L, M=M, F=F, p=p:
                        swv.predict_direct(u, v, w, L, M, F, prec=p))
        else:
            t = swv.Tree(p, 1.1, 0.4, l, m, f)
            out = torch.full((n,), 7.0, dtype=torch.complex128, device="cuda")
            insts.append(dict(route="tree", tree=t, u=u, v=v, w=w, out=out))
            refs.append(lambda u=u, v=v, w=w, t=t: t.predict(u, v, w))
    return insts, refs


def _mismatches(insts, refs, torch):
    """(instance, route, prec, rows differing, first row, max |diff|) of every
    instance whose batched output is not bitwise the single-instance one."""
    bad = []
    for k, (d, ref) in enumerate(zip(insts, refs)):
        r = ref()
        if not torch.equal(d["out"], r):
            diff = (d["out"].to(torch.complex128) - r.to(torch.complex128)).abs()
            rows = torch.nonzero(diff > 0).flatten()
            bad.append((k, d["route"], d.get("prec", "fp64"), int(rows.numel()),
                        int(rows[0]) if rows.numel() else -1, float(diff.max())))
    return bad


def test_batch_equals_single_instance_bitwise(env):
    torch, swv = env
    insts, refs = _instances(torch, swv, np.random.default_rng(1))
    plan = swv.BatchPlan(insts)
    st = plan.stats()
    assert st["n_instances"] == len(insts) and st["n_items"] > 0
    plan.run()
    swv.synchronize()
    first = [d["out"].clone() for d in insts]
    plan.run()
    swv.synchronize()
    assert all(torch.equal(a, d["out"]) for a, d in zip(first, insts)), "batched run not reproducible"
    bad = _mismatches(insts, refs, torch)
    plan.close()
    assert not bad, bad


def test_batch_with_deep_trees_bitwise(env):
    # trees beyond J = 12 go through the branch walker, in the batch as alone
    torch, swv = env
    rng = np.random.default_rng(11)
    insts, refs = [], []
    for J, n, k in ((14, 5000, 90), (20, 3001, 140), (29, 777, 25), (9, 4096, 300)):
        u, v, w = (dev(rng.uniform(-3e5, 3e5, n), torch) for _ in range(3))
        l, m = rng.uniform(-0.02, 0.02, k), rng.uniform(-0.02, 0.02, k)
        t = swv.Tree(J, 0.7, -0.2, l, m, rng.lognormal(-3, 1, k))
        out = torch.full((n,), 7.0, dtype=torch.complex128, device="cuda")
        insts.append(dict(route="tree", tree=t, u=u, v=v, w=w, out=out))
        refs.append(lambda u=u, v=v, w=w, t=t: t.predict(u, v, w))
    plan = swv.BatchPlan(insts)
    plan.run()
    swv.synchronize()
    bad = _mismatches(insts, refs, torch)
    plan.close()
    assert not bad, bad


def test_graph_replay_equals_eager(env):
    torch, swv = env
    insts, refs = _instances(torch, swv, np.random.default_rng(2))
    plan = swv.BatchPlan(insts)
    graph = plan.capture()
    for rep in range(3):
        for d in insts:
            d["out"].zero_()                      # eager work between replays
        torch.cuda.synchronize()
        graph.launch()
        swv.synchronize()
        bad = _mismatches(insts, refs, torch)
        assert not bad, (rep, bad)
    # the captured cycle reads the components again on every replay
    for d in insts:
        if d["route"] == "direct":
            d["flux"].mul_(1.5)
    graph.launch()
    swv.synchronize()
    bad = _mismatches(insts, refs, torch)
    assert not bad, ("after update", bad)
    graph.close()
    plan.close()


def test_autotune_writes_loads_and_keeps_results(env, tmp_path):
    torch, swv = env
    ctx = swv.context()
    path = str(tmp_path / "tune.json")
    t0 = time.time()
    ctx.autotune(path, quick=True)
    note(f"autotune (quick) took {time.time() - t0:.2f} s")
    table = json.load(open(path))
    assert table["format"] == "swvis-tune-1" and len(table["chosen"]) == 10
    chosen = {(e["family"], e["size_class"]): (e["per_lane"], e["block"]) for e in table["chosen"]}
    for (fam, cls), (pl, bl) in chosen.items():
        assert ctx.tune_get(fam, cls) == (pl, bl)
    for e in table["timings"]:
        assert e["ms"] > 0
    fresh = swv.Context()
    fresh.tune_load(path)
    assert all(fresh.tune_get(f, c) == chosen[(f, c)] for f, c in chosen)
    # every compiled direct shape gives the same bits
    rng = np.random.default_rng(3)
    n = 70001
    u, v, w = (dev(rng.uniform(-5e4, 5e4, n), torch) for _ in range(3))
    L, M, F = (dev(rng.uniform(-0.03, 0.03, 50), torch), dev(rng.uniform(-0.03, 0.03, 50), torch),
               dev(rng.lognormal(-3, 1, 50), torch))
    ref = None
    for pl in (1, 2, 4):
        for bl in (64, 128, 256):
            ctx.tune_set(0, 0, pl, bl)
            out = swv.predict_direct(u, v, w, L, M, F)
            ref = out if ref is None else ref
            assert torch.equal(out, ref)
    ctx.tune_load(path)


def _check_instances(B, plan_outputs, chosen, torch, label):
    worst = 0.0
    for k, kind in chosen:
        inst = B.instances[k]
        kept, l, m, f = B.instance_rows_kept(inst)
        rows = configs.sample_rows(kept.size, 384, seed=k, tile=64)
        u, v, w = B.instance_uvw_rows(inst, kept[rows])
        got = host(plan_outputs[(k, kind)][torch.as_tensor(rows, device="cuda")])
        if kind == "direct":
            ref = ov.predict_direct(u, v, w, l, m, f)
        else:
            t = ot.build_tree(inst.J, configs.CFG2.ra_p, configs.CFG2.dec_p, l, m, f)
            ref = ot.predict_tree(t, u, v, w)
        e_max, e_rms = errors(got, ref, f.sum())
        note(f"{label} instance {k} ({kind}, J={inst.J}, N_C={inst.n_comp}, {kept.size} rows): "
             f"E_max={e_max:.3e} E_rms={e_rms:.3e}")
        worst = max(worst, e_max)
    return worst


def _run_batched(torch, swv, B, label):
    """Generates every instance on the GPU, runs the direct and the tree routes
    as two batched plans, returns outputs and throughput."""
    insts_d, insts_t, outs, keep = [], [], {}, []
    ra, dec = configs.CFG2.ra_p, configs.CFG2.dec_p
    total_rows = total_terms = 0
    t_gen = time.time()
    for inst in B.instances:
        kept, l, m, f = B.instance_rows_kept(inst)
        u, v, w = B.instance_uvw_torch(inst, kept, "cuda")
        L, M, F = dev(l, torch), dev(m, torch), dev(f, torch)
        od = torch.empty(kept.size, dtype=torch.complex128, device="cuda")
        ot_ = torch.empty(kept.size, dtype=torch.complex128, device="cuda")
        tree = swv.Tree(inst.J, ra, dec, l, m, f)
        insts_d.append(dict(route="direct", u=u, v=v, w=w, l=L, m=M, flux=F, out=od))
        insts_t.append(dict(route="tree", tree=tree, u=u, v=v, w=w, out=ot_))
        outs[(inst.index, "direct")] = od
        outs[(inst.index, "tree")] = ot_
        total_rows += kept.size
        total_terms += kept.size * inst.n_comp
    torch.cuda.synchronize()
    note(f"{label}: {len(B.instances)} instances, {total_rows} rows, generated in "
         f"{time.time() - t_gen:.1f} s")
    pd, pt = swv.BatchPlan(insts_d), swv.BatchPlan(insts_t)
    gd, gt = pd.capture(), pt.capture()
    for g in (gd, gt):          # warm
        g.launch()
    swv.synchronize()
    times = {}
    for name, g in (("direct", gd), ("tree", gt)):
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        g.launch()
        e.record()
        torch.cuda.synchronize()
        times[name] = s.elapsed_time(e) * 1e-3
        note(f"{label} {name} route: {times[name] * 1e3:.1f} ms, "
             f"{total_terms / times[name] / 1e9:.1f} Gvis.terms/s (N_C terms), "
             f"plan {pd.stats() if name == 'direct' else pt.stats()}")
    swv.synchronize()
    keep += [pd, pt, gd, gt]
    return outs, keep


def test_device_tracks_equal_host_tracks(env):
    # the batched workload's rows are made on the device; the oracle's on the host
    torch, swv = env
    B = configs.BatchedWorkload(scale=0.01)
    for k in (0, 100, 255):
        inst = B.instances[k]
        kept, *_ = B.instance_rows_kept(inst)
        dev_uvw = B.instance_uvw_torch(inst, kept, "cuda")
        rows = configs.sample_rows(kept.size, 512, seed=k, tile=64)
        host_uvw = B.instance_uvw_rows(inst, kept[rows])
        for a, b in zip(dev_uvw, host_uvw):
            assert np.array_equal(host(a[torch.as_tensor(rows, device="cuda")]), b)


def test_batched_workload_scaled(env):
    torch, swv = env
    B = configs.BatchedWorkload(scale=0.01)
    outs, keep = _run_batched(torch, swv, B, "cfg4 x0.01")
    chosen = [(0, "direct"), (77, "tree"), (150, "direct"), (255, "tree")]
    assert _check_instances(B, outs, chosen, torch, "cfg4 x0.01") <= TOL64


def test_batched_workload_full_size(env):
    torch, swv = env
    B = configs.BatchedWorkload()
    outs, keep = _run_batched(torch, swv, B, "cfg4")
    big = max(range(len(B.instances)), key=lambda k: B.instances[k].n_comp)
    chosen = [(big, "direct"), (3, "tree"), (200, "direct"), (131, "tree")]
    assert _check_instances(B, outs, chosen, torch, "cfg4") <= TOL64


def test_batch_level_walker_every_depth_bitwise(env):
    """A plan whose trees all fit the level walker (J <= 10): the four deepest
    depths of the plan run walks compiled for their J, the shallower ones the
    walk with J tested at run time; every output, FP64 and F32C, bitwise the
    single-instance prediction, before and after a graph capture."""
    torch, swv = env
    rng = np.random.default_rng(31)
    insts, refs = [], []
    for J, n, k, prec in ((2, 1000, 30, "fp64"), (4, 3001, 80, "fp64"), (6, 777, 200, "fp64"),
                          (7, 4097, 150, "fp64"), (8, 2048, 300, "fp64"), (9, 5000, 250, "fp64"),
                          (10, 6001, 400, "fp64"), (3, 999, 40, "f32c"), (10, 2500, 300, "f32c"),
                          (1, 65, 3, "fp64")):
        u, v, w = (dev(rng.uniform(-3e4, 3e4, n), torch) for _ in range(3))
        l, m = rng.uniform(-0.04, 0.04, k), rng.uniform(-0.04, 0.04, k)
        t = swv.Tree(J, 1.1, 0.4, l, m, rng.lognormal(-3, 1, k))
        dt = torch.complex64 if prec == "f32c" else torch.complex128
        out = torch.full((n,), 7.0, dtype=dt, device="cuda")
        insts.append(dict(route="tree", prec=prec, tree=t, u=u, v=v, w=w, out=out))
        refs.append(lambda u=u, v=v, w=w, t=t, p=prec: t.predict(u, v, w, prec=p))
    plan = swv.BatchPlan(insts)
    plan.run()
    swv.synchronize()
    assert _mismatches(insts, refs, torch) == []
    graph = plan.capture()
    for d in insts:
        d["out"].fill_(3.0)
    graph.launch()
    swv.synchronize()
    assert _mismatches(insts, refs, torch) == []
    graph.close()
    plan.close()


def test_batch_f32c_trees_bitwise(env):
    """Tree instances in FP32C (and FP64, and F32C direct ones) in one plan:
    every output bitwise equal to the single-instance prediction; the F32C
    trees within the 1e-6 bar of the oracle."""
    torch, swv = env
    rng = np.random.default_rng(21)
    insts, refs, checks = [], [], []
    for J, n, k, prec in ((6, 777, 200, "f32c"), (9, 30011, 300, "f32c"), (9, 20000, 120, "fp64"),
                          (12, 2048, 60, "f32c"), (3, 1, 5, "f32c")):
        uh, vh, wh = (rng.uniform(-3e4, 3e4, n) for _ in range(3))
        u, v, w = dev(uh, torch), dev(vh, torch), dev(wh, torch)
        l, m = rng.uniform(-0.04, 0.04, k), rng.uniform(-0.04, 0.04, k)
        f = rng.lognormal(-3, 1, k)
        t = swv.Tree(J, 1.1, 0.4, l, m, f)
        dt = torch.complex64 if prec == "f32c" else torch.complex128
        out = torch.full((n,), 7.0, dtype=dt, device="cuda")
        insts.append(dict(route="tree", prec=prec, tree=t, u=u, v=v, w=w, out=out))
        refs.append(lambda u=u, v=v, w=w, t=t, p=prec: t.predict(u, v, w, prec=p))
        checks.append((J, l, m, f, uh, vh, wh, prec))
    L, M, F = (dev(rng.uniform(-0.04, 0.04, 50), torch) for _ in range(3))
    ud = dev(rng.uniform(-3e4, 3e4, 5000), torch)
    od = torch.empty(5000, dtype=torch.complex64, device="cuda")
    insts.append(dict(route="direct", prec="f32c", u=ud, v=ud, w=ud, l=L, m=M, flux=F.abs(),
                      out=od))
    refs.append(lambda: swv.predict_direct(ud, ud, ud, L, M, F.abs(), prec="f32c"))
    plan = swv.BatchPlan(insts)
    plan.run()
    swv.synchronize()
    assert _mismatches(insts, refs, torch) == []
    graph = plan.capture()
    for d in insts:
        d["out"].fill_(3.0)
    graph.launch()
    swv.synchronize()
    assert _mismatches(insts, refs, torch) == []
    for d, (J, l, m, f, uh, vh, wh, prec) in zip(insts, checks):
        if prec != "f32c":
            continue
        rt = ot.build_tree(J, 1.1, 0.4, l, m, f)
        ref = ot.predict_tree(rt, uh, vh, wh)
        assert errors(host(d["out"]).astype(np.complex128), ref, f.sum())[0] <= 1e-6
    with pytest.raises(TypeError):
        swv.BatchPlan([dict(route="tree", prec="f32c", tree=insts[0]["tree"], u=insts[0]["u"],
                            v=insts[0]["v"], w=insts[0]["w"],
                            out=torch.empty(777, dtype=torch.complex128, device="cuda"))])
    graph.close()
    plan.close()


def test_plan_keeps_destroyed_tree_alive(env):
    # the caller's tree handle is destroyed right after planning (the C ABI's
    # swv_tree_destroy); the plan and its graph hold their own reference, so
    # their runs still read valid records and predict the same values
    torch, swv = env
    from paper_1909_03956_amd._lib import SWV_OK
    rng = np.random.default_rng(31)
    n, k = 20000, 150
    u, v, w = (dev(rng.uniform(-3e4, 3e4, n), torch) for _ in range(3))
    l, m, f = rng.uniform(-0.03, 0.03, k), rng.uniform(-0.03, 0.03, k), rng.lognormal(-3, 1, k)
    ref = swv.Tree(9, 1.0, 0.3, l, m, f).predict(u, v, w)
    t = swv.Tree(9, 1.0, 0.3, l, m, f)
    out = torch.full((n,), 7.0, dtype=torch.complex128, device="cuda")
    plan = swv.BatchPlan([dict(route="tree", tree=t, u=u, v=v, w=w, out=out)])
    graph = plan.capture()
    assert swv.lib().swv_tree_destroy(t.handle) == SWV_OK   # the caller's reference
    t._h = type(t._h)()                                     # the wrapper must not release it again
    plan.run()
    swv.synchronize()
    assert torch.equal(out, ref)
    out.zero_()
    graph.launch()
    swv.synchronize()
    assert torch.equal(out, ref)
    graph.close()
    plan.close()   # frees the tree with the plan's reference


def test_process_exit_after_every_kind_of_object(env, tmp_path):
    # a process that leaves contexts (with an FFT plan), trees, plans and
    # graphs alive and has run a cooperative Hogbom cycle exits normally: the
    # binding destroys them in dependency order from its exit hook
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = r'''
import numpy as np, torch
import paper_1909_03956_amd as swv
from paper_1909_03956_amd import api
d = torch.device("cuda", 0)
rng = np.random.default_rng(1)
D = lambda x: torch.as_tensor(x, dtype=torch.float64, device=d)
u, v, w = (D(rng.uniform(-400.0, 400.0, 5000)) for _ in range(3))
l, m, f = rng.uniform(-0.02, 0.02, 50), rng.uniform(-0.02, 0.02, 50), rng.lognormal(-3, 1, 50)
t = swv.Tree(8, 0.5, 0.4, l, m, f)
out = torch.empty(5000, dtype=torch.complex128, device=d)
plan = swv.BatchPlan([dict(route="tree", tree=t, u=u, v=v, w=w, out=out)])
g = plan.capture(); g.launch()
img = torch.zeros((160, 160), dtype=torch.float64, device=d); img[80, 80] = 1.0
vis, st = swv.predict_degrid(img, u, v, w, 1e-3, support=6)
beam = torch.zeros((319, 319), dtype=torch.float64, device=d); beam[159, 159] = 1.0
pix, val = swv.hogbom(img, beam, 0.5, 0.0, 5)
torch.cuda.synchronize()
print("live", {k: len(s) for k, s in api._LIVE.items()}, flush=True)
'''
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True,
                       timeout=300)
    note(r.stdout.strip(), r.stderr.strip()[-500:])
    assert r.returncode == 0, (r.returncode, r.stderr[-2000:])
    assert "live" in r.stdout
