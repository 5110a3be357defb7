#!/usr/bin/env python3
"""Throughput of the model-visibility prediction hot path on one MI355X.

One step is one major cycle of the hot path over the measured workload
(8,355,840 visibilities of a 256-antenna, 20 km array tracked 8 h at dec +30
deg, 1.4 GHz; 2,000 clean components, 70 % in five 0.1 deg blobs):

  direct FP64       V = sum_k I_k e_jk                       (N_C terms per row)
  direct FP32c      same, FP64 phase, FP32 sincos + Kahan     (N_C terms)
  tree J = 8, 9, 10 host tree build + wavelet route (Eq. 17)  (N_C terms each)
  residual, chi^2   r = V_obs - V (FP64 model)
  adjoint           residual image on the level-9 pixels within 4 deg (N_pix terms)
  gradients         d chi^2 / d(I, l, m) of every component  (N_C terms)

value = (sum over the step of rows x terms) / step time, in Gvis.terms/s.
Inputs are resident in device memory before the timed region.  One JSON line
goes to stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gvis·terms/s for model-visibility prediction, direct vs tree, FP64 vs FP32-comp"
UNIT = "Gvis·terms/s"
PEAK_FP64_TFLOPS = 78.6        # MI355X FP64 vector: 256 CU x 2.4 GHz x 128 flop/clk
PEAK_FP32_TFLOPS = 157.3       # MI355X FP32 vector (packed)
HBM_GBS = 8000.0
TREE_LEVELS = (8, 9, 10)
CPU_SHARE = 16                 # host cores of one GPU's share of the host

# Algorithmic flops per unit (FMA = 2, other arithmetic = 1; a rint counts 1):
#   phase u l + v m + w (n-1): 1 mul + 2 FMA = 5; reduction rint + sub = 2;
#   phasor: r^2 1, sine polynomial 6 FMA + 1 mul = 13, cosine 6 FMA = 12,
#   4x identities 8 -> 34.  Per-term work after the phasor:
FLOPS = {
    "direct_fp64": 5 + 2 + 34 + 4,            # MAC: 2 FMA                      -> 45
    "adjoint": 5 + 2 + 34 + 8,                # complex MAC: 4 FMA               -> 49
    "grad": 5 + 2 + 34 + 6 + 1 + 6,           # z = conj(y) e; Re z; 3 FMA on Im z -> 54
    # Haar analysis of the plane wave and Eq. 17 (section 2.4): a node with k
    # children forms S and D^0..2 from k-1 complex additions each (the signs
    # +-1 are not arithmetic), then eta = S/4 (2), sigma^m = (sqrt(A_j)/4) D^m
    # (6) and gamma^m sigma^m into V (3 complex x real MACs, 12)
    "tree_leaf": 5 + 2 + 34,                  # eta_J at the leaf
    "tree_node": 2 + 6 + 12,                  # eta, sigma, gamma sigma
    "tree_child": 2 + 6,                      # every child after a node's first: S, D^0..2
    "tree_root": 4,                           # A_1 lambda_1 eta_1 into V
}
# Of those, the FP64 phasor polynomial (one implementation choice of a
# complex exponential; a hardware FP64 sincos would need none of them).
PHASOR_FLOPS = 34

# Algorithmic operations per term of the FP32-compensated forms, by the unit
# that executes them: the FP64 phase and its exact reduction to [0, 1) (1 mul,
# 2 FMA, fract); the conversion of r to FP32; the hardware sine and cosine; the
# FP32 side, where terms enter the Kahan sums in pairs -- direct: per re/im a
# pair's two FMAs (the products I c, less the compensation) and the 3
# additions of a Kahan step, 5 per pair; adjoint: per re/im a pair's four FMAs
# (conj(e) y of both rows, less the compensation) and the 3 additions, 7 per
# pair.
F32C_OPS = {
    "direct_f32c": {"f64": 4, "cvt": 1, "trans": 2, "f32": 5},
    "adjoint_f32c": {"f64": 4, "cvt": 1, "trans": 2, "f32": 7},
}


def tree_flops_per_row(st: dict) -> int:
    """Algorithmic flops per visibility row of the tree route over a tree with
    the given stats: every node but the level-1 ones is some node's child, and
    each internal node has one first child, so the sum over nodes of (k - 1)
    is leaves - roots."""
    roots = st["nodes_per_level"][0]
    return (st["n_leaves"] * FLOPS["tree_leaf"] + st["n_internal"] * FLOPS["tree_node"] +
            (st["n_leaves"] - roots) * FLOPS["tree_child"] + roots * FLOPS["tree_root"])


def precision_errors(low, ref, scale: float) -> dict:
    """A precision-form result against the FP64 form of the same call (device
    tensors): E_max = max |low - ref| / scale (scale the sum of |flux| or of
    |y|, as the tolerances are stated) and E_rms = ||low - ref|| / ||ref||."""
    import torch
    d = (low.to(torch.complex128) - ref).abs()
    nrm = float(ref.abs().square().sum().sqrt())
    return {"E_max_vs_fp64": float(f"{float(d.max()) / scale:.3e}"),
            "E_rms_vs_fp64": float(f"{float(d.square().sum().sqrt()) / nrm:.3e}") if nrm else 0.0}


def f32c_roofline(kind: str, terms_per_s: float, peaks: dict) -> dict:
    """Issue-time ceiling of an FP32-compensated kernel from the measured
    rates of the three units it uses: FP64 lane operations at half the FP64
    FMA flop rate, FP32 lane operations (conversion included) at half the FP32
    FMA flop rate, and transcendentals at twice the sine + cosine pair rate.
    If the units shared one issue port, a term would take at least the sum of
    the three times; `frac` is the achieved rate against that ceiling and
    `shares` each unit's busy fraction."""
    ops = F32C_OPS[kind]
    r64 = peaks["fp64_fma_tflops"] * 1e12 / 2
    r32 = peaks["fp32_fma_tflops"] * 1e12 / 2
    rtr = peaks["sincos_f32_gops"] * 1e9 * 2
    t_term = {"fp64": ops["f64"] / r64, "fp32": (ops["f32"] + ops["cvt"]) / r32,
              "trans": ops["trans"] / rtr}
    ceiling = 1.0 / sum(t_term.values())
    return {"bound": "alu", "unit": "Gterms/s", "achieved": round(terms_per_s / 1e9, 1),
            "peak": round(ceiling / 1e9, 1), "frac": round(terms_per_s / ceiling, 4),
            "shares": {k: round(terms_per_s * v, 4) for k, v in t_term.items()},
            "ops_per_term": ops,
            "peak_model": "1 / (n_f64 / R_f64 + n_f32 / R_f32 + n_trans / R_trans), "
                          "measured rates of this part (measured_peaks)"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--cpu-rows", type=int, default=32768,
                   help="rows of the workload the oracle is timed on")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-clean", action="store_true",
                   help="skip the clean-loop measurement after the step")
    p.add_argument("--batched", action="store_true",
                   help="time the 256-instance batched workload (1.29e9 rows) as captured "
                        "graphs of the batched plans, direct and tree routes, and exit")
    p.add_argument("--clean-only", action="store_true",
                   help="run only the clean loop on the seven-source workload (two calls) "
                        "and the predictor comparison, and print their JSON blocks")
    p.add_argument("--precision", action="store_true",
                   help="time the precision form on its own workload (cfg3: 8,355,840 rows "
                        "of 100 km baselines, 10,000 components, w-term active): FP64 and "
                        "FP32-compensated direct sums, speed-up, and the FP32 form's error "
                        "against the FP64 one on every row; print one JSON line and exit")
    p.add_argument("--profile", action="store_true",
                   help="short run for a profiler: no CPU baseline")
    p.add_argument("--tune", action="store_true",
                   help="run the autotuner (quick sweep) before the warmup instead of using "
                        "the library's default tile shapes")
    p.add_argument("--sweep", action="store_true",
                   help="instead of the step: the tree route's run-time sweep over J = 12..25 "
                        "and 10..140 distinct components on a one-hour, one-second 27-antenna "
                        "track (one JSON line per point, then a summary line)")
    p.add_argument("--tune-out", default=None,
                   help="write the autotuner's table and timings (JSON) to this path")
    p.add_argument("--copy-calibration", action="store_true",
                   help="also run one device copy of 1 GiB (HBM counter calibration)")
    p.add_argument("--threshold", action="store_true",
                   help="coefficient thresholding on the measured workload (cfg2, J = 10 and "
                        "the run-time sweep's track at J = 16): time and error against the "
                        "exact tree route for retained proportions 1 .. 0.005; print one "
                        "JSON line and exit")
    p.add_argument("--adjoint-shapes", action="store_true",
                   help="the adjoint on the step's rows and pixels (8,355,840 x 955) at "
                        "tile shapes 4x128, 4x256, 2x256 and 1x256 (pixels per lane x "
                        "threads): median time of seven launches each, one JSON line; for "
                        "a FETCH_SIZE counter pass per shape")
    p.add_argument("--no-cfg3", action="store_true",
                   help="skip the precision-form leg on its own workload (cfg3)")
    p.add_argument("--no-cfg4", action="store_true",
                   help="skip the batched leg on its own workload (cfg4)")
    return p.parse_args()


# ------------------------------------------------------------ CPU baseline --
def _cpu_worker(args):
    """Times the oracle on a slice of rows for every stage of the step."""
    rows, seed_inputs = args
    import numpy as np
    from oracle import sphere as sp
    from oracle import tree as ot
    from oracle import visibility as ov
    from synth import configs, models
    W = configs.CFG2
    u, v, w = W.track.uvw_rows(rows)
    l, m, f = W.components()
    rng = np.random.default_rng(seed_inputs)
    y = models.complex_noise(rows.size, 0.01, rng)
    pix, pl, pm, pn = sp.pixels_in_disk(9, W.ra_p, W.dec_p, math.radians(4.0))
    t0 = time.perf_counter()
    V = ov.predict_direct(u, v, w, l, m, f)           # FP64 form (and the FP32c reference)
    t_direct = time.perf_counter() - t0
    terms = 2 * rows.size * l.size
    t_trees = 0.0
    for J in TREE_LEVELS:
        t1 = time.perf_counter()
        T = ot.build_tree(J, W.ra_p, W.dec_p, l, m, f)
        ot.predict_tree(T, u, v, w)
        t_trees += time.perf_counter() - t1
        terms += rows.size * l.size
    t1 = time.perf_counter()
    r, _ = ov.residual_chi2(V + y, V, 1e4)
    ov.adjoint(u, v, w, r, pl, pm, pn)
    t_adj = time.perf_counter() - t1
    terms += rows.size * pix.size
    t1 = time.perf_counter()
    ov.grad_direct(u, v, w, r, l, m, f, alpha=-2e4)
    t_grad = time.perf_counter() - t1
    terms += rows.size * l.size
    return terms, 2 * t_direct + t_trees + t_adj + t_grad


def cpu_baseline(n_rows: int) -> dict:
    import multiprocessing as mp

    import numpy as np
    from synth import configs
    cores = min(CPU_SHARE, len(os.sched_getaffinity(0)))
    rows = configs.sample_rows(configs.CFG2.track.n_vis, n_rows, seed=2024, tile=0)
    rows = rows[:n_rows]
    parts = [p for p in np.array_split(rows, cores) if p.size]
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(len(parts)) as pool:
        res = pool.map(_cpu_worker, [(p, 99 + i) for i, p in enumerate(parts)])
    wall = time.perf_counter() - t0
    terms = sum(r[0] for r in res)
    cpu_s = sum(r[1] for r in res)
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    busy = max(r[1] for r in res)
    return {
        "value": terms / busy / 1e9,
        "unit": UNIT,
        "cores": len(parts),
        "kind": "oracle",
        "sample": (f"{rows.size} seeded rows of the 8,355,840-row workload, every stage of the "
                   f"step (direct sum twice: FP64 reference of both forms), split over "
                   f"{len(parts)} worker processes, 1 thread each"),
        "per_core_value": terms / cpu_s / 1e9,
        "cpu_seconds": cpu_s,
        "wall_seconds_incl_spawn": wall,
        "cpu_model": model,
    }


# ------------------------------------------------------------------ GPU --
def _code_tokens(text: str) -> str:
    """C/C++ source without its comments and with runs of whitespace folded
    to one space: what the compiler sees of it."""
    out, i, n = [], 0, len(text)
    while i < n:
        ch = text[i]
        if ch in "\"'":                                  # string or character literal
            j = i + 1
            while j < n and text[j] != ch:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            out.append(" ")
            i = n if j < 0 else j + 2
        else:
            out.append(ch)
            i += 1
    return re.sub(r"\s+", " ", "".join(out)).strip()


def source_digest(kernel_file: str, csrc: str | None = None) -> str:
    """SHA-256 (16 hex digits) of a kernel source together with every local
    header it includes, directly or through other headers, comments left out,
    so that a change to the code of any of them marks recorded counters as
    stale."""
    csrc = csrc or os.path.join(ROOT, "paper_1909_03956_amd", "csrc")
    seen, todo = [], [kernel_file]
    while todo:
        name = todo.pop(0)
        if name in seen or not os.path.exists(os.path.join(csrc, name)):
            continue
        seen.append(name)
        with open(os.path.join(csrc, name)) as fh:
            todo += re.findall(r'^\s*#include\s+"([^"]+)"', fh.read(), re.M)
    h = hashlib.sha256()
    for name in [seen[0]] + sorted(seen[1:]):
        with open(os.path.join(csrc, name)) as fh:
            h.update(name.encode() + b"\0" + _code_tokens(fh.read()).encode())
    return h.hexdigest()[:16]


def traffic_for(kernel_file: str, per_launch_key: str, path: str | None = None,
                csrc: str | None = None):
    """HBM bytes per launch from the committed counter summary, or None if the
    kernel source changed since the counters were taken."""
    path = path or os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh).get(per_launch_key)
    if not rec:
        return None
    if rec.get("source_sha") != source_digest(kernel_file, csrc):
        return None
    return rec.get("bytes_per_launch")


def valu_count_for(kernel_file: str, key: str, path: str | None = None,
                   csrc: str | None = None):
    """VALU wave instructions per launch from the committed counter summary,
    or None if the kernel source changed since the counters were taken."""
    path = path or os.path.join(ROOT, "profiles", "valu_issue.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh).get(key)
    if not rec or rec.get("source_sha") != source_digest(kernel_file, csrc):
        return None
    return rec.get("valu_wave_instructions")


def run_sweep():
    """Time per visibility of the tree route (host build excluded, reported
    apart) against J and against the number of distinct components, the two
    axes of the paper's run-time scaling figure (section 3.6.1)."""
    import numpy as np
    import torch

    import paper_1909_03956_amd as swv
    from synth import configs

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    T = configs.SWEEP_TRACK
    u, v, w = (torch.as_tensor(a, device=dev) for a in T.uvw())
    ra, dec = math.radians(T.ra_deg), math.radians(T.dec_deg)
    n = u.numel()
    out = torch.empty(n, dtype=torch.complex128, device=dev)
    ctx = swv.context(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def point(J, n_comp):
        l, m, f = configs.sweep_components(n_comp)
        t = swv.Tree(J, ra, dec, l, m, f)
        st = t.stats()
        t.predict(u, v, w, out=out)
        ctx.synchronize()
        times = []
        for _ in range(5):
            e0.record()
            t.predict(u, v, w, out=out)
            e1.record()
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
        ms = float(np.median(times))
        rec = {"sweep": True, "J": J, "n_comp": n_comp, "distinct": st["n_leaves"],
               "internal_nodes": st["n_internal"], "max_branching": st["max_branching"],
               "n_vis": n, "ms": round(ms, 4), "ns_per_vis": round(ms * 1e6 / n, 3),
               "Gvis_terms_per_s": round(n * n_comp / (ms * 1e-3) / 1e9, 2),
               "Gvis_nodes_per_s": round(n * (st["n_leaves"] + st["n_internal"]) /
                                         (ms * 1e-3) / 1e9, 2),
               "host_build_ms": round(1e3 * st["build_seconds"], 3)}
        t.close()
        print(json.dumps(rec), flush=True)
        return rec

    by_j = {nc: [point(J, nc) for J in range(12, 26)] for nc in (15, 140)}
    by_n = {J: [point(J, nc) for nc in range(10, 141, 10)] for J in (12, 15, 25)}

    def growth(recs):   # least-squares exp fit: time ~ g^J
        J = np.array([r["J"] for r in recs], float)
        y = np.log([r["ms"] for r in recs])
        return float(np.exp(np.polyfit(J, y, 1)[0]))

    def linearity(recs):   # time against distinct components: slope, intercept, R^2
        x = np.array([r["distinct"] for r in recs], float)
        y = np.array([r["ms"] for r in recs], float)
        a, b = np.polyfit(x, y, 1)
        r2 = 1 - np.sum((y - (a * x + b)) ** 2) / np.sum((y - y.mean()) ** 2)
        return {"ms_per_distinct": round(float(a), 5), "ms_at_zero": round(float(b), 4),
                "r2": round(float(r2), 5)}

    j20 = {nc: next(r for r in by_j[nc] if r["J"] == 20) for nc in by_j}
    print(json.dumps({
        "sweep_summary": True, "track": "27 antennas, 1 h at 1 s, 1,263,600 rows",
        "growth_per_level": {str(nc): round(growth(by_j[nc]), 4) for nc in by_j},
        "paper_growth_per_level": 1.07,
        "time_vs_distinct": {str(J): linearity(by_n[J]) for J in by_n},
        "J20_ms": {str(nc): j20[nc]["ms"] for nc in j20},
        "paper_J20_s_per_major_cycle": {"140": 1000, "15": 146},
    }), flush=True)


def run_clean(swv, torch, np, dev, configs):
    """The wavelet clean loop on the seven-source wide-field workload (outside
    the step): dirty beam, dirty image, then major cycles of 300 Hogbom
    iterations, tree prediction and residual image, as per-stage device times."""
    S = configs.CLEAN7

    def D(x):
        return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)

    u, v, w = S.track.uvw()
    l, m, f = S.sources()
    U, V, Wt = D(u), D(v), D(w)
    vis = swv.predict_direct(U, V, Wt, D(l), D(m), D(f))
    vis += torch.as_tensor(S.noise(), dtype=torch.complex128, device=dev)
    n = S.n_pix
    args = (U, V, Wt, vis, n, n, S.cell, S.J, S.ra_p, S.dec_p, S.gain, 0.0, S.minor_iter,
            S.n_major)
    swv.wavelet_clean(*args)          # first call: scratch allocation, code upload
    t0 = time.perf_counter()
    out = swv.wavelet_clean(*args)
    wall = 1e3 * (time.perf_counter() - t0)
    # the same loop as conventional (FFT + degridding, W = 10) and exact (direct) clean
    others = {}
    for pred in ("degrid", "direct"):
        swv.wavelet_clean(*args, predictor=pred, support=10)   # FFT plan, code upload
        o = swv.wavelet_clean(*args, predictor=pred, support=10)
        others[pred] = {"chi2": [round(c["chi2"], 4) for c in o["cycles"]],
                        "ms_predict": [round(c["ms_predict"], 4) for c in o["cycles"]],
                        "model_pixels": [c["leaves"] for c in o["cycles"]],
                        "residual_rms": float(f"{float(o['residual'].std()):.6g}")}
    # the wavelet clean with FP32-compensated images (beam and residual images)
    t0 = time.perf_counter()
    o = swv.wavelet_clean(*args, image_prec="f32c")
    others["tree_f32c_images"] = {
        "wall_ms": round(1e3 * (time.perf_counter() - t0), 2),
        "beam_ms": round(o["ms_beam"], 3),
        "ms_image": [round(c["ms_image"], 4) for c in o["cycles"]],
        "chi2": [round(c["chi2"], 4) for c in o["cycles"]],
        "residual_rms": float(f"{float(o['residual'].std()):.6g}")}
    cyc = out["cycles"]
    iters = sum(c["found"] for c in cyc)
    ms_minor = sum(c["ms_minor"] for c in cyc)
    ms_image = [c["ms_image"] for c in cyc]
    n_vis = u.size
    return {
        "workload": "clean7: 27-antenna 1.7 km array, 10 MHz, dec +45, 2,016 s at 1 s "
                    "(707,616 vis); seven 1 Jy sources; 256 x 256 image over 42 deg 40'; "
                    f"J={S.J}; gain {S.gain}; {S.n_major} major cycles of {S.minor_iter} "
                    "Hogbom iterations",
        "n_vis": n_vis, "n_pix": n * n, "wall_ms": round(wall, 2),
        "beam_ms": round(out["ms_beam"], 3), "dirty_image_ms": round(out["ms_dirty"], 3),
        "cycles": [{k: (round(c[k], 4) if isinstance(c[k], float) else c[k]) for k in c}
                   for c in cyc],
        "components": int(out["pix"].size), "flux_found": round(float(out["val"].sum()), 4),
        "hogbom_us_per_iter": round(1e3 * ms_minor / max(iters, 1), 3),
        # image read + write and beam read per pixel and iteration
        "hogbom_GB_per_s": round(24 * n * n * iters / (ms_minor * 1e-3) / 1e9, 1),
        "residual_image_Gterms_per_s": round(n_vis * n * n / (float(np.median(ms_image)) * 1e-3)
                                             / 1e9, 1),
        "beam_Gterms_per_s": round(n_vis * (2 * n - 1) ** 2 / (out["ms_beam"] * 1e-3) / 1e9, 1),
        "residual_rms": float(f"{float(out['residual'].std()):.6g}"),
        "same_loop_other_predictors": others,
    }


def run_compare(swv, torch, np, dev, configs):
    """Accuracy against speed of the predictors on the clean7 track and grid
    (outside the step): 140 components on image pixels; the direct sum over
    them is the reference; the tree route at several J (error = the snapping
    of components to level-J pixel centres) and the FFT + degridding predictor
    at several kernel widths W (error = the kernel's aliasing)."""
    S = configs.CLEAN7

    def D(x):
        return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)

    u, v, w = S.track.uvw()
    U, V, Wt = D(u), D(v), D(w)
    n = S.n_pix
    pix, flux = configs.clean7_grid_model()
    gl, gm, gn = (t.cpu().numpy() for t in swv.image_grid(n, n, S.cell, device=dev))
    l, m = gl[pix], gm[pix]
    img = np.zeros(n * n)
    img[pix] = flux
    IMG = D(img.reshape(n, n))
    scale = float(np.abs(flux).sum())

    def timed(fn, reps=3):
        fn()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    ref = torch.empty(u.size, dtype=torch.complex128, device=dev)
    L, M, F = D(l), D(m), D(flux)
    ms_direct = timed(lambda: swv.predict_direct(U, V, Wt, L, M, F, out=ref))
    out = {"workload": f"clean7 track (707,616 vis) and 256 x 256 grid; {pix.size} components "
                       "on image pixels within 30 deg; reference: the direct sum",
           "comparator": "FFT + degridding as a type-2 non-uniform FFT in (u, v, w): "
                         "exponential-of-semicircle kernel over W cells, w planes interpolated "
                         "(improved w-stacking), not the w-kernel convolution of Eq. 3",
           "direct": {"ms": round(ms_direct, 4)}}
    buf = torch.empty_like(ref)
    for J in (11, 16, 20, 25):
        T = swv.Tree(J, S.ra_p, S.dec_p, l, m, flux)
        ms = timed(lambda: T.predict(U, V, Wt, out=buf))
        err = float((buf - ref).abs().max()) / scale
        out[f"tree_J{J}"] = {"ms": round(ms, 4), "E_max": float(f"{err:.3e}"),
                             "leaves": T.stats()["n_leaves"]}
        T.close()
    for W in (6, 10, 14):
        st = {}

        def call():
            _, s2 = swv.predict_degrid(IMG, U, V, Wt, S.cell, W, out=buf)
            st.update(s2)
        ms = timed(call)
        err = float((buf - ref).abs().max()) / scale
        out[f"degrid_W{W}"] = {"ms": round(ms, 4), "E_max": float(f"{err:.3e}"),
                               "w_planes": st["n_planes"]}
    return out


def run_precision(swv, torch, np, dev, configs, peaks=None):
    """The precision form (FP64 phase and reduction, FP32 phasor and products,
    Kahan-compensated FP32 sums) against the FP64 form on cfg3, the workload
    named for it: both timed as single launches (median of five after a
    warm-up), and the FP32 form's error against the FP64 one on every row,
    relative to the summed flux (its bound against the oracle is a test)."""
    W = configs.CFG3

    def D(x):
        return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)

    t_in = time.perf_counter()
    u, v, w = W.track.uvw()
    l, m, f = W.components()
    U, V, Wt, L, M, F = D(u), D(v), D(w), D(l), D(m), D(f)
    n_vis, n_comp = u.size, l.size
    v64 = torch.empty(n_vis, dtype=torch.complex128, device=dev)
    v32 = torch.empty(n_vis, dtype=torch.complex64, device=dev)
    torch.cuda.synchronize()
    log(f"cfg3 inputs ready in {time.perf_counter() - t_in:.1f} s: {n_vis} rows, "
        f"{n_comp} components")

    def timed(fn, reps=5):
        fn()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    ms64 = timed(lambda: swv.predict_direct(U, V, Wt, L, M, F, out=v64))
    ms32 = timed(lambda: swv.predict_direct(U, V, Wt, L, M, F, prec="f32c", out=v32))
    err = (v32.to(torch.complex128) - v64).abs()
    scale = float(np.abs(f).sum())
    terms = n_vis * n_comp
    phi = float(torch.max(torch.abs(U) + torch.abs(V) + torch.abs(Wt)).item())
    if peaks is None:
        peaks = swv.context(dev).measure_peaks()
    fl64 = terms * FLOPS["direct_fp64"]
    ach64 = fl64 / (ms64 * 1e-3) / 1e12
    out = {"workload": "cfg3: 256-antenna 100 km array, 8 h at dec +30, 1.4 GHz, "
                       f"{n_vis:,} vis; {n_comp:,} components uniform over 3 deg",
           "n_vis": n_vis, "n_comp": n_comp, "terms": terms,
           "max_abs_uvw_sum_wavelengths": round(phi, 1),
           "fp64": {"ms": round(ms64, 3),
                    "Gvis_terms_per_s": round(terms / (ms64 * 1e-3) / 1e9, 1),
                    "roofline": {"bound": "alu", "kernel": "k_direct_f64",
                                 "achieved": round(ach64, 2), "peak": PEAK_FP64_TFLOPS,
                                 "unit": "TFLOP/s", "frac": round(ach64 / PEAK_FP64_TFLOPS, 4),
                                 "flops_per_launch": fl64, "avg_launch_ms": round(ms64, 4),
                                 "frac_excl_phasor": round(
                                     ach64 * (FLOPS["direct_fp64"] - PHASOR_FLOPS) /
                                     FLOPS["direct_fp64"] / PEAK_FP64_TFLOPS, 4),
                                 "measured_peak": round(peaks["fp64_fma_tflops"], 2),
                                 "frac_of_measured": round(ach64 / peaks["fp64_fma_tflops"], 4),
                                 "traffic": None}},
           "f32c": {"ms": round(ms32, 3),
                    "Gvis_terms_per_s": round(terms / (ms32 * 1e-3) / 1e9, 1),
                    "roofline": dict(f32c_roofline("direct_f32c", terms / (ms32 * 1e-3), peaks),
                                     kernel="k_direct_f32c", avg_launch_ms=round(ms32, 4),
                                     traffic=None)},
           "speedup_f32c_over_fp64": round(ms64 / ms32, 3),
           "f32c_vs_fp64": {"E_max": float(f"{float(err.max()) / scale:.3e}"),
                            "E_rms": float(f"{float(err.pow(2).mean().sqrt()) / scale:.3e}"),
                            "relative_to": "sum |I_k|, every row"}}
    log(f"cfg3 direct: FP64 {ms64:.2f} ms, F32C {ms32:.2f} ms "
        f"({out['speedup_f32c_over_fp64']}x), E_max {out['f32c_vs_fp64']['E_max']}")
    return out


def run_adjoint_shapes(swv, torch, np, dev, configs, models):
    """The adjoint of the step (cfg2 rows, the J = 9 pixels within 4 deg) at
    several tile shapes, each set in the tuning table of the device's context
    (the large-row class of the adjoint family), which is left at the default
    shape afterwards."""
    W = configs.CFG2

    def D(x):
        return torch.as_tensor(np.ascontiguousarray(x), device=dev)

    u, v, w = (D(a) for a in W.track.uvw())
    y = D(models.complex_noise(u.numel(), configs.CFG5_NOISE_SIGMA,
                               np.random.default_rng(configs.CFG5_SEED_NOISE)))
    _, pl, pm, pn = swv.pixels_in_disk(9, W.ra_p, W.dec_p, math.radians(4.0))
    L, M, N = D(pl), D(pm), D(pn)
    ctx = swv.context(dev)
    from paper_1909_03956_amd._lib import FAM_ADJOINT as fam_adjoint
    large = 1   # size class of 2^20 rows or more
    out = []
    for ppl, block in ((4, 128), (4, 256), (2, 256), (1, 256)):
        ctx.tune_set(fam_adjoint, large, ppl, block)
        img = swv.adjoint(u, v, w, y, L, M, N)
        torch.cuda.synchronize()
        times = []
        for _ in range(7):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            img = swv.adjoint(u, v, w, y, L, M, N)
            e1.record()
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
        out.append({"pixels_per_lane": ppl, "block": block,
                    "tiles": -(-pl.size // (ppl * block)),
                    "ms": round(float(np.median(times)), 4)})
        log(f"adjoint {ppl} x {block}: {out[-1]['ms']} ms")
    ctx.tune_set(fam_adjoint, large, 4, 256)
    return {"workload": f"cfg2 rows ({u.numel():,}) x {pl.size} pixels (J = 9 within 4 deg)",
            "shapes": out}


def run_threshold(swv, torch, np, dev, configs):
    """Retained proportion against time and error (the thresholded variant of
    section 1): each thresholded tree is timed as single launches (median of
    five after a warm-up) and compared with the exact tree route on every row;
    E_max = max |V_p - V| / sum |I|."""
    def D(x):
        return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)

    def timed(fn, reps=5):
        fn()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    cases = []
    W = configs.CFG2
    l, m, f = W.components()
    cases.append(("cfg2 (8,355,840 vis, 2,000 components), J = 10", W.track.uvw(), W.ra_p,
                  W.dec_p, 10, l, m, f))
    T = configs.SWEEP_TRACK
    ls, ms, fs = configs.sweep_components(140)
    cases.append(("run-time sweep track (1,263,600 vis, 140 components), J = 16", T.uvw(),
                  math.radians(T.ra_deg), math.radians(T.dec_deg), 16, ls, ms, fs))
    out = []
    for name, (u, v, w), ra, dec, J, l, m, f in cases:
        U, V, Wt = D(u), D(v), D(w)
        t = swv.Tree(J, ra, dec, l, m, f)
        exact = torch.empty(U.numel(), dtype=torch.complex128, device=dev)
        ms_exact = timed(lambda: t.predict(U, V, Wt, out=exact))
        buf = torch.empty_like(exact)
        ms_leaf = timed(lambda: t.predict_leaves(U, V, Wt, out=buf))
        scale = float(np.abs(f).sum())
        st = t.stats()
        rows = []
        for frac in (1.0, 0.5, 0.2, 0.1, 0.05, 0.02, 0.01, 0.005):
            tp = t.threshold(frac)
            ms = timed(lambda: tp.predict(U, V, Wt, out=buf))
            err = float((buf - exact).abs().max()) / scale
            sp_ = tp.stats()
            kept, n_coeffs = tp.kept()
            rows.append({"fraction": frac, "kept": int(kept.size), "leaves": sp_["n_leaves"],
                         "internal": sp_["n_internal"], "records": sp_["n_records"],
                         "ms": round(ms, 4), "speedup": round(ms_exact / ms, 3),
                         "E_max": float(f"{err:.3e}")})
            log(f"threshold {name}: keep {frac} -> {ms:.3f} ms, E_max {err:.2e}")
            tp.close()
        out.append({"workload": name, "J": J, "leaves": st["n_leaves"],
                    "internal": st["n_internal"], "coefficients": 3 * st["n_internal"],
                    "exact_ms": round(ms_exact, 4), "leaf_sum_ms": round(ms_leaf, 4),
                    "rows": rows})
        t.close()
    return out


def run_batched(swv, torch, np, dev, configs, peaks=None):
    """The batched workload: 64 channels x 4 pointings of the 256-antenna array,
    2M-8M unflagged rows each (1.29e9 in all), made on the device; one plan per
    route and precision (direct and tree, FP64 and FP32-compensated) over all
    256 instances, captured as a graph; each graph launched once warm and then
    timed three times."""
    B = configs.BatchedWorkload()
    ra, dec = configs.CFG2.ra_p, configs.CFG2.dec_p

    def D(x):
        return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)

    insts = {"direct": [], "direct_f32c": [], "tree": [], "tree_f32c": []}
    fluxsum = []
    keep = []
    rows = terms = leaves = tree_fl = 0
    t0 = time.perf_counter()
    for inst in B.instances:
        kept, l, m, f = B.instance_rows_kept(inst)
        u, v, w = B.instance_uvw_torch(inst, kept, dev)
        out_d = torch.empty(kept.size, dtype=torch.complex128, device=dev)
        out_t = torch.empty(kept.size, dtype=torch.complex128, device=dev)
        out_s = torch.empty(kept.size, dtype=torch.complex64, device=dev)
        out_ts = torch.empty(kept.size, dtype=torch.complex64, device=dev)
        tree = swv.Tree(inst.J, ra, dec, l, m, f)
        Ld, Md, Fd = D(l), D(m), D(f)
        insts["direct"].append(dict(route="direct", u=u, v=v, w=w, l=Ld, m=Md, flux=Fd,
                                    out=out_d))
        insts["direct_f32c"].append(dict(route="direct", prec="f32c", u=u, v=v, w=w, l=Ld,
                                         m=Md, flux=Fd, out=out_s))
        fluxsum.append(float(np.abs(f).sum()))
        insts["tree"].append(dict(route="tree", tree=tree, u=u, v=v, w=w, out=out_t))
        insts["tree_f32c"].append(dict(route="tree", prec="f32c", tree=tree, u=u, v=v, w=w,
                                       out=out_ts))
        keep.append(tree)
        st = tree.stats()
        rows += kept.size
        terms += kept.size * inst.n_comp
        leaves += kept.size * (st["n_leaves"] + st["n_internal"])
        tree_fl += kept.size * tree_flops_per_row(st)
    torch.cuda.synchronize()
    log(f"batched workload made in {time.perf_counter() - t0:.1f} s: {len(B.instances)} "
        f"instances, {rows} rows")
    out = {"workload": "cfg4: 64 channels (0.95-1.75 GHz) x 4 pointings of the 256-antenna "
                       "20 km array, 2M-8M unflagged rows per instance, N_C 100-20,000, J 7-10",
           "instances": len(B.instances), "rows": rows, "terms": terms,
           "tree_nodes_x_rows": leaves}
    for name in ("direct", "direct_f32c", "tree", "tree_f32c"):
        plan = swv.BatchPlan(insts[name])
        graph = plan.capture()
        graph.launch()
        torch.cuda.synchronize()
        ts = []
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            graph.launch()
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        ms = float(np.median(ts))
        if name.endswith("_f32c"):
            # the precision form: its speed-up and its error against the FP64
            # plan's visibilities, instance by instance; the direct sum also
            # against its own three-unit ceiling
            base = name[:-len("_f32c")]
            e_max = max(float((d32["out"].to(torch.complex128) - d64["out"]).abs().max()) / fs
                        for d32, d64, fs in zip(insts[name], insts[base], fluxsum))
            out[name] = {"ms": round(ms, 2),
                         "Gvis_terms_per_s": round(terms / (ms * 1e-3) / 1e9, 1),
                         "speedup_over_fp64": round(out[base]["ms"] / ms, 3),
                         "E_max_vs_fp64": float(f"{e_max:.3e}")}
            if base == "direct" and peaks:
                out[name]["roofline"] = dict(
                    f32c_roofline("direct_f32c", terms / (ms * 1e-3), peaks),
                    kernel="k_batch_direct (SWV_F32C)")
            log(f"batched {name}: {ms:.1f} ms")
            graph.close()
            plan.close()
            continue
        fl = terms * FLOPS["direct_fp64"] if name == "direct" else tree_fl
        ach = fl / (ms * 1e-3) / 1e12
        out[name] = {"ms": round(ms, 2), "Gvis_terms_per_s": round(terms / (ms * 1e-3) / 1e9, 1),
                     "Grows_per_s": round(rows / (ms * 1e-3) / 1e9, 3), "plan": plan.stats(),
                     "roofline": {"bound": "alu",
                                  "kernel": "k_batch_direct" if name == "direct" else "k_batch_tree",
                                  "achieved": round(ach, 2), "peak": PEAK_FP64_TFLOPS,
                                  "unit": "TFLOP/s", "frac": round(ach / PEAK_FP64_TFLOPS, 4),
                                  "flops_per_launch": fl, "avg_launch_ms": round(ms, 3),
                                  "traffic": None}}
        log(f"batched {name}: {ms:.1f} ms")
        graph.close()
        plan.close()
    # one major cycle of the tree route over every instance: the batched
    # prediction, then per instance the residual against the direct route's
    # visibilities (the snapping error), chi^2 and the residual image on the
    # level-9 pixels within 4 deg; eager launches against the captured graph
    pix = swv.pixels_in_disk(9, ra, dec, math.radians(4.0))[1:]
    P = tuple(D(a) for a in pix)
    cyc = [dict(route="tree", u=d["u"], v=d["v"], w=d["w"], vis_obs=dd["out"], inv_sigma2=1e4,
                pixels=P, comp_cap=max(1, t.stats()["n_leaves"]), tree_level_cap=10)
           for d, dd, t in zip(insts["tree"], insts["direct"], keep)]
    cy = swv.MajorCycle(cyc)
    for k, t in enumerate(keep):
        cy.set_tree(k, t)

    def timed_cycle(fn, reps=2):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))
    ms_eager = timed_cycle(cy.run)
    cy.capture()
    ms_graph = timed_cycle(cy.launch)
    chi2 = float(sum(float(o["chi2"].item()) for o in cy.out))
    out["major_cycle_tree"] = {
        "steps": "batched tree prediction; per instance residual vs the direct route, chi^2, "
                 f"residual image on {pix[0].size} level-9 pixels",
        "kernel_launches": 2 + 4 * len(cyc), "eager_ms": round(ms_eager, 2),
        "graph_ms": round(ms_graph, 2), "graph_speedup": round(ms_eager / ms_graph, 4),
        "chi2_sum": float(f"{chi2:.6g}")}
    log(f"major cycle (tree, 256 instances): eager {ms_eager:.1f} ms, graph {ms_graph:.1f} ms")
    cy.close()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path (--gpus "
              f"{args.gpus} requested); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.sweep:
        run_sweep()
        return

    import numpy as np
    import torch

    import paper_1909_03956_amd as swv
    from synth import configs, models

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.batched:
        print(json.dumps({"batched": run_batched(swv, torch, np, dev, configs,
                                                 swv.context(dev).measure_peaks())}), flush=True)
        return
    if args.precision:
        print(json.dumps({"precision": run_precision(swv, torch, np, dev, configs)}),
              flush=True)
        return
    if args.threshold:
        print(json.dumps({"threshold": run_threshold(swv, torch, np, dev, configs)}),
              flush=True)
        return
    if args.adjoint_shapes:
        print(json.dumps({"adjoint_shapes": run_adjoint_shapes(swv, torch, np, dev, configs,
                                                                models)}), flush=True)
        return
    if args.clean_only:
        print(json.dumps({"clean_loop": run_clean(swv, torch, np, dev, configs),
                          "predictor_comparison": run_compare(swv, torch, np, dev, configs)}),
              flush=True)
        return
    W = configs.CFG2
    t_in = time.perf_counter()
    u, v, w = W.track.uvw()
    l, m, f = W.components()
    n_vis, n_comp = u.size, l.size

    def D(x):
        return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)

    U, V, Wt = D(u), D(v), D(w)
    L, M, F = D(l), D(m), D(f)
    pix, pl, pm, pn = swv.pixels_in_disk(9, W.ra_p, W.dec_p, math.radians(4.0))
    PL, PM, PN = D(pl), D(pm), D(pn)
    n_pix = pix.size
    rng = np.random.default_rng(configs.CFG5_SEED_PERTURB)
    l2, m2, f2 = models.perturb_model(l, m, f, rng)
    noise = models.complex_noise(n_vis, configs.CFG5_NOISE_SIGMA,
                                 np.random.default_rng(configs.CFG5_SEED_NOISE))
    v_obs = swv.predict_direct(U, V, Wt, D(l2), D(m2), D(f2))
    v_obs += torch.as_tensor(noise, dtype=torch.complex128, device=dev)
    inv_s2 = 1.0 / configs.CFG5_NOISE_SIGMA ** 2
    v64 = torch.empty(n_vis, dtype=torch.complex128, device=dev)
    v32 = torch.empty(n_vis, dtype=torch.complex64, device=dev)
    vt = {J: torch.empty(n_vis, dtype=torch.complex128, device=dev) for J in TREE_LEVELS}
    resid = torch.empty(n_vis, dtype=torch.complex128, device=dev)
    torch.cuda.synchronize()
    log(f"inputs ready in {time.perf_counter() - t_in:.1f} s: {n_vis} rows, {n_comp} "
        f"components, {n_pix} pixels")
    ctx = swv.context(dev)
    families = ("direct_fp64", "direct_f32c", "tree", "adjoint", "grad")
    if args.tune:
        t_tune = time.perf_counter()
        ctx.autotune(cache_path=args.tune_out, quick=True)   # untimed: picks the tile shapes
        log(f"autotuned in {time.perf_counter() - t_tune:.2f} s")
    tuning = {f: ctx.tune_get(i, 1) for i, f in enumerate(families)}
    t_pk = time.perf_counter()
    peaks = ctx.measure_peaks()                   # untimed: measured FP64 ceiling
    log(f"measured peaks in {time.perf_counter() - t_pk:.2f} s: "
        + ", ".join(f"{k} {v:.1f}" for k, v in peaks.items()))

    stages = ["direct_fp64", "direct_f32c"] + [f"tree_J{J}" for J in TREE_LEVELS] + \
        ["residual", "adjoint", "grad"]
    keep_trees = []
    tree_stats = {}

    def step(events):
        def mark(name):
            e = torch.cuda.Event(enable_timing=True)
            e.record()
            events.append((name, e))
        mark("start")
        swv.predict_direct(U, V, Wt, L, M, F, out=v64)
        mark("direct_fp64")
        swv.predict_direct(U, V, Wt, L, M, F, prec="f32c", out=v32)
        mark("direct_f32c")
        for J in TREE_LEVELS:
            T = swv.Tree(J, W.ra_p, W.dec_p, l, m, f)     # host build, once per major cycle
            keep_trees.append(T)
            tree_stats[J] = T.stats()
            T.predict(U, V, Wt, out=vt[J])
            mark(f"tree_J{J}")
        r, chi2 = swv.residual_chi2(v_obs, v64, inv_s2, out=resid)
        mark("residual")
        img = swv.adjoint(U, V, Wt, r, PL, PM, PN)
        mark("adjoint")
        g = swv.grad_direct(U, V, Wt, r, L, M, F, alpha=-2.0 * inv_s2)
        mark("grad")
        return chi2, img, g

    for _ in range(args.warmup):
        step([])
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps)")

    all_events = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ev = []
        step(ev)
        all_events.append(ev)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    swv.synchronize()
    ms_per_step = 1e3 * wall / args.steps
    log(f"timed {args.steps} steps: {ms_per_step:.2f} ms/step")

    # outside the step: the tree route's precision form (FP32 leaf phasors)
    extra_routes = {}
    Tx = swv.Tree(max(TREE_LEVELS), W.ra_p, W.dec_p, l, m, f)
    vx = torch.empty(n_vis, dtype=torch.complex64, device=dev)
    for prec, key in (("fp64", f"tree_J{max(TREE_LEVELS)}_fp64"),
                      ("f32c", f"tree_J{max(TREE_LEVELS)}_f32c")):
        out_x = vx if prec == "f32c" else vt[max(TREE_LEVELS)]
        Tx.predict(U, V, Wt, prec=prec, out=out_x)
        times = []
        for _ in range(max(3, args.steps // 2)):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            Tx.predict(U, V, Wt, prec=prec, out=out_x)
            e1.record()
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
        ms = float(np.median(times))
        extra_routes[key] = {"ms": round(ms, 4),
                             "Gvis_terms_per_s": round(n_vis * n_comp / (ms * 1e-3) / 1e9, 2)}
    extra_routes["tree_speedup_f32c_over_fp64"] = round(
        extra_routes[f"tree_J{max(TREE_LEVELS)}_fp64"]["ms"] /
        extra_routes[f"tree_J{max(TREE_LEVELS)}_f32c"]["ms"], 3)
    extra_routes[f"tree_J{max(TREE_LEVELS)}_f32c"].update(
        precision_errors(vx, vt[max(TREE_LEVELS)], float(np.abs(f).sum())))
    # Eq. 16: the same model visibilities as the direct sum over the tree's
    # merged leaves at their pixel centres (swv_predict_tree_leaves)
    n_leaves = Tx.stats()["n_leaves"]
    out_l = torch.empty(n_vis, dtype=torch.complex128, device=dev)
    Tx.predict_leaves(U, V, Wt, out=out_l)
    times = []
    for _ in range(max(3, args.steps // 2)):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        Tx.predict_leaves(U, V, Wt, out=out_l)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    ms = float(np.median(times))
    diff = float((out_l - vt[max(TREE_LEVELS)]).abs().max()) / float(np.abs(f).sum())
    extra_routes[f"tree_J{max(TREE_LEVELS)}_as_leaf_sum"] = {
        "ms": round(ms, 4), "leaves": int(n_leaves),
        "Gvis_terms_per_s": round(n_vis * n_comp / (ms * 1e-3) / 1e9, 2),
        "max_diff_vs_tree": float(f"{diff:.3e}")}
    Tx.close()
    # the adjoint's precision form on the step's residual (FP32 phasors,
    # products and Kahan sums; complex128 image)
    r_, _ = swv.residual_chi2(v_obs, v64, inv_s2, out=resid)
    img64 = swv.adjoint(U, V, Wt, r_, PL, PM, PN)
    img32 = swv.adjoint(U, V, Wt, r_, PL, PM, PN, prec="f32c")
    times = []
    for _ in range(max(3, args.steps // 2)):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        swv.adjoint(U, V, Wt, r_, PL, PM, PN, prec="f32c")
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    ms = float(np.median(times))
    extra_routes["adjoint_f32c"] = {
        "ms": round(ms, 4), "Gvis_terms_per_s": round(n_vis * n_pix / (ms * 1e-3) / 1e9, 2),
        "roofline": dict(f32c_roofline("adjoint_f32c", n_vis * n_pix / (ms * 1e-3), peaks),
                         kernel="k_adjoint (SWV_F32C)"),
        **precision_errors(img32, img64, float(r_.abs().sum()))}

    # per-stage device times (median over steps)
    per = {s: [] for s in stages}
    for ev in all_events:
        for (a, ea), (b, eb) in zip(ev[:-1], ev[1:]):
            per[b].append(ea.elapsed_time(eb))
    med = {s: float(np.median(per[s])) for s in stages}
    terms = {"direct_fp64": n_vis * n_comp, "direct_f32c": n_vis * n_comp,
             "residual": 0, "adjoint": n_vis * n_pix, "grad": n_vis * n_comp}
    for J in TREE_LEVELS:
        terms[f"tree_J{J}"] = n_vis * n_comp
    step_terms = sum(terms.values())
    value = step_terms / (ms_per_step * 1e-3) / 1e9

    routes = {}
    for s in stages:
        r = {"ms": round(med[s], 4)}
        if terms[s]:
            r["Gvis_terms_per_s"] = round(terms[s] / (med[s] * 1e-3) / 1e9, 2)
        routes[s] = r
    for J in TREE_LEVELS:
        st = tree_stats[J]
        routes[f"tree_J{J}"].update({"leaves": st["n_leaves"], "internal_nodes": st["n_internal"],
                                     "host_build_ms": round(1e3 * st["build_seconds"], 3),
                                     "Gvis_nodes_per_s": round(
                                         n_vis * (st["n_leaves"] + st["n_internal"]) /
                                         (med[f"tree_J{J}"] * 1e-3) / 1e9, 2)})
    routes["residual"]["GB_per_s"] = round(48 * n_vis / (med["residual"] * 1e-3) / 1e9, 1)
    routes["direct_fp64"]["hbm_GB_per_s"] = round(40 * n_vis / (med["direct_fp64"] * 1e-3) / 1e9, 2)
    routes["direct_f32c"]["hbm_GB_per_s"] = round(32 * n_vis / (med["direct_f32c"] * 1e-3) / 1e9, 2)
    routes["speedup_f32c_over_fp64"] = round(med["direct_fp64"] / med["direct_f32c"], 3)
    # the last step's two direct sums, same inputs
    routes["direct_f32c"].update(precision_errors(v32, v64, float(np.abs(f).sum())))

    # roofline of the dominant kernel (largest device time in the step)
    def tree_flops(J):
        return n_vis * tree_flops_per_row(tree_stats[J])
    flops = {"direct_fp64": n_vis * n_comp * FLOPS["direct_fp64"],
             "adjoint": n_vis * n_pix * FLOPS["adjoint"],
             "grad": n_vis * n_comp * FLOPS["grad"]}
    for J in TREE_LEVELS:
        flops[f"tree_J{J}"] = tree_flops(J)
    kernel_of = {"direct_fp64": ("k_direct.hip", "k_direct_f64"),
                 "adjoint": ("k_image.hip", "k_adjoint"), "grad": ("k_image.hip", "k_grad_partial")}
    for J in TREE_LEVELS:
        kernel_of[f"tree_J{J}"] = ("k_tree.hip", f"k_tree_J{J}")
    dom = max(flops, key=lambda s: med[s])
    achieved = flops[dom] / (med[dom] * 1e-3) / 1e12
    src, kname = kernel_of[dom]
    traffic = traffic_for(src, kname)
    roofline = {"bound": "alu", "achieved": round(achieved, 2), "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
                "traffic": traffic, "kernel": kname, "stage": dom,
                "flops_per_launch": flops[dom], "avg_launch_ms": round(med[dom], 4),
                # the FP64 FMA rate a stream of independent FMAs reaches on this part
                "measured_peak": round(peaks["fp64_fma_tflops"], 2),
                "frac_of_measured": round(achieved / peaks["fp64_fma_tflops"], 4)}
    for s in flops:
        routes[s]["TFLOP_per_s"] = round(flops[s] / (med[s] * 1e-3) / 1e12, 2)
        routes[s]["fp64_alu_frac"] = round(flops[s] / (med[s] * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, 4)
    # the same fractions without the phasor polynomial's flops (34 per phasor)
    phasors = {"direct_fp64": n_vis * n_comp, "adjoint": n_vis * n_pix,
               "grad": n_vis * n_comp}
    for J in TREE_LEVELS:
        phasors[f"tree_J{J}"] = n_vis * tree_stats[J]["n_leaves"]
    for s in flops:
        routes[s]["fp64_alu_frac_excl_phasor"] = round(
            (flops[s] - PHASOR_FLOPS * phasors[s]) / (med[s] * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, 4)
    roofline["frac_excl_phasor"] = routes[dom]["fp64_alu_frac_excl_phasor"]
    # counter-based VALU issue: the kernel's VALU instructions (rocprofv3 SQ
    # counters, per launch) at 64 lanes each over the live launch time, against
    # the FP64 FMA lane rate measured on this part
    lane_rate = peaks["fp64_fma_tflops"] / 2 * 1e12
    for s in flops:
        nv = valu_count_for(*kernel_of[s])
        if nv:
            routes[s]["valu_issue_frac"] = round(64 * nv / (med[s] * 1e-3) / lane_rate, 4)
    roofline["valu_issue_frac"] = routes[dom].get("valu_issue_frac")
    routes["direct_f32c"]["roofline"] = dict(
        f32c_roofline("direct_f32c", n_vis * n_comp / (med["direct_f32c"] * 1e-3), peaks),
        kernel="k_direct_f32c")
    # value restricted to the prediction stages (direct FP64, FP32c, trees)
    pred = ["direct_fp64", "direct_f32c"] + [f"tree_J{J}" for J in TREE_LEVELS]
    pred_ms = sum(med[s] for s in pred)
    prediction_only = {"Gvis_terms_per_s": round(sum(terms[s] for s in pred) /
                                                 (pred_ms * 1e-3) / 1e9, 2),
                       "ms": round(pred_ms, 3), "stages": pred}

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": UNIT, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32c", "data": "synthetic",
        "config": {"workload": "cfg2 major cycle: 256-antenna 20 km array, 8 h at dec +30, "
                               "1.4 GHz, 8,355,840 vis; 2,000 components (70% in 5 blobs); "
                               "trees J=8,9,10; adjoint on the J=9 pixels within 4 deg",
                   "n_vis": n_vis, "n_comp": n_comp, "n_pix": int(n_pix),
                   "tree_levels": list(TREE_LEVELS), "terms_per_step": step_terms},
        "routes": routes,
        "prediction_only": prediction_only,
        "roofline": roofline,
        "measured_peaks": {k: round(v, 2) for k, v in peaks.items()},
        # measured after the timed steps, not part of the step or of value
        "extra_routes": extra_routes,
        "tile_shapes": {f: {"per_lane": pl, "block": bl} for f, (pl, bl) in tuning.items()},
    }
    if not (args.no_cfg3 or args.profile):
        log("precision form on its own workload (cfg3) ...")
        out["precision_cfg3"] = run_precision(swv, torch, np, dev, configs, peaks)
    if not (args.no_cfg4 or args.profile):
        log("batched form on its own workload (cfg4) ...")
        out["batched_cfg4"] = run_batched(swv, torch, np, dev, configs, peaks)
    if not (args.no_clean or args.profile):
        log("clean loop on the seven-source workload ...")
        out["clean_loop"] = run_clean(swv, torch, np, dev, configs)
        log("predictor comparison on the clean7 track ...")
        out["predictor_comparison"] = run_compare(swv, torch, np, dev, configs)
    if args.copy_calibration:
        # an elementwise kernel that reads 1 GiB and writes 1 GiB (a memcpy
        # would run on the copy engine, outside the counters' view)
        a = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = a.numel() * 8
    if not (args.no_cpu_baseline or args.profile):
        log("timing the oracle on the host ...")
        out["cpu_baseline"] = cpu_baseline(args.cpu_rows)
    print(json.dumps(out), flush=True)
    for T in keep_trees:
        T.close()


if __name__ == "__main__":
    main()
