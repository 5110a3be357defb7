"""The oracle over full workload sizes, split into row chunks in spawned
worker processes (NumPy only, none touches the GPU).  Test infrastructure for
the GPU parity tests; the sums over rows it splits are linear in the rows, so
chunk results are added."""
import multiprocessing as mp
import os

import numpy as np


def n_workers() -> int:
    """One GPU's share of host cores at most."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _chunks(n, k):
    edges = np.linspace(0, n, k + 1).astype(np.int64)
    return [(int(a), int(b)) for a, b in zip(edges[:-1], edges[1:]) if b > a]


def _cfg5_model_residual(args):
    """V(perturbed model) - V(model) on the given rows of config 5 (no noise)."""
    rows, = args
    from oracle import visibility as ov
    from synth import configs, models
    W = configs.CFG2
    u, v, w = W.track.uvw_rows(rows)
    l, m, f = W.components()
    l2, m2, f2 = models.perturb_model(l, m, f, np.random.default_rng(configs.CFG5_SEED_PERTURB))
    return ov.predict_direct_fp64(u, v, w, l2, m2, f2) - ov.predict_direct_fp64(u, v, w, l, m, f)


def _adjoint(args):
    u, v, w, y, l, m, nm1 = args
    from oracle import visibility as ov
    return ov.adjoint(u, v, w, y, l, m, nm1, chunk=8192)


def _grad(args):
    u, v, w, y, l, m, f, alpha = args
    from oracle import visibility as ov
    return np.stack(ov.grad_direct(u, v, w, y, l, m, f, alpha=alpha, chunk=8192))


def _map(fn, tasks):
    ctx = mp.get_context("spawn")
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    with ctx.Pool(min(n_workers(), len(tasks))) as pool:
        return pool.map(fn, tasks)


def cfg5_residual(rows, noise):
    """Config 5's residual on `rows`: the perturbed model's visibilities plus
    the noise, minus the model's (the noise of those rows is given)."""
    rows = np.asarray(rows, np.int64)
    parts = _map(_cfg5_model_residual, [(rows[a:b],) for a, b in _chunks(rows.size, 4 * n_workers())])
    return np.concatenate(parts) + noise


def adjoint(u, v, w, y, l, m, nm1):
    tasks = [(u[a:b], v[a:b], w[a:b], y[a:b], l, m, nm1)
             for a, b in _chunks(u.size, 2 * n_workers())]
    return np.sum(_map(_adjoint, tasks), axis=0)


def grad_direct(u, v, w, y, l, m, f, alpha):
    tasks = [(u[a:b], v[a:b], w[a:b], y[a:b], l, m, f, alpha)
             for a, b in _chunks(u.size, 2 * n_workers())]
    return tuple(np.sum(_map(_grad, tasks), axis=0))
