"""Torch-facing wrappers of libswvis.  Torch supplies device memory and the
stream; every step of the computation runs in the library's kernels."""
from __future__ import annotations

import atexit
import ctypes as C
import weakref

import numpy as np
import torch

from ._lib import (PREDICTORS, SWV_F32C, SWV_FP64, SWV_HOGBOM_ABS, SWV_HOGBOM_SINGLE,
                   CleanParams, CleanStats, CycleInstance,
                   DegridStats, Instance, PlanStats, TreeStats, check, lib)

PRECISIONS = {"fp64": SWV_FP64, "f32c": SWV_F32C}

# Live library objects by kind.  At interpreter exit they are destroyed in
# dependency order -- graphs, cycles, plans, trees, contexts (and with them the FFT
# plans of the degridding predictor) -- from an atexit hook, which runs before
# Python tears down its modules and before the HIP runtime and any tool
# attached to it shut down.  Finalizers left to module teardown would run in
# no useful order, and objects never destroyed would be released by the
# runtime's own exit handlers.
_LIVE = {kind: weakref.WeakSet() for kind in ("graph", "cycle", "plan", "tree", "ctx")}


def _track(kind, obj):
    _LIVE[kind].add(obj)


def shutdown():
    """Destroys every live library object in dependency order (registered to
    run at interpreter exit; safe to call earlier, objects are then closed)."""
    for kind in ("graph", "cycle", "plan", "tree", "ctx"):
        for obj in list(_LIVE[kind]):
            try:
                obj.close()
            except Exception:
                pass
    _CONTEXTS.clear()


atexit.register(shutdown)


def _prec(p) -> int:
    if isinstance(p, int):
        return p
    try:
        return PRECISIONS[p]
    except KeyError:
        raise ValueError(f"precision must be one of {sorted(PRECISIONS)}") from None


def _ptr(t) -> C.c_void_p:
    return C.c_void_p(t.data_ptr() if t is not None and t.numel() else 0)


def _dev_f64(t, name, device=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a GPU device")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if t.dim() != 1:
        raise ValueError(f"{name} must be 1-D")
    return t.resolve_neg().contiguous()


def _dev_c128(t, name, device):
    if not isinstance(t, torch.Tensor) or t.device != device or t.dtype != torch.complex128:
        raise TypeError(f"{name} must be a complex128 tensor on {device}")
    if t.dim() != 1:
        raise ValueError(f"{name} must be 1-D")
    # a lazily conjugated (or negated) view keeps the original values in
    # memory: materialise it before its pointer is handed to the library
    return t.resolve_conj().resolve_neg().contiguous()


def _host_f64(x):
    if isinstance(x, torch.Tensor):
        x = x.detach().cpu().numpy()
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def _np_ptr(a) -> C.c_void_p:
    return C.c_void_p(a.ctypes.data if a.size else 0)


class Context:
    """A libswvis context on one device and one stream."""

    def __init__(self, device=None, stream=None):
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        self.device = dev
        self.stream = stream
        self._h = C.c_void_p()
        check(lib().swv_ctx_create(dev.index, C.c_void_p(stream.cuda_stream), C.byref(self._h)))
        _track("ctx", self)

    @property
    def handle(self):
        return self._h

    def synchronize(self):
        """Waits for the stream and raises the first deferred kernel error."""
        check(lib().swv_ctx_synchronize(self._h))

    def tune_get(self, family: int, size_class: int):
        pl, bl = C.c_int(), C.c_int()
        check(lib().swv_tune_get(self._h, family, size_class, C.byref(pl), C.byref(bl)))
        return pl.value, bl.value

    def tune_set(self, family: int, size_class: int, per_lane: int, block: int):
        check(lib().swv_tune_set(self._h, family, size_class, per_lane, block))

    def autotune(self, cache_path=None, quick=False):
        p = cache_path.encode() if cache_path else None
        check(lib().swv_autotune(self._h, p, 1 if quick else 0))

    def measure_peaks(self) -> dict:
        """Measured arithmetic ceilings of this context's device (about 0.3 s)."""
        from ._lib import Peaks
        p = Peaks()
        check(lib().swv_measure_peaks(self._h, C.byref(p)))
        return {"fp64_fma_tflops": p.fp64_fma_tflops, "fp32_fma_tflops": p.fp32_fma_tflops,
                "sincos_f32_gops": p.sincos_f32_gops, "cis2pi_f64_gops": p.cis2pi_f64_gops}

    def tune_load(self, cache_path):
        check(lib().swv_tune_load(self._h, cache_path.encode()))

    def close(self):
        if self._h:
            lib().swv_ctx_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        # never raises (at interpreter exit shutdown() has already closed it)
        try:
            self.close()
        except Exception:
            pass


_CONTEXTS: dict = {}


def context(device=None) -> Context:
    """The cached context for a device and torch's current stream on it."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None \
        else torch.device(device)
    if dev.index is None:
        dev = torch.device("cuda", torch.cuda.current_device())
    st = torch.cuda.current_stream(dev)
    key = (dev.index, st.cuda_stream)
    ctx = _CONTEXTS.get(key)
    if ctx is None:
        ctx = _CONTEXTS[key] = Context(dev, st)
    return ctx


# ---------------------------------------------------------------- direct --
def predict_direct(u, v, w, l, m, flux, sign: int = -1, prec="fp64", out=None):
    """V_j = sum_k flux_k exp(s 2 pi i (u_j l_k + v_j m_k + w_j (n_k - 1))) (Eq. 12).

    u, v, w, l, m, flux: 1-D float64 tensors on one GPU.  Returns complex128
    (prec "fp64") or complex64 ("f32c")."""
    u = _dev_f64(u, "u")
    dev = u.device
    v, w = _dev_f64(v, "v", dev), _dev_f64(w, "w", dev)
    l, m, flux = _dev_f64(l, "l", dev), _dev_f64(m, "m", dev), _dev_f64(flux, "flux", dev)
    n, k = u.numel(), l.numel()
    if v.numel() != n or w.numel() != n or m.numel() != k or flux.numel() != k:
        raise ValueError("length mismatch")
    p = _prec(prec)
    dt = torch.complex128 if p == SWV_FP64 else torch.complex64
    if out is None:
        out = torch.empty(n, dtype=dt, device=dev)
    elif out.dtype != dt or out.numel() != n or not out.is_contiguous() or out.device != dev:
        raise ValueError("out has the wrong dtype, size or device")
    ctx = context(dev)
    check(lib().swv_predict_direct(ctx.handle, n, _ptr(u), _ptr(v), _ptr(w), k, _ptr(l),
                                   _ptr(m), _ptr(flux), sign, p, _ptr(out)))
    return out


# ------------------------------------------------------------------ tree --
class Tree:
    """Sparse spherical-Haar coefficient tree of a component list (built on the host)."""

    def __init__(self, J: int, ra_p: float, dec_p: float, l, m, flux):
        l, m, flux = _host_f64(l), _host_f64(m), _host_f64(flux)
        if not (l.shape == m.shape == flux.shape and l.ndim == 1):
            raise ValueError("l, m, flux must be 1-D of one length")
        self._h = C.c_void_p()
        check(lib().swv_tree_build(int(J), float(ra_p), float(dec_p), l.size, _np_ptr(l),
                                   _np_ptr(m), _np_ptr(flux), C.byref(self._h)))
        _track("tree", self)
        self.J, self.ra_p, self.dec_p = int(J), float(ra_p), float(dec_p)

    @classmethod
    def from_pixels(cls, J: int, ra_p: float, dec_p: float, pix, flux):
        """The tree of components given by their level-J pixel ids (the
        cross-referenced form of section 3.5)."""
        pix = np.ascontiguousarray(np.asarray(pix, dtype=np.int64))
        flux = _host_f64(flux)
        if pix.shape != flux.shape or pix.ndim != 1:
            raise ValueError("pix, flux must be 1-D of one length")
        t = cls.__new__(cls)
        t._h = C.c_void_p()
        check(lib().swv_tree_build_pixels(int(J), float(ra_p), float(dec_p), pix.size,
                                          _np_ptr(pix), _np_ptr(flux), C.byref(t._h)))
        _track("tree", t)
        t.J, t.ra_p, t.dec_p = int(J), float(ra_p), float(dec_p)
        return t

    @property
    def handle(self):
        return self._h

    def stats(self) -> dict:
        s = TreeStats()
        check(lib().swv_tree_stats(self._h, C.byref(s)))
        return {"J": s.J, "n_comp": s.n_comp, "n_leaves": s.n_leaves,
                "n_internal": s.n_internal,
                "nodes_per_level": [s.n_nodes[j] for j in range(1, s.J + 1)],
                "n_records": s.n_records, "sparsity": s.sparsity,
                "build_seconds": s.build_seconds, "max_branching": s.max_branching}

    def leaves(self) -> dict:
        n = self.stats()["n_leaves"]
        pix = np.empty(n, np.int64)
        arrs = [np.empty(n) for _ in range(4)]
        check(lib().swv_tree_leaves(self._h, _np_ptr(pix), *[_np_ptr(a) for a in arrs]))
        return {"pix": pix, "l": arrs[0], "m": arrs[1], "nm1": arrs[2], "flux": arrs[3]}

    def level(self, j: int) -> dict:
        n = self.stats()["nodes_per_level"][j - 1]
        pix = np.empty(n, np.int64)
        mask = np.empty(n, np.int32)
        lam = np.empty(n)
        gam = np.empty((n, 3))
        check(lib().swv_tree_level(self._h, j, _np_ptr(pix), _np_ptr(mask), _np_ptr(lam),
                                   _np_ptr(gam)))
        return {"pix": pix, "mask": mask, "lambda": lam, "gamma": gam}

    def threshold(self, fraction: float) -> "Tree":
        """A thresholded copy keeping the given proportion of the wavelet
        coefficients (largest |gamma|); nodes with nothing kept below them
        become leaves at their own level."""
        t = Tree.__new__(Tree)
        t._h = C.c_void_p()
        check(lib().swv_tree_threshold(self._h, float(fraction), C.byref(t._h)))
        _track("tree", t)
        t.J, t.ra_p, t.dec_p = self.J, self.ra_p, self.dec_p
        return t

    def prune(self, kept) -> "Tree":
        """A thresholded copy keeping the coefficients with the given flat
        indices (increasing; 3 x nodes of the levels above + 3 k + m)."""
        k = np.ascontiguousarray(np.asarray(kept, dtype=np.int64))
        t = Tree.__new__(Tree)
        t._h = C.c_void_p()
        check(lib().swv_tree_prune(self._h, k.size, _np_ptr(k), C.byref(t._h)))
        _track("tree", t)
        t.J, t.ra_p, t.dec_p = self.J, self.ra_p, self.dec_p
        return t

    def kept(self):
        """(retained flat indices, number of coefficients) of a thresholded tree."""
        n, nc = C.c_int64(), C.c_int64()
        check(lib().swv_tree_kept(self._h, 0, C.c_void_p(0), C.byref(n), C.byref(nc)))
        out = np.empty(n.value, np.int64)
        check(lib().swv_tree_kept(self._h, n.value, _np_ptr(out), C.byref(n), C.byref(nc)))
        return out, nc.value

    def set_leaf_flux(self, flux):
        """New flux per leaf (leaf order), same pixel set; coefficients recomputed."""
        f = _host_f64(flux)
        if f.size != self.stats()["n_leaves"]:
            raise ValueError("one flux per leaf is needed")
        check(lib().swv_tree_set_flux(self._h, _np_ptr(f)))

    def predict(self, u, v, w, sign: int = -1, prec="fp64", out=None):
        """Model visibilities by the wavelet route (Eqs. 14-17): complex128
        (prec "fp64") or complex64 ("f32c", FP32 phasors at the leaves)."""
        u = _dev_f64(u, "u")
        dev = u.device
        v, w = _dev_f64(v, "v", dev), _dev_f64(w, "w", dev)
        n = u.numel()
        if v.numel() != n or w.numel() != n:
            raise ValueError("length mismatch")
        p = _prec(prec)
        dt = torch.complex128 if p == SWV_FP64 else torch.complex64
        if out is None:
            out = torch.empty(n, dtype=dt, device=dev)
        elif out.dtype != dt or out.numel() != n or not out.is_contiguous() or out.device != dev:
            raise ValueError("out has the wrong dtype, size or device")
        ctx = context(dev)
        check(lib().swv_predict_tree(ctx.handle, self._h, n, _ptr(u), _ptr(v), _ptr(w), sign, p,
                                     _ptr(out)))
        return out

    def predict_leaves(self, u, v, w, sign: int = -1, prec="fp64", out=None):
        """The same model visibilities as predict() in the form of Eq. 16: the
        direct sum over the merged leaves at their pixel centres."""
        u = _dev_f64(u, "u")
        dev = u.device
        v, w = _dev_f64(v, "v", dev), _dev_f64(w, "w", dev)
        n = u.numel()
        if v.numel() != n or w.numel() != n:
            raise ValueError("length mismatch")
        p = _prec(prec)
        dt = torch.complex128 if p == SWV_FP64 else torch.complex64
        if out is None:
            out = torch.empty(n, dtype=dt, device=dev)
        elif out.dtype != dt or out.numel() != n or not out.is_contiguous() or out.device != dev:
            raise ValueError("out has the wrong dtype, size or device")
        check(lib().swv_predict_tree_leaves(context(dev).handle, self._h, n, _ptr(u), _ptr(v),
                                            _ptr(w), sign, p, _ptr(out)))
        return out

    def close(self):
        if self._h:
            lib().swv_tree_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        # never raises (at interpreter exit shutdown() has already closed it)
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- pixels --
def ang2pix(J, ra_p, dec_p, l, m) -> np.ndarray:
    l, m = _host_f64(l), _host_f64(m)
    pix = np.empty(l.size, np.int64)
    check(lib().swv_ang2pix(int(J), float(ra_p), float(dec_p), l.size, _np_ptr(l), _np_ptr(m),
                            _np_ptr(pix)))
    return pix


def pixel_centres(J, ra_p, dec_p, pix):
    pix = np.ascontiguousarray(np.asarray(pix, np.int64))
    out = [np.empty(pix.size) for _ in range(3)]
    check(lib().swv_pixel_centres(int(J), float(ra_p), float(dec_p), pix.size, _np_ptr(pix),
                                  *[_np_ptr(a) for a in out]))
    return tuple(out)


def pixels_in_disk(J, ra_p, dec_p, radius):
    """(pix, l, m, nm1) of the level-J pixels within `radius` of the phase centre."""
    n = C.c_int64()
    z = C.c_void_p(0)
    check(lib().swv_pixels_in_disk(int(J), float(ra_p), float(dec_p), float(radius), 0, z, z, z,
                                   z, C.byref(n)))
    pix = np.empty(n.value, np.int64)
    arrs = [np.empty(n.value) for _ in range(3)]
    check(lib().swv_pixels_in_disk(int(J), float(ra_p), float(dec_p), float(radius), n.value,
                                   _np_ptr(pix), *[_np_ptr(a) for a in arrs], C.byref(n)))
    return pix, arrs[0], arrs[1], arrs[2]


# ------------------------------------------------- subtract, image, grads --
def residual_chi2(vis_obs, vis_model, inv_sigma2: float, out=None):
    """(V_obs - V_model, chi^2 as a 1-element float64 tensor)."""
    dev = vis_obs.device
    vis_obs = _dev_c128(vis_obs, "vis_obs", dev)
    vis_model = _dev_c128(vis_model, "vis_model", dev)
    n = vis_obs.numel()
    if vis_model.numel() != n:
        raise ValueError("length mismatch")
    if out is None:
        resid = torch.empty_like(vis_obs)
    else:
        resid = _dev_c128(out, "out", dev)
        if resid.numel() != n or resid.data_ptr() != out.data_ptr():
            raise ValueError("out must be a contiguous complex128 tensor of the same length")
    chi2 = torch.empty(1, dtype=torch.float64, device=dev)
    ctx = context(dev)
    check(lib().swv_residual_chi2(ctx.handle, n, _ptr(vis_obs), _ptr(vis_model),
                                  float(inv_sigma2), _ptr(resid), _ptr(chi2)))
    return resid, chi2


def adjoint(u, v, w, y, l, m, nm1, sign: int = -1, prec="fp64", out=None, noalloc=False):
    """x_p = sum_j conj(e_jp) y_j on the pixel set (l, m, n - 1); complex128.

    noalloc=True calls swv_adjoint_noalloc, which keeps its partial sums in
    the library's fixed device array (the same bits; pass `out` as well for a
    call that allocates nothing)."""
    u = _dev_f64(u, "u")
    dev = u.device
    v, w = _dev_f64(v, "v", dev), _dev_f64(w, "w", dev)
    y = _dev_c128(y, "y", dev)
    l, m, nm1 = _dev_f64(l, "l", dev), _dev_f64(m, "m", dev), _dev_f64(nm1, "nm1", dev)
    n, P = u.numel(), l.numel()
    if v.numel() != n or w.numel() != n or y.numel() != n or m.numel() != P or nm1.numel() != P:
        raise ValueError("length mismatch")
    if out is None:
        out = torch.empty(P, dtype=torch.complex128, device=dev)
    elif (out.dtype != torch.complex128 or out.numel() != P or not out.is_contiguous()
          or out.device != dev):
        raise ValueError("out must be a contiguous complex128 tensor of n_pix entries")
    ctx = context(dev)
    fn = lib().swv_adjoint_noalloc if noalloc else lib().swv_adjoint
    check(fn(ctx.handle, n, _ptr(u), _ptr(v), _ptr(w), _ptr(y), P, _ptr(l), _ptr(m), _ptr(nm1),
             sign, _prec(prec), _ptr(out)))
    return out


def grad_direct(u, v, w, y, l, m, flux, sign: int = -1, alpha: float = 1.0):
    """Gradient of alpha Re sum_j conj(y_j) V_j with respect to (flux, l, m)."""
    u = _dev_f64(u, "u")
    dev = u.device
    v, w = _dev_f64(v, "v", dev), _dev_f64(w, "w", dev)
    y = _dev_c128(y, "y", dev)
    l, m, flux = _dev_f64(l, "l", dev), _dev_f64(m, "m", dev), _dev_f64(flux, "flux", dev)
    n, k = u.numel(), l.numel()
    if v.numel() != n or w.numel() != n or y.numel() != n or m.numel() != k or flux.numel() != k:
        raise ValueError("length mismatch")
    outs = [torch.empty(k, dtype=torch.float64, device=dev) for _ in range(3)]
    ctx = context(dev)
    check(lib().swv_grad_direct(ctx.handle, n, _ptr(u), _ptr(v), _ptr(w), _ptr(y), k, _ptr(l),
                                _ptr(m), _ptr(flux), sign, float(alpha),
                                *[_ptr(o) for o in outs]))
    return tuple(outs)


# --------------------------------------------------------------- batched --
ROUTES = {"direct": 0, "tree": 1}


# ----------------------------------------------------------------- clean --
def _dev(device):
    if device is None:
        return torch.device("cuda", torch.cuda.current_device())
    return torch.device(device)


def _uvw(u, v, w):
    u = _dev_f64(u, "u")
    dev = u.device
    v, w = _dev_f64(v, "v", dev), _dev_f64(w, "w", dev)
    if v.numel() != u.numel() or w.numel() != u.numel():
        raise ValueError("length mismatch")
    return u, v, w, dev


def _image(t, name, shape, device):
    if not isinstance(t, torch.Tensor) or t.device != device or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 tensor on {device}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def image_grid(nx: int, ny: int, cell: float, cx=None, cy=None, device=None):
    """Directions (l, m, n - 1) of the pixels of an (ny, nx) grid, phase centre
    at pixel (cx, cy) (default (nx // 2, ny // 2)); 1-D float64 tensors."""
    dev = _dev(device)
    n = int(nx) * int(ny)
    l, m, nm1 = (torch.empty(n, dtype=torch.float64, device=dev) for _ in range(3))
    cx = int(nx) // 2 if cx is None else int(cx)
    cy = int(ny) // 2 if cy is None else int(cy)
    check(lib().swv_image_grid(context(dev).handle, int(nx), int(ny), cx, cy, float(cell),
                               _ptr(l), _ptr(m), _ptr(nm1)))
    return l, m, nm1


def dirty_image(u, v, w, y, nx: int, ny: int, cell: float, cx=None, cy=None, sign: int = -1,
                prec="fp64"):
    """(1 / N_vis) Re sum_j conj(e_jp) y_j on an (ny, nx) grid; y None means
    unit visibilities; prec "f32c" takes the adjoint's FP32-compensated form.
    Returns a (ny, nx) float64 tensor."""
    u, v, w, dev = _uvw(u, v, w)
    yp = C.c_void_p(0)
    if y is not None:
        y = _dev_c128(y, "y", dev)
        if y.numel() != u.numel():
            raise ValueError("length mismatch")
        yp = _ptr(y)
    cx = int(nx) // 2 if cx is None else int(cx)
    cy = int(ny) // 2 if cy is None else int(cy)
    out = torch.empty((int(ny), int(nx)), dtype=torch.float64, device=dev)
    check(lib().swv_dirty_image(context(dev).handle, u.numel(), _ptr(u), _ptr(v), _ptr(w), yp,
                                int(nx), int(ny), cx, cy, float(cell), int(sign), _prec(prec),
                                _ptr(out)))
    return out


def dirty_beam(u, v, w, nx: int, ny: int, cell: float, sign: int = -1, prec="fp64"):
    """Dirty beam of an (ny, nx) image: the (2 ny - 1, 2 nx - 1) image of a
    unit source at the phase centre, zero offset at (ny - 1, nx - 1)."""
    return dirty_image(u, v, w, None, 2 * int(nx) - 1, 2 * int(ny) - 1, cell, int(nx) - 1,
                       int(ny) - 1, sign, prec)


def hogbom(image, beam, gain: float, threshold: float, max_iter: int, absolute=False,
           single_workgroup=False):
    """Hogbom minor cycle (Eqs. 4, 5) on a (ny, nx) float64 image, updated in
    place to the residual.  Returns (pixel ids, component values g C_n) as
    device tensors; waits for the kernel to learn their number.
    single_workgroup keeps a large image's cycle in one workgroup (the same
    bits as the grid-wide form)."""
    if not isinstance(image, torch.Tensor) or image.dim() != 2:
        raise ValueError("image must be a 2-D tensor")
    dev = image.device
    ny, nx = image.shape
    _image(image, "image", (ny, nx), dev)
    _image(beam, "beam", (2 * ny - 1, 2 * nx - 1), dev)
    k = int(max_iter)
    pix = torch.empty(max(k, 1), dtype=torch.int64, device=dev)
    val = torch.empty(max(k, 1), dtype=torch.float64, device=dev)
    n = torch.zeros(1, dtype=torch.int64, device=dev)
    check(lib().swv_hogbom(context(dev).handle, nx, ny, _ptr(image), _ptr(beam), float(gain),
                           float(threshold), k, (SWV_HOGBOM_ABS if absolute else 0) |
                           (SWV_HOGBOM_SINGLE if single_workgroup else 0), _ptr(pix),
                           _ptr(val), _ptr(n)))
    found = int(n.item())
    if found < 0:
        raise RuntimeError("the grid-wide Hogbom cycle timed out waiting for a workgroup")
    return pix[:found], val[:found]


def cross_reference(J: int, ra_p: float, dec_p: float, nx: int, ny: int, cell: float):
    """Level-J sphere pixel of every image pixel (section 3.5): int64 numpy [ny * nx]."""
    out = np.empty(int(nx) * int(ny), np.int64)
    check(lib().swv_cross_reference(int(J), float(ra_p), float(dec_p), int(nx), int(ny),
                                    float(cell), _np_ptr(out)))
    return out


def fit_clean_beam(beam):
    """(a, b, c) of the clean beam exp(-(a dx^2 + 2 b dx dy + c dy^2)) fitted to
    the main lobe of a dirty beam (2-D, zero offset at its centre)."""
    if isinstance(beam, torch.Tensor):
        beam = beam.detach().cpu().numpy()
    b = np.ascontiguousarray(np.asarray(beam, dtype=np.float64))
    if b.ndim != 2:
        raise ValueError("beam must be 2-D")
    abc = np.empty(3)
    check(lib().swv_fit_clean_beam(b.shape[1], b.shape[0], _np_ptr(b), _np_ptr(abc)))
    return tuple(float(x) for x in abc)


def restore(nx: int, ny: int, pix, val, abc, residual=None):
    """Clean image of Eq. 6 (plus the residual image if given): (ny, nx) float64."""
    if not isinstance(pix, torch.Tensor) or pix.dtype != torch.int64 or pix.dim() != 1:
        raise TypeError("pix must be a 1-D int64 tensor")
    dev = pix.device
    pix = pix.contiguous()
    val = _dev_f64(val, "val", dev)
    if val.numel() != pix.numel():
        raise ValueError("pix and val differ in length")
    if residual is not None:
        residual = _image(residual, "residual", (int(ny), int(nx)), dev)
    out = torch.empty((int(ny), int(nx)), dtype=torch.float64, device=dev)
    a = np.asarray(abc, dtype=np.float64)
    check(lib().swv_restore(context(dev).handle, int(nx), int(ny), pix.numel(), _ptr(pix),
                            _ptr(val), _np_ptr(a), _ptr(residual), _ptr(out)))
    return out


def predict_degrid(image, u, v, w, cell: float, support: int = 10, sign: int = -1, out=None):
    """Model visibilities of a (ny, nx) float64 image by FFT + degridding (the
    conventional predictor; exponential-of-semicircle kernel over `support`
    cells in u, v and w).  Returns (complex128 visibilities, stats dict)."""
    u, v, w, dev = _uvw(u, v, w)
    if not isinstance(image, torch.Tensor) or image.dim() != 2:
        raise ValueError("image must be a 2-D tensor")
    ny, nx = image.shape
    _image(image, "image", (ny, nx), dev)
    n = u.numel()
    if out is None:
        out = torch.empty(n, dtype=torch.complex128, device=dev)
    elif out.dtype != torch.complex128 or out.numel() != n or out.device != dev:
        raise ValueError("out has the wrong dtype, size or device")
    st = DegridStats()
    check(lib().swv_predict_degrid(context(dev).handle, nx, ny, float(cell), _ptr(image), n,
                                   _ptr(u), _ptr(v), _ptr(w), int(support), int(sign), _ptr(out),
                                   C.byref(st)))
    return out, {"n_planes": st.n_planes, "grid": (st.grid_ny, st.grid_nx), "w0": st.w0,
                 "dw": st.dw, "c": st.c, "plane_bytes": st.plane_bytes, "host_ms": st.host_ms}


def wavelet_clean(u, v, w, vis_obs, nx: int, ny: int, cell: float, J: int, ra_p: float,
                  dec_p: float, gain: float = 0.1, threshold: float = 0.0, minor_iter: int = 100,
                  n_major: int = 1, absolute=False, sign: int = -1, predictor: str = "tree",
                  support: int = 10, image_prec="fp64"):
    """Cotton-Schwab cleaning with the wavelet predictor (sections 2.2, 3.5);
    predictor "degrid" (FFT + degridding of the model image, kernel width
    `support`) or "direct" (direct sum over the model pixels) runs the same
    loop as conventional or exact clean; image_prec "f32c" forms the dirty
    beam, the dirty image and the residual images with the FP32-compensated
    adjoint.  Returns a dict: pix, val (numpy, all
    components in order), residual and beam (device images), vis_model
    (device complex128) and per-cycle stats."""
    if predictor not in PREDICTORS:
        raise ValueError(f"predictor must be one of {sorted(PREDICTORS)}")
    u, v, w, dev = _uvw(u, v, w)
    vis_obs = _dev_c128(vis_obs, "vis_obs", dev)
    n = u.numel()
    if vis_obs.numel() != n:
        raise ValueError("length mismatch")
    P = CleanParams(int(nx), int(ny), float(cell), int(J), float(ra_p), float(dec_p),
                    float(gain), float(threshold), int(minor_iter), int(n_major),
                    SWV_HOGBOM_ABS if absolute else 0, int(sign), PREDICTORS[predictor],
                    int(support), _prec(image_prec))
    beam = torch.empty((2 * int(ny) - 1, 2 * int(nx) - 1), dtype=torch.float64, device=dev)
    resid = torch.empty((int(ny), int(nx)), dtype=torch.float64, device=dev)
    vm = torch.empty(n, dtype=torch.complex128, device=dev)
    cap = max(int(minor_iter) * int(n_major), 1)
    pix = np.empty(cap, np.int64)
    val = np.empty(cap)
    nc = C.c_int64(0)
    st = CleanStats()
    check(lib().swv_wavelet_clean(context(dev).handle, C.byref(P), n, _ptr(u), _ptr(v), _ptr(w),
                                  _ptr(vis_obs), _ptr(beam), _ptr(resid), _ptr(vm), cap,
                                  _np_ptr(pix), _np_ptr(val), C.byref(nc), C.byref(st)))
    k = st.n_cycles
    cycles = [{"found": st.found[i], "leaves": st.leaves[i], "chi2": st.chi2[i],
               "ms_minor": st.ms_minor[i], "ms_build": st.ms_build[i],
               "ms_predict": st.ms_predict[i], "ms_image": st.ms_image[i]} for i in range(k)]
    return {"pix": pix[:nc.value].copy(), "val": val[:nc.value].copy(), "residual": resid,
            "beam": beam, "vis_model": vm, "cycles": cycles, "ms_beam": st.ms_beam,
            "ms_dirty": st.ms_dirty}


class Graph:
    """A captured batched prediction; launch() replays it on the plan's stream."""

    def __init__(self, plan):
        self.plan = plan
        self._h = C.c_void_p()
        check(lib().swv_graph_capture(plan.handle, C.byref(self._h)))
        _track("graph", self)

    def launch(self):
        check(lib().swv_graph_launch(self._h))

    def close(self):
        if self._h:
            lib().swv_graph_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        # never raises (at interpreter exit shutdown() has already closed it)
        try:
            self.close()
        except Exception:
            pass


class BatchPlan:
    """One persistent launch per route over many prediction instances.

    instances: dicts with keys route ("direct" | "tree"), u, v, w (float64 GPU
    tensors), out (complex128, or complex64 for a "f32c" instance),
    sign (default -1), prec (default "fp64"), and l, m, flux (float64 GPU
    tensors, direct) or tree (a Tree).  The tensors and trees must outlive the
    plan; the plan keeps references to them."""

    def __init__(self, instances, device=None):
        self._keep = []
        arr = (Instance * max(1, len(instances)))()
        dev = None
        for k, d in enumerate(instances):
            u = _dev_f64(d["u"], "u")
            dev = dev or u.device
            v, w = _dev_f64(d["v"], "v", u.device), _dev_f64(d["w"], "w", u.device)
            out = d["out"]
            n = u.numel()
            if v.numel() != n or w.numel() != n or out.numel() != n or not out.is_contiguous():
                raise ValueError(f"instance {k}: length mismatch")
            I = arr[k]
            I.route = ROUTES[d.get("route", "direct")]
            I.prec = _prec(d.get("prec", "fp64"))
            want = torch.complex128 if I.prec == SWV_FP64 else torch.complex64
            if out.dtype != want or out.device != u.device:
                raise TypeError(f"instance {k}: out must be {want} on {u.device}")
            I.sign = int(d.get("sign", -1))
            I.n_vis = n
            I.u, I.v, I.w = _ptr(u).value, _ptr(v).value, _ptr(w).value
            I.vis_out = _ptr(out).value
            self._keep += [u, v, w, out]
            if I.route == 0:
                l = _dev_f64(d["l"], "l", u.device)
                m = _dev_f64(d["m"], "m", u.device)
                f = _dev_f64(d["flux"], "flux", u.device)
                I.n_comp = l.numel()
                I.l, I.m, I.flux = _ptr(l).value, _ptr(m).value, _ptr(f).value
                self._keep += [l, m, f]
            else:
                t = d["tree"]
                I.tree = t.handle.value
                self._keep.append(t)
        self.ctx = context(dev if device is None else device)
        self._h = C.c_void_p()
        check(lib().swv_batch_plan(self.ctx.handle, len(instances), arr, C.byref(self._h)))
        _track("plan", self)

    @property
    def handle(self):
        return self._h

    def stats(self) -> dict:
        s = PlanStats()
        check(lib().swv_plan_stats(self._h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in PlanStats._fields_}

    def run(self):
        check(lib().swv_batch_run(self._h))

    def capture(self) -> Graph:
        return Graph(self)

    def close(self):
        if self._h:
            lib().swv_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        # never raises (at interpreter exit shutdown() has already closed it)
        try:
            self.close()
        except Exception:
            pass


class MajorCycle:
    """Major cycles over many instances, eager or as one captured HIP graph:
    batched prediction, then per instance the residual and chi^2, the residual
    image on a pixel set and (direct instances) the chi^2 gradients.

    instances: dicts with route ("direct" | "tree"), u, v, w, vis_obs
    (complex128), inv_sigma2, optional sign (-1), pixels (l, m, nm1) of the
    residual image, comp_cap (direct: most components; tree: most leaves),
    tree_level_cap (tree: largest J) and grads (direct: True to form d chi^2 /
    d(flux, l, m)).  The cycle allocates the outputs: vis_model, resid, chi2,
    image and grads per instance (tensors, overwritten by every cycle).  Models
    are set with set_components / set_tree and may change between cycles
    without a new capture."""

    def __init__(self, instances, device=None):
        self._keep = []
        self.out = []
        arr = (CycleInstance * max(1, len(instances)))()
        dev = None
        for k, d in enumerate(instances):
            u = _dev_f64(d["u"], "u")
            dev = dev or u.device
            v, w = _dev_f64(d["v"], "v", u.device), _dev_f64(d["w"], "w", u.device)
            obs = _dev_c128(d["vis_obs"], "vis_obs", u.device)
            n = u.numel()
            if v.numel() != n or w.numel() != n or obs.numel() != n:
                raise ValueError(f"instance {k}: length mismatch")
            I = arr[k]
            I.route = ROUTES[d.get("route", "direct")]
            I.sign = int(d.get("sign", -1))
            I.n_vis = n
            I.u, I.v, I.w, I.vis_obs = (_ptr(t).value for t in (u, v, w, obs))
            o = {"vis_model": torch.empty(n, dtype=torch.complex128, device=u.device),
                 "resid": torch.empty(n, dtype=torch.complex128, device=u.device),
                 "chi2": torch.zeros(1, dtype=torch.float64, device=u.device)}
            I.vis_model, I.resid, I.chi2 = (_ptr(o[x]).value for x in ("vis_model", "resid",
                                                                         "chi2"))
            I.inv_sigma2 = float(d["inv_sigma2"])
            self._keep += [u, v, w, obs]
            if d.get("pixels") is not None:
                pl, pm, pn = (_dev_f64(t, "pixels", u.device) for t in d["pixels"])
                if pm.numel() != pl.numel() or pn.numel() != pl.numel():
                    raise ValueError(f"instance {k}: pixel arrays differ in length")
                o["image"] = torch.empty(pl.numel(), dtype=torch.complex128, device=u.device)
                I.n_pix = pl.numel()
                I.pix_l, I.pix_m, I.pix_nm1 = _ptr(pl).value, _ptr(pm).value, _ptr(pn).value
                I.image = _ptr(o["image"]).value
                self._keep += [pl, pm, pn]
            I.comp_cap = int(d.get("comp_cap", 0))
            I.tree_level_cap = int(d.get("tree_level_cap", 1 if I.route == 0 else 10))
            if d.get("grads"):
                g = [torch.zeros(max(I.comp_cap, 1), dtype=torch.float64, device=u.device)
                     for _ in range(3)]
                o["grads"] = g
                I.d_flux, I.d_l, I.d_m = (_ptr(t).value for t in g)
            self.out.append(o)
        self.ctx = context(dev if device is None else device)
        self._h = C.c_void_p()
        check(lib().swv_cycle_create(self.ctx.handle, len(instances), arr, C.byref(self._h)))
        _track("cycle", self)
        self._models = [None] * len(instances)

    def set_components(self, k: int, l, m, flux):
        dev = self.ctx.device
        l, m, flux = _dev_f64(l, "l", dev), _dev_f64(m, "m", dev), _dev_f64(flux, "flux", dev)
        if m.numel() != l.numel() or flux.numel() != l.numel():
            raise ValueError("l, m, flux differ in length")
        check(lib().swv_cycle_set_components(self._h, int(k), l.numel(), _ptr(l), _ptr(m),
                                             _ptr(flux)))
        self._models[k] = (l, m, flux)     # read on every run: keep them alive

    def set_tree(self, k: int, tree):
        check(lib().swv_cycle_set_tree(self._h, int(k), tree.handle))
        self._models[k] = None              # the records were copied

    def run(self):
        check(lib().swv_cycle_run(self._h))

    def capture(self):
        check(lib().swv_cycle_capture(self._h))

    def launch(self):
        check(lib().swv_cycle_launch(self._h))

    def close(self):
        if self._h:
            lib().swv_cycle_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        # never raises (at interpreter exit shutdown() has already closed it)
        try:
            self.close()
        except Exception:
            pass


def synchronize(device=None):
    """Waits for the current stream and raises deferred kernel errors."""
    context(device).synchronize()


__all__ = ["Context", "context", "predict_direct", "Tree", "ang2pix", "pixel_centres",
           "pixels_in_disk", "residual_chi2", "adjoint", "grad_direct", "synchronize",
           "BatchPlan", "Graph", "MajorCycle"]
