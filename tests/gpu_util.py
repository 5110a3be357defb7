"""Helpers of the GPU parity tests (imported by tests/test_gpu_*.py only)."""
import sys

import numpy as np
import pytest


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1909_03956_amd as swv
    swv.lib()   # raises if the library is not built: no fallback exists
    return torch, swv


def dev(x, torch):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def dev_c(x, torch):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.complex128, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def errors(got, ref, scale):
    """(E_max, E_rms): max |dV| / scale and ||dV||_2 / ||V||_2."""
    d = np.abs(np.asarray(got, np.complex128) - ref)
    e_max = float(d.max() / scale) if d.size else 0.0
    nrm = float(np.linalg.norm(ref))
    e_rms = float(np.linalg.norm(d) / nrm) if nrm > 0 else 0.0
    return e_max, e_rms


def note(*args):
    print(*args, flush=True)
    sys.stdout.flush()


U_R = 2.0 ** -53


def fp64_row_bound(u, v, w, l, m, nm1, amp):
    """Per-row bound on |V_gpu - V_exact| of an FP64 direct sum: the phase
    phi = fma(u, l, fma(v, m, w (n-1))) carries at most 3 u_r Phi rounding
    (Phi = |u l| + |v m| + |w (n-1)|, u_r = 2^-53), the phasor ~4e-16, the
    sum and the oracle another ~1e-15 per term."""
    u, v, w = (np.abs(np.asarray(a))[:, None] for a in (u, v, w))
    l, m, nm1 = (np.abs(np.asarray(a))[None, :] for a in (l, m, nm1))
    phi = u * l + v * m + w * nm1
    return (np.abs(np.asarray(amp))[None, :] * (2 * np.pi * 3 * U_R * phi + 2e-15)).sum(axis=1)
