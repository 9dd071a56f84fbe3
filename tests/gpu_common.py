"""Helpers shared by the GPU tests: device buffers via torch, and plain
numpy/oracle references for single kernels."""
from __future__ import annotations

import numpy as np

import oracle as O


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a HIP device")
    return torch


def to_device_planes(arr: np.ndarray):
    """(3, S) complex -> device float64 tensor in the stage-plane layout
    d[(i*S + site)*2 + comp]."""
    torch = torch_cuda()
    flat = np.stack([arr.real, arr.imag], axis=-1).reshape(-1)
    return torch.from_numpy(np.ascontiguousarray(flat)).to("cuda")


def from_device_planes(t, sites: int) -> np.ndarray:
    a = t.cpu().numpy().reshape(3, sites, 2)
    return a[..., 0] + 1j * a[..., 1]


def oracle_update_residual(orc: O.MB4Oracle, u0, U, rbar):
    """U' = U + (T (x) I) rbar and Phibar(U') = (T^-1 (x) I) Phi(U') by the oracle."""
    k = orc.k
    Un = U + np.tensordot(k.T, rbar, axes=(1, 0)) if rbar is not None else U.copy()
    phi = orc.residual(u0, Un)
    return Un, np.tensordot(k.Tinv, phi, axes=(1, 0))


def block_jacobi_reference(nx, ny, v, shift, t, g, h, lam, u0, phib, sweeps):
    """Plain numpy block-Jacobi for (I - h lam_i J) r_i = -phib_i, J frozen at
    u0 (the hopping links taken from the previous iterate), from r = 0."""
    p, q = u0.real, u0.imag
    vs = v + shift
    a = 2 * g * p * q
    bb = vs + g * (p * p + 3 * q * q)
    cc = vs + g * (3 * p * p + q * q)
    out = np.zeros_like(phib)
    for i in range(3):
        hl = h * lam[i]
        det = 1 + hl * hl * (bb * cc - a * a)
        r = np.zeros(nx * ny, dtype=complex)
        for _ in range(sweeps):
            r2 = r.reshape(ny, nx)
            s = (np.roll(r2, 1, 1) + np.roll(r2, -1, 1) + np.roll(r2, 1, 0)
                 + np.roll(r2, -1, 0)).reshape(-1)
            bp = -phib[i].real - hl * t * s.imag
            bq = -phib[i].imag + hl * t * s.real
            rp = ((1 + hl * a) * bp + hl * bb * bq) / det
            rq = ((1 - hl * a) * bq - hl * cc * bp) / det
            r = rp + 1j * rq
        out[i] = r
    return out
