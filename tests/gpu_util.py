"""Helpers of the GPU parity tests: device transfer, the oracle comparison metrics
and the tolerances (FP32 path: z within 1e-4 and LLRs within 1e-3 of the FP64
oracle, per vector; FP16-stored inputs: z within 3e-3)."""

import sys

import numpy as np
import torch

import oracle

Z_TOL_F32 = 1e-4
LLR_TOL_F32 = 1e-3
Z_TOL_F16 = 3e-3


def say(*msg):
    print("[gpu-test]", *msg, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def to_f16_pairs(a):
    """complex array -> float16 [..., 2] (the FP16 storage of H and y)."""
    a = np.ascontiguousarray(a)
    return np.stack([a.real, a.imag], axis=-1).astype(np.float16)


def from_f16_pairs(a):
    a = a.astype(np.float64)
    return a[..., 0] + 1j * a[..., 1]


def host(t):
    return t.detach().cpu().numpy()


def z_rel_err(zg, zo):
    """max over vectors of ||z_gpu - z_oracle||_2 / ||z_oracle||_2 (absolute if the norm is 0)."""
    U = zo.shape[-1]
    d = np.linalg.norm((zg.astype(np.complex128) - zo).reshape(-1, U), axis=1)
    n = np.linalg.norm(zo.reshape(-1, U), axis=1)
    return float(np.max(np.where(n > 0, d / np.maximum(n, 1e-300), d))) if d.size else 0.0


def llr_rel_err(Lg, Lo):
    """max over vectors of ||L_gpu - L_oracle||_inf / ||L_oracle||_inf."""
    if Lo.size == 0:
        return 0.0
    U, Q = Lo.shape[-2:]
    d = np.max(np.abs(Lg.astype(np.float64) - Lo).reshape(-1, U * Q), axis=1)
    n = np.max(np.abs(Lo).reshape(-1, U * Q), axis=1)
    return float(np.max(np.where(n > 0, d / np.maximum(n, 1e-300), d)))


def oracle_ref(H, y, K, Q, mode, N0, Es=1.0, lam=None, beta=0.0, hist=False):
    """FP64 oracle on exactly the values the GPU received (promoted)."""
    H = np.asarray(H, np.complex128)
    y = np.asarray(y, np.complex128)
    lam64 = None if lam is None else np.asarray(lam, np.float64)
    out = oracle.ocd(H, y, K, Q, mode, N0=N0, Es=Es, lam=lam64, beta=beta, hist=hist, threads=0)
    z, zh = (out if hist else (out, None))
    L = oracle.llr(H, z, K, Q, mode, N0=N0, Es=Es, lam=lam64, beta=beta, threads=0)
    return z, L, zh
