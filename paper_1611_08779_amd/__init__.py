"""Python binding of libocd.so: OCD soft-output MU-MIMO-OFDM detection on MI355X.

The functions named ``ocd_*`` mirror the C ABI declared in ``include/ocd.h``
one to one; they only marshal torch device tensors into pointers, check that
every buffer is large enough for the problem, and pass torch's current HIP
stream.  All arithmetic runs in the HIP kernels of ``libocd.so``; there is no
other implementation and no fallback: if the library is not built, importing
this package raises.

Convenience wrappers (:func:`detect`, :func:`preprocess`, :func:`backward`,
:func:`detect_jobs`) allocate outputs with torch and return them.

Tensor conventions (device tensors, C-contiguous):

* FP32 storage: ``H`` complex64 ``[W, U, B]``, ``y`` complex64 ``[W, S, B]``
  (float32 with a trailing dimension of 2 is accepted too).
* FP16 storage: ``H`` float16 ``[W, U, B, 2]``, ``y`` float16 ``[W, S, B, 2]``.
* ``z`` complex64 ``[W, S, U]``, ``llr`` float32 ``[W, S, U, Q]``,
  ``z_hist`` complex64 ``[W, S, K, U]``, ``lam`` float32 ``[K]``.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

__all__ = [
    "Problem", "Plan", "OCDError", "MODES", "STORAGES", "LIB_PATH",
    "ocd_status_str", "ocd_version", "ocd_preprocess", "ocd_detect",
    "ocd_backward_workspace_bytes", "ocd_detect_backward", "ocd_detect_backward_bce",
    "ocd_detect_backward_bce_noalloc", "ocd_detect_train_bce", "ocd_train_plan",
    "ocd_autotune_train", "ocd_probe_fma",
    "ocd_get_plan", "ocd_set_plan",
    "ocd_autotune", "ocd_autotune_inputs", "ocd_autotune_backward", "ocd_jobs_workspace_bytes",
    "ocd_detect_jobs",
    "ocd_release_graphs", "ocd_detect_mmse", "ocd_detect_fixed", "ocd_ofdm_demodulate",
    "OfdmShape", "ofdm_demodulate",
    "problem", "detect", "preprocess", "backward", "train_step", "detect_jobs", "detect_mmse", "detect_fixed",
    "OCD_JOBS_GRAPH",
    "OCD_JOBS_TUNE",
    "OCD_JOBS_PERSISTENT", "OCD_JOBS_LANE_MODE", "JobsCall", "ocd_jobs_schedule",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libocd.so")

MODES = {"mmse": 0, "box": 1, "hybrid": 2}
STORAGES = {"f32": 0, "f16": 1}
OCD_JOBS_GRAPH = 1
OCD_JOBS_TUNE = 2
OCD_JOBS_PERSISTENT = 4


def OCD_JOBS_LANE_MODE(m):
    """ocd_detect_jobs flag: run lane mode m (0, 1, 2) instead of the tuned one."""
    return (m + 1) << 4

_STATUS = {0: "OCD_OK", -1: "OCD_EINVAL", -2: "OCD_EUNSUPPORTED", -3: "OCD_EDEVICE",
           -4: "OCD_ESCRATCH"}


class Problem(ctypes.Structure):
    """``ocd_problem``: B, U, W, S, Q, K, mode, storage, N0, Es, beta."""

    _fields_ = [("B", ctypes.c_int), ("U", ctypes.c_int), ("W", ctypes.c_int), ("S", ctypes.c_int),
                ("Q", ctypes.c_int), ("K", ctypes.c_int), ("mode", ctypes.c_int),
                ("storage", ctypes.c_int), ("N0", ctypes.c_float), ("Es", ctypes.c_float),
                ("beta", ctypes.c_float)]

    def __repr__(self):
        return ("Problem(B=%d, U=%d, W=%d, S=%d, Q=%d, K=%d, mode=%d, storage=%d, N0=%g, Es=%g, "
                "beta=%g)" % (self.B, self.U, self.W, self.S, self.Q, self.K, self.mode,
                              self.storage, self.N0, self.Es, self.beta))


class Plan(ctypes.Structure):
    """``ocd_plan``: lanes per vector, vectors per workgroup, XCD remap, whether
    each vector keeps its channel columns in registers instead of sharing an
    LDS-staged H_w, and the staggering of the staged loads."""

    _fields_ = [("lanes_per_vector", ctypes.c_int), ("vectors_per_block", ctypes.c_int),
                ("xcd_remap", ctypes.c_int), ("channel_in_registers", ctypes.c_int),
                ("stagger", ctypes.c_int)]

    def as_dict(self):
        return {"lanes_per_vector": self.lanes_per_vector,
                "vectors_per_block": self.vectors_per_block, "xcd_remap": self.xcd_remap,
                "channel_in_registers": self.channel_in_registers, "stagger": self.stagger}


class OfdmShape(ctypes.Structure):
    """Mirror of ocd_ofdm_shape."""
    _fields_ = [("B", ctypes.c_int), ("S", ctypes.c_int), ("N", ctypes.c_int),
                ("Ncp", ctypes.c_int), ("W", ctypes.c_int)]


class OCDError(RuntimeError):
    def __init__(self, fn, status):
        super().__init__("%s failed: %s" % (fn, _STATUS.get(status, status)))
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libocd.so is not built: run `python paper_1611_08779_amd/build.py` "
                          "(or __graft_entry__.build()) first")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(Problem)
    vp, fp, sz = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t
    sigs = {
        "ocd_status_str": ([ctypes.c_int], ctypes.c_char_p),
        "ocd_version": ([], ctypes.c_int),
        "ocd_preprocess": ([P, vp, fp, fp, fp, fp, vp], ctypes.c_int),
        "ocd_detect": ([P, vp, vp, fp, fp, fp, fp, fp, fp, fp, vp], ctypes.c_int),
        "ocd_backward_workspace_bytes": ([P], sz),
        "ocd_detect_backward": ([P, vp, vp, fp, fp, fp, fp, fp, fp, vp, sz, vp], ctypes.c_int),
        "ocd_detect_backward_bce": ([P, vp, vp, fp, fp, vp, fp, fp, fp, vp, sz, vp], ctypes.c_int),
        "ocd_detect_backward_bce_noalloc": ([P, vp, vp, fp, fp, vp, fp, fp, fp, vp], ctypes.c_int),
        "ocd_detect_train_bce": ([P, vp, vp, fp, vp, fp, fp, fp, fp, fp, fp, vp, sz, vp],
                                 ctypes.c_int),
        "ocd_train_plan": ([P, ctypes.POINTER(Plan)], ctypes.c_int),
        "ocd_autotune_train": ([P, vp, vp, fp, vp, fp, fp, fp, fp, vp, sz, ctypes.c_int,
                                ctypes.POINTER(Plan), vp], ctypes.c_int),
        "ocd_get_plan": ([P, ctypes.POINTER(Plan)], ctypes.c_int),
        "ocd_set_plan": ([P, ctypes.POINTER(Plan)], ctypes.c_int),
        "ocd_autotune": ([P, vp, vp, fp, fp, ctypes.c_int, ctypes.POINTER(Plan), vp], ctypes.c_int),
        "ocd_autotune_inputs": ([P, ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(vp), fp, fp,
                                 ctypes.c_int, ctypes.POINTER(Plan), vp], ctypes.c_int),
        "ocd_autotune_backward": ([P, vp, vp, fp, fp, fp, fp, fp, fp, vp, sz, ctypes.c_int,
                                   ctypes.POINTER(Plan), vp], ctypes.c_int),
        "ocd_jobs_workspace_bytes": ([P, ctypes.c_int], sz),
        "ocd_detect_jobs": ([P, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                             ctypes.POINTER(vp), ctypes.c_int, vp, sz, ctypes.c_int, vp], ctypes.c_int),
        "ocd_release_graphs": ([], None),
        "ocd_jobs_schedule": ([P, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                               ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)],
                              ctypes.c_int),
        "ocd_detect_mmse": ([P, vp, vp, fp, fp, ctypes.POINTER(Plan), vp], ctypes.c_int),
        "ocd_detect_fixed": ([P, vp, vp, vp, fp, vp], ctypes.c_int),
        "ocd_ofdm_demodulate": ([ctypes.POINTER(OfdmShape), vp, vp, vp], ctypes.c_int),
        "ocd_probe_fma": ([ctypes.c_int, ctypes.c_int, vp, ctypes.POINTER(ctypes.c_double), vp],
                          ctypes.c_int),
    }
    for name, (args, res) in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


_lib = _load()


# ---------------------------------------------------------------- marshalling

def _stream(stream=None):
    if stream is not None:
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_ptr(t, name, dtypes, nbytes_min, device=None):
    """Pointer of a contiguous device tensor of an allowed dtype holding >= nbytes_min."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if t.device.type != "cuda":
        raise ValueError("%s must be a device tensor (got %s)" % (name, t.device))
    if device is not None and t.device != device:
        raise ValueError("%s is on %s, expected %s" % (name, t.device, device))
    if t.dtype not in dtypes:
        raise TypeError("%s has dtype %s, expected one of %s" % (name, t.dtype, dtypes))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    nbytes = t.numel() * t.element_size()
    if nbytes < nbytes_min:
        raise ValueError("%s holds %d bytes, the problem needs %d" % (name, nbytes, nbytes_min))
    return t.data_ptr()


def _check(fn, status):
    if status != 0:
        raise OCDError(fn, status)


def _in_dtypes(pb):
    return (torch.float16,) if pb.storage == 1 else (torch.complex64, torch.float32)


def _cbytes(pb):
    return 4 if pb.storage == 1 else 8


def problem(B, U, W, S, Q, K, mode="mmse", storage="f32", N0=1.0, Es=1.0, beta=0.0) -> Problem:
    return Problem(int(B), int(U), int(W), int(S), int(Q), int(K),
                   MODES[mode] if isinstance(mode, str) else int(mode),
                   STORAGES[storage] if isinstance(storage, str) else int(storage),
                   float(N0), float(Es), float(beta))


# ---------------------------------------------------------------- C ABI, one to one

def ocd_status_str(status: int) -> str:
    return _lib.ocd_status_str(int(status)).decode()


def ocd_version() -> int:
    return _lib.ocd_version()


def ocd_preprocess(pb: Problem, H, lam, g, dinv, p, stream=None) -> None:
    Kt = pb.K if lam is not None else 1
    dev = H.device
    f32 = (torch.float32,)
    st = _lib.ocd_preprocess(
        ctypes.byref(pb), _dev_ptr(H, "H", _in_dtypes(pb), pb.W * pb.U * pb.B * _cbytes(pb)),
        _dev_ptr(lam, "lam", f32, pb.K * 4, dev),
        _dev_ptr(g, "g", f32, pb.W * pb.U * 4, dev),
        _dev_ptr(dinv, "dinv", f32, pb.W * Kt * pb.U * 4, dev),
        _dev_ptr(p, "p", f32, pb.W * Kt * pb.U * 4, dev), _stream(stream))
    _check("ocd_preprocess", st)


def ocd_detect(pb: Problem, H, y, lam=None, g=None, dinv=None, p=None, z=None, llr=None,
               z_hist=None, stream=None) -> None:
    Kt = pb.K if lam is not None else 1
    dev = H.device
    f32 = (torch.float32,)
    zt = (torch.complex64, torch.float32)
    st = _lib.ocd_detect(
        ctypes.byref(pb), _dev_ptr(H, "H", _in_dtypes(pb), pb.W * pb.U * pb.B * _cbytes(pb)),
        _dev_ptr(y, "y", _in_dtypes(pb), pb.W * pb.S * pb.B * _cbytes(pb), dev),
        _dev_ptr(lam, "lam", f32, pb.K * 4, dev),
        _dev_ptr(g, "g", f32, pb.W * pb.U * 4, dev),
        _dev_ptr(dinv, "dinv", f32, pb.W * Kt * pb.U * 4, dev),
        _dev_ptr(p, "p", f32, pb.W * Kt * pb.U * 4, dev),
        _dev_ptr(z, "z", zt, pb.W * pb.S * pb.U * 8, dev),
        _dev_ptr(llr, "llr", f32, pb.W * pb.S * pb.U * pb.Q * 4, dev),
        _dev_ptr(z_hist, "z_hist", zt, pb.W * pb.S * pb.K * pb.U * 8, dev), _stream(stream))
    _check("ocd_detect", st)


def ocd_backward_workspace_bytes(pb: Problem) -> int:
    return int(_lib.ocd_backward_workspace_bytes(ctypes.byref(pb)))


def ocd_detect_backward(pb: Problem, H, y, lam, z_hist, dllr, dlam, dbeta, dy, workspace,
                        stream=None) -> None:
    dev = H.device
    f32 = (torch.float32,)
    zt = (torch.complex64, torch.float32)
    ws_need = ocd_backward_workspace_bytes(pb)
    st = _lib.ocd_detect_backward(
        ctypes.byref(pb), _dev_ptr(H, "H", _in_dtypes(pb), pb.W * pb.U * pb.B * _cbytes(pb)),
        _dev_ptr(y, "y", _in_dtypes(pb), pb.W * pb.S * pb.B * _cbytes(pb), dev),
        _dev_ptr(lam, "lam", f32, pb.K * 4, dev),
        _dev_ptr(z_hist, "z_hist", zt, pb.W * pb.S * pb.K * pb.U * 8, dev),
        _dev_ptr(dllr, "dllr", f32, pb.W * pb.S * pb.U * pb.Q * 4, dev),
        _dev_ptr(dlam, "dlam", f32, pb.K * 4, dev),
        _dev_ptr(dbeta, "dbeta", f32, 4, dev),
        _dev_ptr(dy, "dy", zt, pb.W * pb.S * pb.B * 8, dev),
        _dev_ptr(workspace, "workspace", (torch.uint8,), ws_need, dev), ws_need, _stream(stream))
    _check("ocd_detect_backward", st)


def ocd_detect_backward_bce(pb: Problem, H, y, lam, z_hist, bits, dlam, dbeta, dy, workspace,
                            stream=None) -> None:
    """ocd_detect_backward for the mean BCE of the LLRs: bits (uint8 [W,S,U,Q]) in
    place of dLoss/dLLR, which the adjoint kernel forms itself."""
    dev = H.device
    f32 = (torch.float32,)
    zt = (torch.complex64, torch.float32)
    ws_need = ocd_backward_workspace_bytes(pb)
    st = _lib.ocd_detect_backward_bce(
        ctypes.byref(pb), _dev_ptr(H, "H", _in_dtypes(pb), pb.W * pb.U * pb.B * _cbytes(pb)),
        _dev_ptr(y, "y", _in_dtypes(pb), pb.W * pb.S * pb.B * _cbytes(pb), dev),
        _dev_ptr(lam, "lam", f32, pb.K * 4, dev),
        _dev_ptr(z_hist, "z_hist", zt, pb.W * pb.S * pb.K * pb.U * 8, dev),
        _dev_ptr(bits, "bits", (torch.uint8,), pb.W * pb.S * pb.U * pb.Q, dev),
        _dev_ptr(dlam, "dlam", f32, pb.K * 4, dev),
        _dev_ptr(dbeta, "dbeta", f32, 4, dev),
        _dev_ptr(dy, "dy", zt, pb.W * pb.S * pb.B * 8, dev),
        _dev_ptr(workspace, "workspace", (torch.uint8,), ws_need, dev), ws_need, _stream(stream))
    _check("ocd_detect_backward_bce", st)


def ocd_detect_backward_bce_noalloc(pb: Problem, H, y, lam, z_hist, bits, dlam, dbeta, dy,
                                    stream=None) -> None:
    """ocd_detect_backward_bce with its scratch in the library's static device array
    instead of a workspace (for callers that cannot allocate device memory)."""
    dev = H.device
    f32 = (torch.float32,)
    zt = (torch.complex64, torch.float32)
    st = _lib.ocd_detect_backward_bce_noalloc(
        ctypes.byref(pb), _dev_ptr(H, "H", _in_dtypes(pb), pb.W * pb.U * pb.B * _cbytes(pb)),
        _dev_ptr(y, "y", _in_dtypes(pb), pb.W * pb.S * pb.B * _cbytes(pb), dev),
        _dev_ptr(lam, "lam", f32, pb.K * 4, dev),
        _dev_ptr(z_hist, "z_hist", zt, pb.W * pb.S * pb.K * pb.U * 8, dev),
        _dev_ptr(bits, "bits", (torch.uint8,), pb.W * pb.S * pb.U * pb.Q, dev),
        _dev_ptr(dlam, "dlam", f32, pb.K * 4, dev),
        _dev_ptr(dbeta, "dbeta", f32, 4, dev),
        _dev_ptr(dy, "dy", zt, pb.W * pb.S * pb.B * 8, dev), _stream(stream))
    _check("ocd_detect_backward_bce_noalloc", st)


def ocd_detect_train_bce(pb: Problem, H, y, lam, bits, z, llr, loss, dlam, dbeta, dy, workspace,
                         stream=None) -> None:
    """One training step in one launch: detection, the mean BCE of the LLRs against
    bits (uint8 [W,S,U,Q]) into loss [1], and its gradients dlam, dbeta, dy."""
    dev = H.device
    f32 = (torch.float32,)
    zt = (torch.complex64, torch.float32)
    ws_need = ocd_backward_workspace_bytes(pb)
    st = _lib.ocd_detect_train_bce(
        ctypes.byref(pb), _dev_ptr(H, "H", _in_dtypes(pb), pb.W * pb.U * pb.B * _cbytes(pb)),
        _dev_ptr(y, "y", _in_dtypes(pb), pb.W * pb.S * pb.B * _cbytes(pb), dev),
        _dev_ptr(lam, "lam", f32, pb.K * 4, dev),
        _dev_ptr(bits, "bits", (torch.uint8,), pb.W * pb.S * pb.U * pb.Q, dev),
        _dev_ptr(z, "z", zt, pb.W * pb.S * pb.U * 8, dev),
        _dev_ptr(llr, "llr", f32, pb.W * pb.S * pb.U * pb.Q * 4, dev),
        _dev_ptr(loss, "loss", f32, 4, dev),
        _dev_ptr(dlam, "dlam", f32, pb.K * 4, dev),
        _dev_ptr(dbeta, "dbeta", f32, 4, dev),
        _dev_ptr(dy, "dy", zt, pb.W * pb.S * pb.B * 8, dev),
        _dev_ptr(workspace, "workspace", (torch.uint8,), ws_need, dev), ws_need, _stream(stream))
    _check("ocd_detect_train_bce", st)


def ocd_autotune_train(pb: Problem, H, y, lam, bits, loss, dlam, dbeta, dy, workspace, repeats=5,
                       stream=None) -> Plan:
    """Times the valid training-step plans, caches the fastest for the shape."""
    dev = H.device
    f32 = (torch.float32,)
    zt = (torch.complex64, torch.float32)
    ws_need = ocd_backward_workspace_bytes(pb)
    best = Plan()
    st = _lib.ocd_autotune_train(
        ctypes.byref(pb), _dev_ptr(H, "H", _in_dtypes(pb), pb.W * pb.U * pb.B * _cbytes(pb)),
        _dev_ptr(y, "y", _in_dtypes(pb), pb.W * pb.S * pb.B * _cbytes(pb), dev),
        _dev_ptr(lam, "lam", f32, pb.K * 4, dev),
        _dev_ptr(bits, "bits", (torch.uint8,), pb.W * pb.S * pb.U * pb.Q, dev),
        _dev_ptr(loss, "loss", f32, 4, dev),
        _dev_ptr(dlam, "dlam", f32, pb.K * 4, dev),
        _dev_ptr(dbeta, "dbeta", f32, 4, dev),
        _dev_ptr(dy, "dy", zt, pb.W * pb.S * pb.B * 8, dev),
        _dev_ptr(workspace, "workspace", (torch.uint8,), ws_need, dev), ws_need, int(repeats),
        ctypes.byref(best), _stream(stream))
    _check("ocd_autotune_train", st)
    return best


def ocd_train_plan(pb: Problem) -> Plan:
    pl = Plan()
    _check("ocd_train_plan", _lib.ocd_train_plan(ctypes.byref(pb), ctypes.byref(pl)))
    return pl


def ocd_get_plan(pb: Problem) -> Plan:
    pl = Plan()
    _check("ocd_get_plan", _lib.ocd_get_plan(ctypes.byref(pb), ctypes.byref(pl)))
    return pl


def ocd_set_plan(pb: Problem, plan: Plan) -> None:
    _check("ocd_set_plan", _lib.ocd_set_plan(ctypes.byref(pb), ctypes.byref(plan)))


def ocd_autotune(pb: Problem, H, y, z, llr, repeats=5, stream=None) -> Plan:
    dev = H.device
    pl = Plan()
    st = _lib.ocd_autotune(
        ctypes.byref(pb), _dev_ptr(H, "H", _in_dtypes(pb), pb.W * pb.U * pb.B * _cbytes(pb)),
        _dev_ptr(y, "y", _in_dtypes(pb), pb.W * pb.S * pb.B * _cbytes(pb), dev),
        _dev_ptr(z, "z", (torch.complex64, torch.float32), pb.W * pb.S * pb.U * 8, dev),
        _dev_ptr(llr, "llr", (torch.float32,), pb.W * pb.S * pb.U * pb.Q * 4, dev),
        int(repeats), ctypes.byref(pl), _stream(stream))
    _check("ocd_autotune", st)
    return pl


def ocd_autotune_inputs(pb: Problem, Hs, ys, z, llr, repeats=2, stream=None) -> Plan:
    """``ocd_autotune`` over several input sets (sequences of H and y tensors of the
    problem's shape, one device), each candidate timed over `repeats` passes
    through all of them."""
    if len(Hs) != len(ys) or not Hs:
        raise ValueError("ocd_autotune_inputs: Hs and ys must be non-empty and of equal length")
    dev = Hs[0].device
    n = len(Hs)
    hp = (ctypes.c_void_p * n)(*[_dev_ptr(H, "H", _in_dtypes(pb), pb.W * pb.U * pb.B * _cbytes(pb), dev)
                                 for H in Hs])
    yp = (ctypes.c_void_p * n)(*[_dev_ptr(y, "y", _in_dtypes(pb), pb.W * pb.S * pb.B * _cbytes(pb), dev)
                                 for y in ys])
    pl = Plan()
    st = _lib.ocd_autotune_inputs(
        ctypes.byref(pb), n, hp, yp,
        _dev_ptr(z, "z", (torch.complex64, torch.float32), pb.W * pb.S * pb.U * 8, dev),
        _dev_ptr(llr, "llr", (torch.float32,), pb.W * pb.S * pb.U * pb.Q * 4, dev),
        int(repeats), ctypes.byref(pl), _stream(stream))
    _check("ocd_autotune_inputs", st)
    return pl


def ocd_autotune_backward(pb: Problem, H, y, lam, z_hist, dllr, dlam, dbeta, dy, workspace,
                          repeats=5, stream=None) -> Plan:
    dev = H.device
    f32 = (torch.float32,)
    zt = (torch.complex64, torch.float32)
    ws_need = ocd_backward_workspace_bytes(pb)
    pl = Plan()
    st = _lib.ocd_autotune_backward(
        ctypes.byref(pb), _dev_ptr(H, "H", _in_dtypes(pb), pb.W * pb.U * pb.B * _cbytes(pb)),
        _dev_ptr(y, "y", _in_dtypes(pb), pb.W * pb.S * pb.B * _cbytes(pb), dev),
        _dev_ptr(lam, "lam", f32, pb.K * 4, dev),
        _dev_ptr(z_hist, "z_hist", zt, pb.W * pb.S * pb.K * pb.U * 8, dev),
        _dev_ptr(dllr, "dllr", f32, pb.W * pb.S * pb.U * pb.Q * 4, dev),
        _dev_ptr(dlam, "dlam", f32, pb.K * 4, dev),
        _dev_ptr(dbeta, "dbeta", f32, 4, dev),
        _dev_ptr(dy, "dy", zt, pb.W * pb.S * pb.B * 8, dev),
        _dev_ptr(workspace, "workspace", (torch.uint8,), ws_need, dev), ws_need, int(repeats),
        ctypes.byref(pl), _stream(stream))
    _check("ocd_autotune_backward", st)
    return pl


def ocd_detect_mmse(pb: Problem, H, y, z=None, llr=None, plan=None, stream=None) -> None:
    dev = H.device
    st = _lib.ocd_detect_mmse(
        ctypes.byref(pb), _dev_ptr(H, "H", _in_dtypes(pb), pb.W * pb.U * pb.B * _cbytes(pb)),
        _dev_ptr(y, "y", _in_dtypes(pb), pb.W * pb.S * pb.B * _cbytes(pb), dev),
        _dev_ptr(z, "z", (torch.complex64, torch.float32), pb.W * pb.S * pb.U * 8, dev),
        _dev_ptr(llr, "llr", (torch.float32,), pb.W * pb.S * pb.U * pb.Q * 4, dev),
        ctypes.byref(plan) if plan is not None else None, _stream(stream))
    _check("ocd_detect_mmse", st)


def ocd_detect_fixed(pb: Problem, H, y, z=None, llr=None, stream=None) -> None:
    dev = H.device
    i16 = (torch.int16,)
    st = _lib.ocd_detect_fixed(
        ctypes.byref(pb), _dev_ptr(H, "H", i16, pb.W * pb.U * pb.B * 4),
        _dev_ptr(y, "y", i16, pb.W * pb.S * pb.B * 4, dev),
        _dev_ptr(z, "z", i16, pb.W * pb.S * pb.U * 4, dev),
        _dev_ptr(llr, "llr", (torch.float32,), pb.W * pb.S * pb.U * pb.Q * 4, dev), _stream(stream))
    _check("ocd_detect_fixed", st)


def ocd_ofdm_demodulate(sh: OfdmShape, x, y, stream=None) -> None:
    c = (torch.complex64, torch.float32)
    st = _lib.ocd_ofdm_demodulate(
        ctypes.byref(sh), _dev_ptr(x, "x", c, sh.B * sh.S * (sh.Ncp + sh.N) * 8),
        _dev_ptr(y, "y", c, sh.W * sh.S * sh.B * 8, x.device), _stream(stream))
    _check("ocd_ofdm_demodulate", st)


def _problem_array(jobs):
    arr = (Problem * len(jobs))()
    for i, pb in enumerate(jobs):
        arr[i] = pb
    return arr


def ocd_jobs_workspace_bytes(jobs) -> int:
    arr = _problem_array(jobs)
    return int(_lib.ocd_jobs_workspace_bytes(arr, len(jobs)))


class JobsCall:
    """Arguments of ``ocd_detect_jobs`` marshalled once, for repeated launches on the
    same buffers (the batched form is meant to be replayed; checking 4 tensors per
    job on every call would cost more host time than the launch)."""

    def __init__(self, jobs, H, y, z, llr, workspace, flags=0):
        n = len(jobs)
        self.n = n
        self.arr = _problem_array(jobs)
        self.ptrs = [(ctypes.c_void_p * n)() for _ in range(4)]
        dev = H[0].device
        for j, pb in enumerate(jobs):
            self.ptrs[0][j] = _dev_ptr(H[j], "H[%d]" % j, _in_dtypes(pb), pb.W * pb.U * pb.B * _cbytes(pb), dev)
            self.ptrs[1][j] = _dev_ptr(y[j], "y[%d]" % j, _in_dtypes(pb), pb.W * pb.S * pb.B * _cbytes(pb), dev)
            self.ptrs[2][j] = _dev_ptr(z[j] if z is not None else None, "z[%d]" % j,
                                       (torch.complex64, torch.float32), pb.W * pb.S * pb.U * 8, dev)
            self.ptrs[3][j] = _dev_ptr(llr[j] if llr is not None else None, "llr[%d]" % j,
                                       (torch.float32,), pb.W * pb.S * pb.U * pb.Q * 4, dev)
        self.ws_need = ocd_jobs_workspace_bytes(jobs)
        if self.ws_need == 0:
            raise OCDError("ocd_jobs_workspace_bytes", -1)
        self.wsp = _dev_ptr(workspace, "workspace", (torch.uint8,), self.ws_need, dev)
        if self.wsp % 256:
            raise ValueError("workspace must be 256-byte aligned")
        self.has_z, self.has_llr = z is not None, llr is not None
        self.flags = int(flags)
        self._keep = (H, y, z, llr, workspace)   # the buffers must outlive the call object

    def __call__(self, flags=None, stream=None):
        st = _lib.ocd_detect_jobs(self.arr, self.ptrs[0], self.ptrs[1],
                                  self.ptrs[2] if self.has_z else None,
                                  self.ptrs[3] if self.has_llr else None, self.n, self.wsp,
                                  self.ws_need, self.flags if flags is None else int(flags),
                                  _stream(stream))
        _check("ocd_detect_jobs", st)


def ocd_detect_jobs(jobs, H, y, z, llr, workspace, flags=0, stream=None) -> None:
    JobsCall(jobs, H, y, z, llr, workspace, flags)(stream=stream)


def ocd_jobs_schedule(jobs) -> dict:
    """The schedule ocd_detect_jobs runs for this list of shapes (the tuned one, else
    the default): persistent or one workgroup per tile, tile policy, lane mode."""
    arr = _problem_array(jobs)
    pers, pol, mode = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check("ocd_jobs_schedule", _lib.ocd_jobs_schedule(arr, len(jobs), ctypes.byref(pers),
                                                       ctypes.byref(pol), ctypes.byref(mode)))
    return {"persistent": pers.value, "tile_policy": pol.value, "lane_mode": mode.value}


def ocd_probe_fma(blocks, iters, out, stream=None) -> float:
    """Launches the FP32 FMA-rate probe; returns the launch's flop count."""
    fl = ctypes.c_double(0.0)
    _check("ocd_probe_fma", _lib.ocd_probe_fma(int(blocks), int(iters),
                                               _dev_ptr(out, "out", (torch.float32,), 1024),
                                               ctypes.byref(fl), _stream(stream)))
    return fl.value


def ocd_release_graphs() -> None:
    _lib.ocd_release_graphs()


# ---------------------------------------------------------------- convenience

def _shape_of(H, y, storage):
    if storage == "f16" or (isinstance(storage, int) and storage == 1):
        W, U, B = H.shape[:3]
        S = y.shape[1]
    elif H.dtype == torch.complex64:
        W, U, B = H.shape
        S = y.shape[1]
    else:
        W, U, B = H.shape[:3]
        S = y.shape[1]
    return W, U, B, S


def preprocess(H, K, Q, mode="mmse", N0=1.0, Es=1.0, lam=None, storage="f32", stream=None):
    """Returns (g [W,U], dinv [W,Kt,U], p [W,Kt,U])."""
    W, U, B = H.shape[:3]
    pb = problem(B, U, W, 1, Q, K, mode, storage, N0, Es)
    Kt = K if lam is not None else 1
    g = torch.empty(W, U, device=H.device, dtype=torch.float32)
    dinv = torch.empty(W, Kt, U, device=H.device, dtype=torch.float32)
    p = torch.empty(W, Kt, U, device=H.device, dtype=torch.float32)
    ocd_preprocess(pb, H, lam, g, dinv, p, stream)
    return g, dinv, p


def detect(H, y, K, Q, mode="mmse", N0=1.0, Es=1.0, beta=0.0, lam=None, storage="f32",
           want_z=True, want_llr=True, want_hist=False, pre=None, stream=None):
    """Runs ocd_detect; returns (z, llr, z_hist) with None for outputs not asked for."""
    W, U, B, S = _shape_of(H, y, storage)
    pb = problem(B, U, W, S, Q, K, mode, storage, N0, Es, beta)
    dev = H.device
    z = torch.empty(W, S, U, device=dev, dtype=torch.complex64) if want_z else None
    llr = torch.empty(W, S, U, Q, device=dev, dtype=torch.float32) if want_llr else None
    zh = torch.empty(W, S, K, U, device=dev, dtype=torch.complex64) if want_hist else None
    g, dinv, p = pre if pre is not None else (None, None, None)
    ocd_detect(pb, H, y, lam, g, dinv, p, z, llr, zh, stream)
    return z, llr, zh


def backward(H, y, z_hist, dllr, K, Q, mode="mmse", N0=1.0, Es=1.0, beta=0.0, lam=None,
             storage="f32", want_dy=True, stream=None, bits=None):
    """Runs ocd_detect_backward (or, with dllr None and bits given, the fused
    cross-entropy form ocd_detect_backward_bce); returns (dlam [K], dbeta [1],
    dy [W,S,B] or None)."""
    W, U, B, S = _shape_of(H, y, storage)
    pb = problem(B, U, W, S, Q, K, mode, storage, N0, Es, beta)
    dev = H.device
    dlam = torch.empty(K, device=dev, dtype=torch.float32)
    dbeta = torch.empty(1, device=dev, dtype=torch.float32)
    dy = torch.empty(W, S, B, device=dev, dtype=torch.complex64) if want_dy else None
    ws = torch.zeros(ocd_backward_workspace_bytes(pb), device=dev, dtype=torch.uint8)   # counter starts at 0
    if dllr is None:
        ocd_detect_backward_bce(pb, H, y, lam, z_hist, bits, dlam, dbeta, dy, ws, stream)
    else:
        ocd_detect_backward(pb, H, y, lam, z_hist, dllr, dlam, dbeta, dy, ws, stream)
    return dlam, dbeta, dy


def train_step(H, y, bits, K, Q, mode="hybrid", N0=1.0, Es=1.0, beta=0.0, lam=None,
               storage="f32", want_z=False, want_llr=False, want_dy=True, workspace=None,
               stream=None):
    """Runs ocd_detect_train_bce; returns (loss [1], dlam [K], dbeta [1], dy or None,
    z or None, llr or None)."""
    W, U, B, S = _shape_of(H, y, storage)
    pb = problem(B, U, W, S, Q, K, mode, storage, N0, Es, beta)
    dev = H.device
    loss = torch.empty(1, device=dev, dtype=torch.float32)
    dlam = torch.empty(K, device=dev, dtype=torch.float32)
    dbeta = torch.empty(1, device=dev, dtype=torch.float32)
    dy = torch.empty(W, S, B, device=dev, dtype=torch.complex64) if want_dy else None
    z = torch.empty(W, S, U, device=dev, dtype=torch.complex64) if want_z else None
    llr = torch.empty(W, S, U, Q, device=dev, dtype=torch.float32) if want_llr else None
    ws = workspace
    if ws is None:   # the completion counter starts at zero
        ws = torch.zeros(ocd_backward_workspace_bytes(pb), device=dev, dtype=torch.uint8)
    ocd_detect_train_bce(pb, H, y, lam, bits, z, llr, loss, dlam, dbeta, dy, ws, stream)
    return loss, dlam, dbeta, dy, z, llr


def detect_mmse(H, y, Q, N0=1.0, Es=1.0, storage="f32", want_z=True, want_llr=True, plan=None,
                stream=None):
    """Runs ocd_detect_mmse (explicit MMSE, exact soft output); returns (z, llr) with None
    for outputs not asked for.  plan: a Plan, an (L, vectors_per_block[, xcd[, stagger]])
    tuple or None."""
    W, U, B, S = _shape_of(H, y, storage)
    pb = problem(B, U, W, S, Q, 1, "mmse", storage, N0, Es)
    dev = H.device
    z = torch.empty(W, S, U, device=dev, dtype=torch.complex64) if want_z else None
    llr = torch.empty(W, S, U, Q, device=dev, dtype=torch.float32) if want_llr else None
    if plan is not None and not isinstance(plan, Plan):
        plan = Plan(int(plan[0]), int(plan[1]), int(plan[2]) if len(plan) > 2 else 0, 0,
                    int(plan[3]) if len(plan) > 3 else 0)
    ocd_detect_mmse(pb, H, y, z, llr, plan, stream)
    return z, llr


def detect_fixed(H, y, K, Q, mode="mmse", N0=1.0, Es=1.0, beta=0.0, want_z=True, want_llr=True,
                 stream=None):
    """Runs ocd_detect_fixed on int16 Q5.11 pairs H [W,U,B,2], y [W,S,B,2]; returns
    (z int16 [W,S,U,2], llr [W,S,U,Q]) with None for outputs not asked for."""
    if H.dim() != 4 or y.dim() != 4 or H.shape[-1] != 2 or y.shape[-1] != 2:
        raise ValueError("H and y must be int16 [W,U,B,2] and [W,S,B,2]")
    W, U, B, _ = H.shape
    S = y.shape[1]
    pb = problem(B, U, W, S, Q, K, mode, "f32", N0, Es, beta)
    dev = H.device
    z = torch.empty(W, S, U, 2, device=dev, dtype=torch.int16) if want_z else None
    llr = torch.empty(W, S, U, Q, device=dev, dtype=torch.float32) if want_llr else None
    ocd_detect_fixed(pb, H, y, z, llr, stream)
    return z, llr


def ofdm_demodulate(x, N, Ncp, W, stream=None):
    """Runs ocd_ofdm_demodulate: time-domain x complex64 [B,S,Ncp+N] -> y complex64
    [W,S,B], the detector's receive-vector layout."""
    if x.dim() != 3 or x.shape[-1] != Ncp + N:
        raise ValueError("x must be [B, S, Ncp + N]")
    B, S, _ = x.shape
    y = torch.empty(W, S, B, device=x.device, dtype=torch.complex64)
    ocd_ofdm_demodulate(OfdmShape(B, S, N, Ncp, W), x, y, stream)
    return y


def detect_jobs(jobs, H, y, flags=0, workspace=None, stream=None):
    """Runs ocd_detect_jobs on a list of Problems; returns (z list, llr list, workspace)."""
    dev = H[0].device
    z = [torch.empty(pb.W, pb.S, pb.U, device=dev, dtype=torch.complex64) for pb in jobs]
    llr = [torch.empty(pb.W, pb.S, pb.U, pb.Q, device=dev, dtype=torch.float32) for pb in jobs]
    if workspace is None:
        workspace = torch.empty(ocd_jobs_workspace_bytes(jobs) + 256, device=dev, dtype=torch.uint8)
    ocd_detect_jobs(jobs, H, y, z, llr, workspace, flags, stream)
    return z, llr, workspace
