"""FP64 CPU oracle for OCD detection -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The HIP detector never imports it, and
the two share no code.  The arithmetic lives in ``ocd_oracle.c`` (plain C99,
``double complex``); this module compiles it with gcc and marshals numpy
arrays through ctypes.  See the header of ``ocd_oracle.c`` for the passages
of the paper that each function follows and for what pins it.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ocd_oracle.c")
_LIB = os.path.join(_HERE, "libocd_oracle.so")

MODES = {"mmse": 0, "box": 1, "hybrid": 2}

_lib = None


def build(force: bool = True) -> str:
    """Compile ``ocd_oracle.c`` into ``libocd_oracle.so`` (gcc, FP64, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
               _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _open(path):
    """Open a compiled oracle library and declare its C signatures."""
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    i, d = ctypes.c_int, ctypes.c_double
    common = [i, i, i, i, i, i, i, d, d, dp, d]
    lib.oracle_ocd.argtypes = common + [dp, dp, dp, dp, i]
    lib.oracle_cd.argtypes = common + [dp, dp, dp, i]
    lib.oracle_llr.argtypes = common + [dp, dp, dp, i]
    lib.oracle_detect.argtypes = common + [dp, dp, dp, dp, i]
    lib.oracle_hard.argtypes = common + [dp, dp, ctypes.POINTER(ctypes.c_ubyte)]
    lib.oracle_grad.argtypes = common + [dp, dp, dp, dp, dp, dp]
    i8 = ctypes.POINTER(ctypes.c_int8)
    lib.oracle_active_set.argtypes = common + [dp, dp, i8, i8]
    lib.oracle_ocd_trace.argtypes = [i, i, i, i, i, d, d, dp, d, dp, dp, dp]
    lib.oracle_constellation.argtypes = [i, dp, ctypes.POINTER(ctypes.c_uint)]
    lib.oracle_mmse.argtypes = [i, i, i, i, i, d, d, dp, dp, dp, dp, dp, i]
    sp = ctypes.POINTER(ctypes.c_int16)
    lib.oracle_ocd_fixed.argtypes = [i, i, i, i, i, i, i, d, d, d, sp, sp, sp, dp, i]
    lib.oracle_fx_recip.argtypes = [ctypes.c_int64]
    lib.oracle_fx_recip.restype = ctypes.c_int64
    for f in ("oracle_ocd", "oracle_cd", "oracle_llr", "oracle_detect", "oracle_hard",
              "oracle_grad", "oracle_active_set", "oracle_ocd_trace", "oracle_constellation", "oracle_mmse",
              "oracle_ocd_fixed"):
        getattr(lib, f).restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        _lib = _open(_LIB)
    return _lib


def _c128(a):
    return np.ascontiguousarray(np.asarray(a), dtype=np.complex128)


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _lam(lam, K):
    if lam is None:
        return None
    lam = np.ascontiguousarray(np.asarray(lam, dtype=np.float64).reshape(-1))
    if lam.size != K:
        raise ValueError("lambda must have K entries")
    return lam


def _common(H, y_or_z_shape_S, K, Q, mode, N0, Es, lam, beta):
    W, U, B = H.shape
    return [B, U, W, y_or_z_shape_S, K, Q, MODES[mode], float(N0), float(Es), _ptr(lam),
            float(beta)]


def _threads(threads):
    if threads is None:
        return 1
    if threads <= 0:
        return len(os.sched_getaffinity(0))
    return int(threads)


def ocd(H, y, K, Q, mode="mmse", N0=1.0, Es=1.0, lam=None, beta=0.0, hist=False, threads=1):
    """Algorithm 1 (form ii).  H [W,U,B], y [W,S,B] -> z [W,S,U] (and z_hist [W,S,K,U])."""
    lib = _load()
    H, y = _c128(H), _c128(y)
    W, U, B = H.shape
    S = y.shape[1]
    lam = _lam(lam, K)
    z = np.zeros((W, S, U), np.complex128)
    zh = np.zeros((W, S, K, U), np.complex128) if hist else None
    rc = lib.oracle_ocd(*_common(H, S, K, Q, mode, N0, Es, lam, beta), _ptr(H), _ptr(y),
                        _ptr(z), _ptr(zh), _threads(threads))
    if rc:
        raise ValueError("oracle_ocd rejected its arguments")
    return (z, zh) if hist else z


def cd(H, y, K, Q, mode="mmse", N0=1.0, Es=1.0, lam=None, beta=0.0, threads=1):
    """Plain coordinate descent (form i, eq:CDrule / eq:CDruleBOX)."""
    lib = _load()
    H, y = _c128(H), _c128(y)
    W, U, B = H.shape
    S = y.shape[1]
    lam = _lam(lam, K)
    z = np.zeros((W, S, U), np.complex128)
    rc = lib.oracle_cd(*_common(H, S, K, Q, mode, N0, Es, lam, beta), _ptr(H), _ptr(y),
                       _ptr(z), _threads(threads))
    if rc:
        raise ValueError("oracle_cd rejected its arguments")
    return z


def ocd_trace(h, y, K, Q, mode="mmse", N0=1.0, Es=1.0, lam=None, beta=0.0):
    """z after every coordinate update of one vector: h [U,B], y [B] -> [K,U,U]."""
    lib = _load()
    h, y = _c128(h), _c128(y)
    U, B = h.shape
    lam = _lam(lam, K)
    tr = np.zeros((K, U, U), np.complex128)
    rc = lib.oracle_ocd_trace(B, U, K, Q, MODES[mode], float(N0), float(Es), _ptr(lam),
                              float(beta), _ptr(h), _ptr(y), _ptr(tr))
    if rc:
        raise ValueError("oracle_ocd_trace rejected its arguments")
    return tr


def llr(H, z, K, Q, mode="mmse", N0=1.0, Es=1.0, lam=None, beta=0.0, threads=1):
    """Max-log LLRs (eq:exactinversellr with Section III-C's mu, rho): [W,S,U,Q]."""
    lib = _load()
    H, z = _c128(H), _c128(z)
    W, U, B = H.shape
    S = z.shape[1]
    lam = _lam(lam, K)
    out = np.zeros((W, S, U, Q), np.float64)
    rc = lib.oracle_llr(*_common(H, S, K, Q, mode, N0, Es, lam, beta), _ptr(H), _ptr(z),
                        _ptr(out), _threads(threads))
    if rc:
        raise ValueError("oracle_llr rejected its arguments")
    return out


def hard(H, z, K, Q, mode="mmse", N0=1.0, Es=1.0, lam=None, beta=0.0):
    """Sliced bits of x = z/(mu sqrt(Es)) (eq:slicing): [W,S,U,Q] uint8."""
    lib = _load()
    H, z = _c128(H), _c128(z)
    W, U, B = H.shape
    S = z.shape[1]
    lam = _lam(lam, K)
    out = np.zeros((W, S, U, Q), np.uint8)
    rc = lib.oracle_hard(*_common(H, S, K, Q, mode, N0, Es, lam, beta), _ptr(H), _ptr(z),
                         out.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)))
    if rc:
        raise ValueError("oracle_hard rejected its arguments")
    return out


def detect(H, y, K, Q, mode="mmse", N0=1.0, Es=1.0, lam=None, beta=0.0, threads=1):
    """The whole path of one slot: returns (z, llr)."""
    lib = _load()
    H, y = _c128(H), _c128(y)
    W, U, B = H.shape
    S = y.shape[1]
    lam = _lam(lam, K)
    z = np.zeros((W, S, U), np.complex128)
    out = np.zeros((W, S, U, Q), np.float64)
    rc = lib.oracle_detect(*_common(H, S, K, Q, mode, N0, Es, lam, beta), _ptr(H), _ptr(y),
                           _ptr(z), _ptr(out), _threads(threads))
    if rc:
        raise ValueError("oracle_detect rejected its arguments")
    return z, out


def grad(H, y, dllr, K, Q, mode="mmse", N0=1.0, Es=1.0, lam=None, beta=0.0):
    """Reverse-mode reference gradient: returns (dlambda [K], dbeta, dy [W,S,B])."""
    lib = _load()
    H, y = _c128(H), _c128(y)
    W, U, B = H.shape
    S = y.shape[1]
    lam = _lam(lam, K)
    dllr = np.ascontiguousarray(dllr, dtype=np.float64)
    dlam = np.zeros(K, np.float64)
    dbeta = np.zeros(1, np.float64)
    dy = np.zeros((W, S, B), np.complex128)
    rc = lib.oracle_grad(*_common(H, S, K, Q, mode, N0, Es, lam, beta), _ptr(H), _ptr(y),
                         _ptr(dllr), _ptr(dlam), _ptr(dbeta), _ptr(dy))
    if rc:
        raise ValueError("oracle_grad rejected its arguments")
    return dlam, float(dbeta[0]), dy


def active_set(H, y, K, Q, mode="mmse", N0=1.0, Es=1.0, lam=None, beta=0.0):
    """The pieces of the path in use at these inputs: (clip [W,S,K,U,2] in {-1,0,1}, the
    side of the box of every projection; amin [W,S,U,Q,2], the two max-log minimisers of
    every bit).  The loss is smooth across a step that leaves both unchanged."""
    lib = _load()
    H, y = _c128(H), _c128(y)
    W, U, B = H.shape
    S = y.shape[1]
    lam = _lam(lam, K)
    clip = np.zeros((W, S, K, U, 2), np.int8)
    amin = np.zeros((W, S, U, Q, 2), np.int8)
    i8 = ctypes.POINTER(ctypes.c_int8)
    rc = lib.oracle_active_set(*_common(H, S, K, Q, mode, N0, Es, lam, beta), _ptr(H), _ptr(y),
                               clip.ctypes.data_as(i8), amin.ctypes.data_as(i8))
    if rc:
        raise ValueError("oracle_active_set rejected its arguments")
    return clip, amin


def constellation(Q):
    """The oracle's own unit-energy Gray QAM: (points complex [2^Q], labels [2^Q])."""
    lib = _load()
    n = 1 << Q
    pts = np.zeros(2 * n, np.float64)
    lab = np.zeros(n, np.uint32)
    rc = lib.oracle_constellation(Q, _ptr(pts), lab.ctypes.data_as(ctypes.POINTER(ctypes.c_uint)))
    if rc != n:
        raise ValueError("bad Q")
    return pts[0::2] + 1j * pts[1::2], lab


def mmse(H, y, Q, N0=1.0, Es=1.0, threads=1):
    """Explicit MMSE detection with the exact soft output (Sections II-B, II-E):
    H [W,U,B], y [W,S,B] -> z [W,S,U], llr [W,S,U,Q], mu [W,U]."""
    lib = _load()
    H, y = _c128(H), _c128(y)
    W, U, B = H.shape
    S = y.shape[1]
    z = np.zeros((W, S, U), np.complex128)
    out = np.zeros((W, S, U, Q), np.float64)
    mu = np.zeros((W, U), np.float64)
    rc = lib.oracle_mmse(B, U, W, S, Q, float(N0), float(Es), _ptr(H), _ptr(y), _ptr(z),
                         _ptr(out), _ptr(mu), _threads(threads))
    if rc:
        raise ValueError("oracle_mmse rejected its arguments")
    return z, out, mu


def _i16(a):
    return np.ascontiguousarray(np.asarray(a), dtype=np.int16)


def ocd_fixed(Hq, yq, K, Q, mode="mmse", N0=1.0, Es=1.0, beta=0.0, threads=1):
    """Algorithm 1 in the fixed-point datapath of Section IV-C (readings F1-F8 in
    ocd_oracle.c).  Hq [W,U,B,2], yq [W,S,B,2] int16 Q5.11 -> z [W,S,U,2] int16 and
    LLRs [W,S,U,Q] (floating point from the fixed-point z and p)."""
    lib = _load()
    Hq, yq = _i16(Hq), _i16(yq)
    W, U, B, _ = Hq.shape
    S = yq.shape[1]
    z = np.zeros((W, S, U, 2), np.int16)
    out = np.zeros((W, S, U, Q), np.float64)
    sp = ctypes.POINTER(ctypes.c_int16)
    rc = lib.oracle_ocd_fixed(B, U, W, S, K, Q, MODES[mode], float(N0), float(Es), float(beta),
                              Hq.ctypes.data_as(sp), yq.ctypes.data_as(sp), z.ctypes.data_as(sp),
                              _ptr(out), _threads(threads))
    if rc:
        raise ValueError("oracle_ocd_fixed rejected its arguments or a sum left 36 bits")
    return z, out


def fx_recip(x):
    """The fixed-point reciprocal unit (reading F5): Q.22 integer x -> Q.11 integer."""
    return int(_load().oracle_fx_recip(int(x)))


def ofdm_demodulate(x, N, Ncp, W):
    """OFDM demodulation at the base station (Section II-A): per antenna b and
    symbol s, drop the first Ncp samples (the cyclic prefix), take the unitary
    N-point DFT X[k] = N^-1/2 sum_n x[Ncp + n] exp(-2 pi i k n / N) (numpy's FFT in
    FP64 as the DFT), and keep the W used bins -W/2 .. -1, +1 .. +W/2 (DC empty) in
    increasing frequency.  x [B][S][Ncp + N] -> y [W][S][B] complex128."""
    x = np.asarray(x, np.complex128)
    if W % 2 or W // 2 >= N // 2 or x.shape[-1] != Ncp + N:
        raise ValueError("bad OFDM shape")
    X = np.fft.fft(x[..., Ncp:Ncp + N], axis=-1, norm="ortho")
    kneg = np.arange(N - W // 2, N)          # -W/2 .. -1
    kpos = np.arange(1, W // 2 + 1)          # +1 .. +W/2
    Y = X[..., np.concatenate([kneg, kpos])]  # [B][S][W]
    return np.ascontiguousarray(np.transpose(Y, (2, 1, 0)))
