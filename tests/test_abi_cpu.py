"""The C ABI without a GPU: libocd.so loads, exports every function declared in
include/ocd.h, and rejects invalid problems before touching the device."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ocd.h")
LIB = os.path.join(ROOT, "paper_1611_08779_amd", "libocd.so")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import importlib.util
        spec = importlib.util.spec_from_file_location(
            "ocd_hip_build", os.path.join(ROOT, "paper_1611_08779_amd", "build.py"))
        b = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(b)
        b.build()
    return ctypes.CDLL(LIB)


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(ocd_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("ocd_preprocess", "ocd_detect", "ocd_detect_backward", "ocd_detect_jobs",
                     "ocd_autotune", "ocd_status_str"):
        assert required in names


C_CALLER = r'''
#include "ocd.h"
#include <stdio.h>
int main(void)
{
    ocd_problem pb = {128, 8, 1200, 14, 6, 3, OCD_MMSE, OCD_STORE_F32, 0.01f, 1.0f, 0.0f};
    ocd_problem bad = pb;
    ocd_plan pl;
    bad.Q = 5;
    if (ocd_get_plan(&pb, &pl) != OCD_OK || pl.lanes_per_vector < 4) return 1;
    if (ocd_backward_workspace_bytes(&pb) != 256 + 16800u * 5u * 4u) return 2;
    if (ocd_get_plan(&bad, &pl) != OCD_EINVAL) return 3;
    printf("%s %d\n", ocd_status_str(OCD_OK), ocd_version());
    return 0;
}
'''


def test_header_compiles_as_c99_and_a_c_program_links(tmp_path, lib):
    """The boundary is plain C: a C99 program includes ocd.h, links libocd.so and
    calls the host-side entry points (no GPU needed for these)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "caller.c"
    src.write_text(C_CALLER)
    exe = tmp_path / "caller"
    libdir = os.path.dirname(LIB)
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Werror=implicit-function-declaration",
                        "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROOT, "include"),
                        "-I/opt/rocm/include", str(src), "-o", str(exe), "-L" + libdir, "-locd",
                        "-Wl,-rpath," + libdir], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert run.returncode == 0, (run.returncode, run.stdout, run.stderr)
    assert run.stdout.startswith("OCD_OK")


def test_every_declared_symbol_is_exported(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_python_binding_names_match_the_header():
    import paper_1611_08779_amd as ocd
    for name in _declared_functions():
        assert callable(getattr(ocd, name)), name


class Problem(ctypes.Structure):
    _fields_ = [("B", ctypes.c_int), ("U", ctypes.c_int), ("W", ctypes.c_int), ("S", ctypes.c_int),
                ("Q", ctypes.c_int), ("K", ctypes.c_int), ("mode", ctypes.c_int),
                ("storage", ctypes.c_int), ("N0", ctypes.c_float), ("Es", ctypes.c_float),
                ("beta", ctypes.c_float)]


def _good():
    return dict(B=128, U=8, W=1200, S=14, Q=6, K=3, mode=0, storage=0, N0=0.01, Es=1.0, beta=0.0)


BAD = [
    dict(B=0), dict(B=1025), dict(U=0), dict(U=33), dict(B=4, U=5), dict(W=-1), dict(S=0),
    dict(Q=3), dict(Q=8), dict(K=0), dict(K=257), dict(mode=3), dict(storage=2),
    dict(N0=0.0), dict(N0=-1.0), dict(N0=float("nan")), dict(Es=0.0), dict(Es=float("inf")),
    dict(beta=float("nan")),
]


@pytest.mark.parametrize("bad", BAD, ids=[str(b) for b in BAD])
def test_invalid_problems_are_rejected_before_any_launch(lib, bad):
    kw = _good()
    kw.update(bad)
    pb = Problem(**kw)
    lib.ocd_detect.restype = ctypes.c_int
    lib.ocd_detect.argtypes = [ctypes.POINTER(Problem)] + [ctypes.c_void_p] * 10
    dummy = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    st = lib.ocd_detect(ctypes.byref(pb), dummy, dummy, None, None, None, None, dummy, dummy,
                        None, None)
    assert st == -1


def test_status_strings_and_version(lib):
    lib.ocd_status_str.restype = ctypes.c_char_p
    assert lib.ocd_status_str(0) == b"OCD_OK"
    assert b"EINVAL" in lib.ocd_status_str(-1)
    assert b"EUNSUPPORTED" in lib.ocd_status_str(-2)
    assert b"EDEVICE" in lib.ocd_status_str(-3)
    assert lib.ocd_version() >= 10000


def test_partial_preprocessing_arguments_are_rejected(lib):
    pb = Problem(**_good())
    lib.ocd_detect.restype = ctypes.c_int
    lib.ocd_detect.argtypes = [ctypes.POINTER(Problem)] + [ctypes.c_void_p] * 10
    d = ctypes.c_void_p(0x1000)
    # g given without dinv and p
    assert lib.ocd_detect(ctypes.byref(pb), d, d, None, d, None, None, d, d, None, None) == -1


def test_backward_workspace_size_and_null_checks(lib):
    pb = Problem(**_good())
    lib.ocd_backward_workspace_bytes.restype = ctypes.c_size_t
    lib.ocd_backward_workspace_bytes.argtypes = [ctypes.POINTER(Problem)]
    n = lib.ocd_backward_workspace_bytes(ctypes.byref(pb))
    assert n >= 1200 * 14 * 4 * 4
    bad = Problem(**dict(_good(), K=0))
    assert lib.ocd_backward_workspace_bytes(ctypes.byref(bad)) == 0
    lib.ocd_detect_backward.restype = ctypes.c_int
    lib.ocd_detect_backward.argtypes = ([ctypes.POINTER(Problem)] + [ctypes.c_void_p] * 8 +
                                        [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p])
    d = ctypes.c_void_p(0x1000)
    # missing dlambda
    assert lib.ocd_detect_backward(ctypes.byref(pb), d, d, None, d, d, None, d, d, d, n, None) == -1
    # workspace too small
    assert lib.ocd_detect_backward(ctypes.byref(pb), d, d, None, d, d, d, d, d, d, 16, None) == -1
    # the fused cross-entropy form: the same checks, bits in place of dllr
    lib.ocd_detect_backward_bce.restype = ctypes.c_int
    lib.ocd_detect_backward_bce.argtypes = lib.ocd_detect_backward.argtypes
    bce = lib.ocd_detect_backward_bce
    assert bce(ctypes.byref(pb), d, d, None, d, None, d, d, d, d, n, None) == -1   # no bits
    assert bce(ctypes.byref(pb), d, d, None, None, d, d, d, d, d, n, None) == -1   # no z_hist
    assert bce(ctypes.byref(pb), d, d, None, d, d, None, d, d, d, n, None) == -1   # no dlambda
    assert bce(ctypes.byref(pb), d, d, None, d, d, d, d, d, d, 16, None) == -1     # small workspace
    assert bce(ctypes.byref(Problem(**dict(_good(), Q=5))), d, d, None, d, d, d, d, d, d, n,
               None) == -1


def test_backward_autotune_rejects_bad_arguments(lib):
    pb = Problem(**_good())
    lib.ocd_backward_workspace_bytes.restype = ctypes.c_size_t
    lib.ocd_backward_workspace_bytes.argtypes = [ctypes.POINTER(Problem)]
    n = lib.ocd_backward_workspace_bytes(ctypes.byref(pb))
    lib.ocd_autotune_backward.restype = ctypes.c_int
    lib.ocd_autotune_backward.argtypes = ([ctypes.POINTER(Problem)] + [ctypes.c_void_p] * 8 +
                                          [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int,
                                           ctypes.c_void_p, ctypes.c_void_p])
    d = ctypes.c_void_p(0x1000)
    best = ctypes.create_string_buffer(64)
    # no place for the plan
    assert lib.ocd_autotune_backward(ctypes.byref(pb), d, d, None, d, d, d, d, d, d, n, 1, None,
                                     None) == -1
    # missing dbeta
    assert lib.ocd_autotune_backward(ctypes.byref(pb), d, d, None, d, d, d, None, d, d, n, 1, best,
                                     None) == -1
    # workspace too small
    assert lib.ocd_autotune_backward(ctypes.byref(pb), d, d, None, d, d, d, d, d, d, 16, 1, best,
                                     None) == -1


def test_multi_input_autotune_rejects_bad_arguments(lib):
    pb = Problem(**_good())
    f = lib.ocd_autotune_inputs
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.POINTER(Problem), ctypes.c_int] + [ctypes.c_void_p] * 4 + [
        ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    d = 0x1000
    two = (ctypes.c_void_p * 2)(d, d)
    hole = (ctypes.c_void_p * 2)(d, None)
    best = ctypes.create_string_buffer(64)
    assert f(ctypes.byref(pb), 0, two, two, d, d, 1, best, None) == -1      # no input set
    assert f(ctypes.byref(pb), 65537, two, two, d, d, 1, best, None) == -1  # too many sets
    assert f(ctypes.byref(pb), 2, two, hole, d, d, 1, best, None) == -1     # a NULL y
    assert f(ctypes.byref(pb), 2, None, two, d, d, 1, best, None) == -1     # no H array
    assert f(ctypes.byref(pb), 2, two, two, d, None, 1, best, None) == -1   # no llr
    assert f(ctypes.byref(pb), 2, two, two, d, d, 1, None, None) == -1      # no place for the plan


def test_jobs_rejects_null_arguments(lib):
    lib.ocd_detect_jobs.restype = ctypes.c_int
    lib.ocd_detect_jobs.argtypes = [ctypes.POINTER(Problem), ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                    ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p]
    pb = Problem(**_good())
    assert lib.ocd_detect_jobs(ctypes.byref(pb), None, None, None, None, 1, None, 0, 0, None) == -1
    assert lib.ocd_detect_jobs(ctypes.byref(pb), None, None, None, None, 0, None, 0, 0, None) == -1


def test_jobs_accept_small_antenna_counts(lib):
    """Jobs with B <= 16 (fewer than 8 entries per lane even at 4 lanes) run at the
    batched kernel's built width, zero-padded: the planner accepts them beside large
    ones (the workspace query is host-only)."""
    lib.ocd_jobs_workspace_bytes.restype = ctypes.c_size_t
    lib.ocd_jobs_workspace_bytes.argtypes = [ctypes.POINTER(Problem), ctypes.c_int]
    for B in list(range(1, 17)) + [17, 33]:
        jobs = (Problem * 2)(Problem(**dict(_good(), B=B, U=max(1, min(32, B // 2)))),
                             Problem(**dict(_good(), B=256, U=8)))
        assert lib.ocd_jobs_workspace_bytes(jobs, 2) > 0, B


class Plan(ctypes.Structure):
    _fields_ = [("lanes_per_vector", ctypes.c_int), ("vectors_per_block", ctypes.c_int),
                ("xcd_remap", ctypes.c_int), ("channel_in_registers", ctypes.c_int),
                ("stagger", ctypes.c_int)]


REG_PLANS = [
    # (problem overrides, plan, expected status)
    (dict(), (16, 14, 1, 0, 2), 0),          # staggered staging
    (dict(), (16, 14, 1, 0, 17), -2),        # stagger beyond 16
    (dict(), (16, 14, 1, 0, -1), -2),
    (dict(S=1), (16, 16, 0, 1), 0),
    (dict(S=1), (32, 8, 0, 1), 0),
    (dict(S=1), (32, 9, 0, 1), -2),          # more than 256 lanes per workgroup
    (dict(S=1), (8, 32, 0, 1), -2),          # register plans take 16 or 32 lanes
    (dict(S=1, U=9), (16, 16, 0, 1), -2),    # above the register user bound
    (dict(S=1, B=300), (32, 8, 0, 1), -2),   # more than 8 entries per lane
    (dict(S=1), (16, 32, 0, 2), -2),         # no such placement
    (dict(S=1), (16, 16, 0, -1), -2),
]


@pytest.mark.parametrize("over,plan,status", REG_PLANS, ids=[str(p) for p in REG_PLANS])
def test_register_plans_are_checked_on_the_host(lib, over, plan, status):
    lib.ocd_set_plan.restype = ctypes.c_int
    lib.ocd_set_plan.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Plan)]
    pb = Problem(**{**_good(), **over})
    assert lib.ocd_set_plan(ctypes.byref(pb), ctypes.byref(Plan(*plan))) == status


def test_mmse_detector_checks_its_arguments_on_the_host(lib):
    lib.ocd_detect_mmse.restype = ctypes.c_int
    lib.ocd_detect_mmse.argtypes = [ctypes.POINTER(Problem), ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(Plan),
                                    ctypes.c_void_p]
    d = ctypes.c_void_p(0x1000)

    def call(over=None, H=d, y=d, z=d, llr=d, plan=None):
        pb = Problem(**{**_good(), **(over or {})})
        return lib.ocd_detect_mmse(ctypes.byref(pb), H, y, z, llr,
                                   ctypes.byref(Plan(*plan)) if plan else None, None)

    assert call(H=None) == -1
    assert call(y=None) == -1
    assert call(z=None, llr=None) == -1
    assert call(dict(B=0)) == -1
    assert call(dict(mode=1)) == -2                     # no closed form for the box problem
    assert call(dict(mode=2)) == -2
    assert call(dict(B=600)) == -2                      # above the kernel's antenna bound
    assert call(plan=(4, 16, 0, 0)) == -2               # lane groups of 8, 16 or 32
    assert call(plan=(16, 14, 0, 1)) == -2              # channel in registers: OCD only
    assert call(plan=(16, 33, 0, 0)) == -2              # more than 512 lanes per workgroup
    assert call(dict(W=0), plan=(0, 14, 0, 0)) == 0     # matrix cores: U <= 8, S <= 16
    assert call(dict(W=0), plan=(0, 0, 1, 0)) == 0
    assert call(plan=(0, 7, 0, 0)) == -2                # one subcarrier per workgroup: S
    assert call(dict(U=9), plan=(0, 14, 0, 0)) == -2
    assert call(dict(S=17), plan=(0, 17, 0, 0)) == -2
    assert call(dict(W=0), plan=(16, 14, 0, 0)) == 0    # nothing to do
    # staggered staging, both forms: 0..16 accepted, anything else refused
    assert call(dict(W=0), plan=(16, 14, 0, 0, 4)) == 0
    assert call(dict(W=0), plan=(0, 14, 0, 0, 16)) == 0
    assert call(plan=(16, 14, 0, 0, 17)) == -2
    assert call(plan=(0, 14, 0, 0, 17)) == -2
    assert call(plan=(0, 14, 0, 0, -1)) == -2


@pytest.mark.parametrize("B,U,S", [(512, 8, 2), (256, 16, 3), (128, 8, 14), (64, 32, 2), (33, 4, 2),
                                   (100, 8, 3), (16, 1, 5)])
def test_mmse_heuristic_plan_fits(lib, B, U, S):
    """The default plan of ocd_detect_mmse is valid for every shape whose single
    subcarrier fits the 64 KiB of LDS assumed without a device (W = 0: nothing runs)."""
    lib.ocd_detect_mmse.restype = ctypes.c_int
    lib.ocd_detect_mmse.argtypes = [ctypes.POINTER(Problem), ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(Plan),
                                    ctypes.c_void_p]
    d = ctypes.c_void_p(0x1000)
    pb = Problem(**{**_good(), "B": B, "U": U, "S": S, "W": 0})
    assert lib.ocd_detect_mmse(ctypes.byref(pb), d, d, d, d, None, None) == 0


def test_fixed_point_detector_checks_its_arguments_on_the_host(lib):
    lib.ocd_detect_fixed.restype = ctypes.c_int
    lib.ocd_detect_fixed.argtypes = [ctypes.POINTER(Problem)] + [ctypes.c_void_p] * 5
    d = ctypes.c_void_p(0x1000)

    def call(over=None, H=d, y=d, z=d, llr=d):
        pb = Problem(**{**_good(), **(over or {})})
        return lib.ocd_detect_fixed(ctypes.byref(pb), H, y, z, llr, None)

    assert call(H=None) == -1
    assert call(y=None) == -1
    assert call(z=None, llr=None) == -1
    assert call(dict(Q=5)) == -1
    assert call(dict(mode=2)) == -2      # HYBRID: per-sweep regularisers are not in the design
    assert call(dict(W=0)) == 0
    assert call(dict(W=0, mode=1)) == 0
    # alpha = round(N0/Es 2^22) must fit the 36-bit adder: checked before any launch
    assert call(dict(N0=1e7)) == -1
    assert call(dict(N0=8000.0, W=0)) == 0
    assert call(dict(N0=1e7, mode=1, W=0)) == 0     # BOX has no regulariser
    assert call(dict(beta=1e30, mode=1, W=0)) == 0  # a bound beyond the word range is no error


class OfdmShape(ctypes.Structure):
    _fields_ = [("B", ctypes.c_int), ("S", ctypes.c_int), ("N", ctypes.c_int),
                ("Ncp", ctypes.c_int), ("W", ctypes.c_int)]


@pytest.mark.parametrize("bad", [
    dict(N=1000), dict(N=128), dict(N=8192), dict(Ncp=-1), dict(Ncp=2049), dict(W=1201),
    dict(W=0), dict(W=2048), dict(W=-2), dict(B=0), dict(S=0)])
def test_ofdm_shapes_are_checked_on_the_host(lib, bad):
    lib.ocd_ofdm_demodulate.restype = ctypes.c_int
    lib.ocd_ofdm_demodulate.argtypes = [ctypes.POINTER(OfdmShape)] + [ctypes.c_void_p] * 3
    good = dict(B=128, S=14, N=2048, Ncp=144, W=1200)
    d = ctypes.c_void_p(0x1000)
    sh = OfdmShape(**{**good, **bad})
    assert lib.ocd_ofdm_demodulate(ctypes.byref(sh), d, d, None) == -1
    assert lib.ocd_ofdm_demodulate(ctypes.byref(OfdmShape(**good)), None, d, None) == -1


def test_fma_probe_checks_its_arguments_on_the_host(lib):
    lib.ocd_probe_fma.restype = ctypes.c_int
    lib.ocd_probe_fma.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                  ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]
    d = ctypes.c_void_p(0x1000)
    fl = ctypes.c_double(0.0)
    assert lib.ocd_probe_fma(0, 10, d, ctypes.byref(fl), None) == -1
    assert lib.ocd_probe_fma(10, 0, d, ctypes.byref(fl), None) == -1
    assert lib.ocd_probe_fma(10, 10, None, ctypes.byref(fl), None) == -1
    assert lib.ocd_probe_fma(10, 10, d, None, None) == -1


_CACHE_READER = r"""
import ctypes, json, sys
lib = ctypes.CDLL(sys.argv[1])
class Problem(ctypes.Structure):
    _fields_ = [("B", ctypes.c_int), ("U", ctypes.c_int), ("W", ctypes.c_int), ("S", ctypes.c_int),
                ("Q", ctypes.c_int), ("K", ctypes.c_int), ("mode", ctypes.c_int),
                ("storage", ctypes.c_int), ("N0", ctypes.c_float), ("Es", ctypes.c_float),
                ("beta", ctypes.c_float)]
class Plan(ctypes.Structure):
    _fields_ = [("lanes_per_vector", ctypes.c_int), ("vectors_per_block", ctypes.c_int),
                ("xcd_remap", ctypes.c_int), ("channel_in_registers", ctypes.c_int),
                ("stagger", ctypes.c_int)]
out = []
for B, U, W, S, Q, K in json.loads(sys.argv[2]):
    pb = Problem(B, U, W, S, Q, K, 0, 0, 0.01, 1.0, 0.0)
    pl = Plan()
    st = lib.ocd_get_plan(ctypes.byref(pb), ctypes.byref(pl))
    out.append([st, pl.lanes_per_vector, pl.vectors_per_block, pl.xcd_remap,
                pl.channel_in_registers, pl.stagger])
print(json.dumps(out))
"""


def test_plan_cache_file_is_read(tmp_path):
    """Plans persisted in the OCD_TUNE_CACHE file (one JSON object a line, keyed by
    GPU architecture and shape) are what ocd_get_plan returns for those shapes: a
    line written before the stagger field loads with stagger 0, a plan that is not
    valid for its shape gives way to the heuristic, other lines are ignored.  Read
    in a fresh process (the file is loaded once per process) with the GPUs hidden,
    so that the architecture part of the key is "unknown"."""
    import json
    import subprocess
    import sys
    if not os.path.exists(LIB):
        pytest.skip("libocd.so is not built")
    key = "unknown|fwd|B%d|U%d|W%d|S%d|K%d|Q%d|m0|s0|l0"
    shapes = [(128, 8, 1200, 14, 6, 3), (64, 4, 10, 2, 4, 2), (32, 4, 10, 2, 4, 2)]
    lines = [
        '{"key": "%s", "lanes_per_vector": 16, "vectors_per_block": 28, "xcd_remap": 1, '
        '"channel_in_registers": 0, "stagger": 2}' % (key % (128, 8, 1200, 14, 3, 6)),
        "not a plan",
        '{"key": "%s", "lanes_per_vector": 8, "vectors_per_block": 4, "xcd_remap": 0, '
        '"channel_in_registers": 0}' % (key % (64, 4, 10, 2, 2, 4)),
        '{"key": "%s", "lanes_per_vector": 64, "vectors_per_block": 4, "xcd_remap": 0, '
        '"channel_in_registers": 0, "stagger": 0}' % (key % (32, 4, 10, 2, 2, 4)),
    ]
    cache = tmp_path / "plans.json"
    cache.write_text("\n".join(lines) + "\n")
    env = dict(os.environ, OCD_TUNE_CACHE=str(cache), HIP_VISIBLE_DEVICES="-1",
               ROCR_VISIBLE_DEVICES="-1")
    r = subprocess.run([sys.executable, "-c", _CACHE_READER, LIB, json.dumps(shapes)],
                       capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stderr
    got = json.loads(r.stdout.strip().splitlines()[-1])
    assert got[0] == [0, 16, 28, 1, 0, 2]
    assert got[1] == [0, 8, 4, 0, 0, 0]
    assert got[2][0] == 0 and got[2][1] in (4, 8, 16, 32)   # the heuristic's, not 64 lanes
