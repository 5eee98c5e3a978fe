"""The host-side entry points under random and extreme arguments (no GPU): problem
validation, plan queries and plans set by the caller, and the workspace sizes.
Whatever the problem, each call returns a status of the header's set (never
crashes); a valid problem gets a plan of the documented ranges and the documented
workspace size, an invalid one an error and a zero size."""

import ctypes
import math
import os

import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1611_08779_amd", "libocd.so")

STATUSES = {0, -1, -2, -3, -4}


class Problem(ctypes.Structure):
    _fields_ = [("B", ctypes.c_int), ("U", ctypes.c_int), ("W", ctypes.c_int), ("S", ctypes.c_int),
                ("Q", ctypes.c_int), ("K", ctypes.c_int), ("mode", ctypes.c_int),
                ("storage", ctypes.c_int), ("N0", ctypes.c_float), ("Es", ctypes.c_float),
                ("beta", ctypes.c_float)]


class Plan(ctypes.Structure):
    _fields_ = [("lanes_per_vector", ctypes.c_int), ("vectors_per_block", ctypes.c_int),
                ("xcd_remap", ctypes.c_int), ("channel_in_registers", ctypes.c_int),
                ("stagger", ctypes.c_int)]


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libocd.so is not built")
    lib = ctypes.CDLL(LIB)
    P, PL = ctypes.POINTER(Problem), ctypes.POINTER(Plan)
    for name, args, res in [
            ("ocd_backward_workspace_bytes", [P], ctypes.c_size_t),
            ("ocd_jobs_workspace_bytes", [P, ctypes.c_int], ctypes.c_size_t),
            ("ocd_get_plan", [P, PL], ctypes.c_int), ("ocd_train_plan", [P, PL], ctypes.c_int),
            ("ocd_set_plan", [P, PL], ctypes.c_int)]:
        f = getattr(lib, name)
        f.argtypes, f.restype = args, res
    return lib


INT32 = st.integers(-(1 << 31), (1 << 31) - 1)
FLOATS = st.one_of(st.floats(allow_nan=True, allow_infinity=True, width=32),
                   st.sampled_from([0.0, -0.0, 1e-30, 1.0, 1e30]))


def near(lo, hi):
    """Mostly in the valid range, sometimes just outside it, sometimes anywhere."""
    return st.one_of(st.integers(lo, hi), st.integers(lo - 2, hi + 2), INT32)


problems = st.builds(
    Problem, B=near(1, 1024), U=near(1, 32), W=st.one_of(near(0, 4096), st.integers(0, 1 << 30)),
    S=st.one_of(near(1, 16), st.integers(1, 1 << 20)), Q=st.sampled_from([-1, 0, 2, 3, 4, 6, 8]),
    K=near(1, 256), mode=near(0, 2), storage=near(0, 1), N0=FLOATS, Es=FLOATS, beta=FLOATS)


def valid(pb):
    f32 = lambda x: math.isfinite(x)
    return (1 <= pb.B <= 1024 and 1 <= pb.U <= 32 and pb.U <= pb.B and pb.W >= 0 and pb.S >= 1
            and pb.Q in (2, 4, 6) and 1 <= pb.K <= 256 and pb.mode in (0, 1, 2)
            and pb.storage in (0, 1) and f32(pb.N0) and pb.N0 > 0 and f32(pb.Es) and pb.Es > 0
            and f32(pb.beta))


def plan_ok(pl):
    return (pl.lanes_per_vector in (4, 8, 16, 32) and pl.vectors_per_block >= 1
            and pl.xcd_remap in (0, 1) and pl.channel_in_registers in (0, 1)
            and 0 <= pl.stagger <= 16)


@settings(max_examples=600, deadline=None, suppress_health_check=[HealthCheck.function_scoped_fixture])
@given(pb=problems)
def test_validation_queries_and_workspace_sizes(lib, pb):
    ok = valid(pb)
    in_range = ok and pb.W * pb.S <= (1 << 30)
    ws = lib.ocd_backward_workspace_bytes(ctypes.byref(pb))
    if in_range:
        assert ws == 256 + max(1, pb.W * pb.S) * (pb.K + 2) * 4
    elif not ok:
        assert ws == 0
    for q in (lib.ocd_get_plan, lib.ocd_train_plan):
        pl = Plan()
        s = q(ctypes.byref(pb), ctypes.byref(pl))
        assert s in STATUSES
        if not ok:
            assert s != 0
        elif s == 0:
            assert plan_ok(pl), (pl.lanes_per_vector, pl.vectors_per_block)
    jobs = (Problem * 2)(pb, pb)
    jw = lib.ocd_jobs_workspace_bytes(jobs, 2)
    if not ok:
        assert jw == 0


@settings(max_examples=600, deadline=None, suppress_health_check=[HealthCheck.function_scoped_fixture])
@given(pb=problems, L=st.sampled_from([-1, 0, 2, 4, 8, 16, 32, 64]), vpb=near(1, 512),
       xcd=near(0, 1), cir=near(0, 1), stagger=near(0, 16))
def test_plans_set_by_the_caller(lib, pb, L, vpb, xcd, cir, stagger):
    pl = Plan(L, vpb, xcd, cir, stagger)
    s = lib.ocd_set_plan(ctypes.byref(pb), ctypes.byref(pl))
    assert s in STATUSES
    if not valid(pb) or not plan_ok(pl):
        assert s != 0
    if s == 0:   # an accepted plan is the one the next query returns
        got = Plan()
        assert lib.ocd_get_plan(ctypes.byref(pb), ctypes.byref(got)) == 0
        assert (got.lanes_per_vector, got.vectors_per_block, got.xcd_remap,
                got.channel_in_registers, got.stagger) == (L, vpb, xcd, cir, stagger)
