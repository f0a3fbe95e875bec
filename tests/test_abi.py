"""CPU checks of the C ABI: the library loads, exports every function that
include/ge.h declares, and validates its arguments without touching a GPU
(every call here returns before any work would be enqueued)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_1310_3422_amd import ge

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.skipif(not os.path.exists(ge.LIB_PATH),
                                reason="libge.so not built")


def declared_functions():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if not h.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w \*]*?\b(ge_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert "ge_step_n" in names and "ge_plan" in names and "ge_solve_batch" in names
    h = ctypes.CDLL(ge.LIB_PATH)
    missing = [n for n in names if not hasattr(h, n)]
    assert not missing, missing


def test_status_strings_and_version():
    assert ge.status_str(0) == "GE_OK"
    assert ge.status_str(5) == "GE_ERR_NONFINITE"
    assert ge.status_str(6) == "GE_ERR_SYNC"
    assert ge.lib().ge_plan_check(None, None) == ge.GE_ERR_INVALID
    assert ge.lib().ge_version().decode().count(".") == 2


def _plan(**kw):
    d = dict(n=1000, r=1.0, precision=0, tile=0, depth=0, waves=0, g_left=0.0,
             g_right=0.0, src_b=None)
    d.update(kw)
    desc = ge.GeDesc(**d)
    h = ctypes.c_void_p()
    st = ge.lib().ge_plan(ctypes.byref(h), ctypes.byref(desc))
    return st, h


@pytest.mark.parametrize("kw,status", [
    (dict(n=0), ge.GE_ERR_INVALID),
    (dict(n=-5), ge.GE_ERR_INVALID),
    (dict(r=0.0), ge.GE_ERR_INVALID),
    (dict(r=-1.0), ge.GE_ERR_INVALID),
    (dict(r=float("nan")), ge.GE_ERR_NONFINITE),
    (dict(r=float("inf")), ge.GE_ERR_NONFINITE),
    (dict(g_left=float("nan")), ge.GE_ERR_NONFINITE),
    (dict(precision=7), ge.GE_ERR_INVALID),
    (dict(tile=6), ge.GE_ERR_INVALID),
    (dict(waves=3), ge.GE_ERR_INVALID),
    (dict(depth=-2), ge.GE_ERR_INVALID),
    (dict(n=10 ** 6, tile=8, waves=1, depth=200), ge.GE_ERR_INVALID),
    (dict(src_b=ctypes.c_void_p(0x1004)), ge.GE_ERR_INVALID),
])
def test_plan_rejects(kw, status):
    st, h = _plan(**kw)
    assert st == status
    assert not h.value
    assert ge.last_error()


def test_null_arguments():
    lib = ge.lib()
    assert lib.ge_plan(None, None) == ge.GE_ERR_INVALID
    h = ctypes.c_void_p()
    assert lib.ge_plan(ctypes.byref(h), None) == ge.GE_ERR_INVALID
    assert lib.ge_step_n(None, None, None, 0, 1, None, None, None, None, None) == ge.GE_ERR_INVALID
    lib.ge_destroy(None)


@pytest.mark.parametrize("prec,depth", [(0, 1), (0, 32), (1, 7), (2, 33)])
def test_plan_config_halo_rule(prec, depth):
    st, h = _plan(n=10 ** 6, precision=prec, depth=depth)
    assert st == ge.GE_OK
    t, d, w, hal = (ctypes.c_int32() for _ in range(4))
    assert ge.lib().ge_plan_config(h, ctypes.byref(t), ctypes.byref(d), ctypes.byref(w),
                                   ctypes.byref(hal)) == ge.GE_OK
    align = 2 if prec == 0 else 4
    assert d.value == depth
    assert hal.value == (depth + 1 + align - 1) // align * align
    ge.lib().ge_destroy(h)


def test_single_window_rod_needs_no_halo():
    st, h = _plan(n=1024, precision=0, tile=16, waves=4)
    assert st == ge.GE_OK
    hal = ctypes.c_int32()
    ge.lib().ge_plan_config(h, None, None, None, ctypes.byref(hal))
    assert hal.value == 0
    ge.lib().ge_destroy(h)


def test_workspace_bytes():
    lib = ge.lib()
    for prec, n, want in ((0, 1000, 8000), (1, 1000, 4000), (2, 1000, 8 * 1024), (2, 64, 512)):
        desc = ge.GeDesc(n=n, r=1.0, precision=prec)
        assert lib.ge_workspace_bytes(ctypes.byref(desc)) == want
    assert lib.ge_workspace_bytes(None) == 0
    assert ge.comp_offset(1) == 64 and ge.comp_offset(128) == 128 and ge.comp_offset(-1) == -1


def test_step_n_validation_enqueues_nothing():
    """Fake (never dereferenced) device addresses: every call below must be
    rejected, or be a no-op, before any launch."""
    lib = ge.lib()
    st, h = _plan(n=10 ** 6, precision=0)
    assert st == ge.GE_OK
    u = ctypes.c_void_p(0x10000000)
    ws = ctypes.c_void_p(0x20000000)
    call = lambda *a: lib.ge_step_n(h, *a)
    assert call(None, ws, 0, 5, None, None, None, None, None) == ge.GE_ERR_INVALID
    assert call(u, None, 0, 5, None, None, None, None, None) == ge.GE_ERR_INVALID
    assert call(u, ws, -1, 5, None, None, None, None, None) == ge.GE_ERR_INVALID
    assert call(u, ws, 0, -5, None, None, None, None, None) == ge.GE_ERR_INVALID
    assert call(ctypes.c_void_p(0x10000008), ws, 0, 5, None, None, None, None, None) == ge.GE_ERR_INVALID
    assert call(u, ctypes.c_void_p(0x20000004), 0, 5, None, None, None, None, None) == ge.GE_ERR_INVALID
    # overlapping buffers
    assert call(u, ctypes.c_void_p(0x10000000 + 8 * 1000), 0, 5, None, None, None, None,
                None) == ge.GE_ERR_INVALID
    # a source array without a source profile
    assert call(u, ws, 0, 5, None, None, ctypes.c_void_p(0x30000000), None, None) == ge.GE_ERR_INVALID
    # nothing to do
    assert call(u, ws, 0, 0, None, None, None, None, None) == ge.GE_OK
    lib.ge_destroy(h)


@pytest.mark.parametrize("depth", list(range(1, 17)))
@pytest.mark.parametrize("step0", [0, 1])
def test_halo_of_depth_plus_one_is_enough_and_tight(depth, step0):
    """The library recomputes a halo of depth+1 points (rounded up) on each
    side of a tile instead of exchanging it.  On the oracle: cutting a rod at
    an even index and feeding garbage in at the cut leaves every point more
    than depth+1 away from the cut exact after `depth` levels."""
    rng = np.random.default_rng(depth)
    n = 200
    u = rng.standard_normal(n)
    full = oracle.step_n(u, 2.5, depth, step0=step0)
    a, b = 60, 140
    h = 1.0 / (n + 1)
    cut = oracle.step_n(u[a:b], 2.5, depth, step0=step0, gl=1e3, gr=-1e3, tau=2.5 * h * h, h=h)
    lo, hi = depth + 1, (b - a) - depth - 1
    np.testing.assert_array_equal(cut[lo:hi], full[a + lo:a + hi])
    # starting on an even level the bound is reached: one point closer to
    # either cut is contaminated (starting on an odd level depth suffices)
    if step0 == 0:
        assert cut[lo - 1] != full[a + lo - 1] and cut[hi] != full[a + hi]


def _batch_desc(n, offsets, r=None, gl=None, gr=None, precision=1, tune=0, sync=0):
    nr = len(n)
    arrs = dict(n=np.asarray(n, np.int64), offsets=np.asarray(offsets, np.int64),
                r=np.asarray(r if r is not None else [1.0] * nr, np.float64),
                gl=np.asarray(gl if gl is not None else [0.0] * nr, np.float64),
                gr=np.asarray(gr if gr is not None else [0.0] * nr, np.float64))
    c = lambda a: ctypes.c_void_p(a.ctypes.data)
    d = ge.GeBatchDesc(nrods=nr, n=c(arrs["n"]), offsets=c(arrs["offsets"]), r=c(arrs["r"]),
                       g_left=c(arrs["gl"]), g_right=c(arrs["gr"]), precision=precision,
                       tune=tune, sync=sync)
    return d, arrs


@pytest.mark.parametrize("case,status", [
    (dict(n=[100, 0], offsets=[0, 100, 200]), ge.GE_ERR_INVALID),
    (dict(n=[100, 50], offsets=[0, 98, 200]), ge.GE_ERR_INVALID),        # overlap
    (dict(n=[100, 50], offsets=[0, 102, 200]), ge.GE_ERR_INVALID),       # not a multiple of 4
    (dict(n=[100, 50], offsets=[0, 100, 200], r=[1.0, 0.0]), ge.GE_ERR_INVALID),
    (dict(n=[100, 50], offsets=[0, 100, 200], r=[1.0, float("nan")]), ge.GE_ERR_NONFINITE),
    (dict(n=[100], offsets=[0, 100], sync=4), ge.GE_ERR_INVALID),
    (dict(n=[100], offsets=[0, 100], sync=-1), ge.GE_ERR_INVALID),
    (dict(n=[100], offsets=[0, 100], precision=9), ge.GE_ERR_INVALID),
])
def test_batch_plan_rejects(case, status):
    d, keep = _batch_desc(**case)
    h = ctypes.c_void_p()
    assert ge.lib().ge_batch_plan(ctypes.byref(h), ctypes.byref(d)) == status
    assert not h.value


def test_batch_null_arguments():
    lib = ge.lib()
    assert lib.ge_batch_plan(None, None) == ge.GE_ERR_INVALID
    assert lib.ge_solve_batch(None, None, None, 0, 1, None) == ge.GE_ERR_INVALID
    assert lib.ge_batch_check(None, None) == ge.GE_ERR_INVALID
    assert lib.ge_batch_set_wait_polls(None, 5) == ge.GE_ERR_INVALID
    assert lib.ge_batch_state_elems(None) == -1
    assert lib.ge_batch_workspace_bytes(None) == 0
    lib.ge_batch_destroy(None)


def test_nn_parameter_count_and_create_rejects():
    lib = ge.lib()
    assert lib.ge_nn_param_count() == 83201
    h = ctypes.c_void_p()
    assert lib.ge_nn_create(None, 4096, 4, 0) == ge.GE_ERR_INVALID
    for width, batch in [(0, 1), (100, 1), (4096 + 64, 1), (4096, 0), (4096, 1 << 20)]:
        assert lib.ge_nn_create(ctypes.byref(h), width, batch, 0) == ge.GE_ERR_INVALID, (width, batch)
        assert h.value is None
    assert b"multiple of 128" in lib.ge_last_error() or b"out of range" in lib.ge_last_error()


def test_nn_calls_reject_null_network():
    lib = ge.lib()
    fake = ctypes.c_void_p(0x1000)
    assert lib.ge_nn_forward(None, fake, fake, 1, fake, fake, None) == ge.GE_ERR_INVALID
    assert lib.ge_nn_jump(None, fake, fake, 1, fake, None) == ge.GE_ERR_INVALID
    assert lib.ge_nn_grads(None, fake, fake, fake, 1, None, None) == ge.GE_ERR_INVALID
    assert lib.ge_nn_train_step(None, fake, fake, fake, 1, ctypes.c_float(1e-3), None,
                                None) == ge.GE_ERR_INVALID
    assert lib.ge_nn_train_step(None, fake, fake, fake, 1, ctypes.c_float(-1.0), None,
                                None) == ge.GE_ERR_INVALID
    assert lib.ge_nn_set_params(None, None, 0) == ge.GE_ERR_INVALID
    assert lib.ge_nn_get_params(None, None, 0) == ge.GE_ERR_INVALID
    assert lib.ge_nn_gradient(None, None, None) == ge.GE_ERR_INVALID
    lib.ge_nn_destroy(None)


def test_advance_and_conversions_validate_before_enqueueing():
    lib = ge.lib()
    fake = ctypes.c_void_p(0x1000)
    n = ctypes.c_int64(7)
    assert lib.ge_nn_advance(None, fake, fake, fake, fake, 1, 0, 1, 8, 1e-4, None, None, None,
                             ctypes.byref(n), None) == ge.GE_ERR_INVALID
    assert lib.ge_f32_to_f64(fake, fake, -1, None) == ge.GE_ERR_INVALID
    assert lib.ge_f64_to_f32(None, None, 5, None) == ge.GE_ERR_INVALID
    assert lib.ge_f32_to_f64(None, None, 0, None) == ge.GE_OK
    assert lib.ge_f64_to_f32(None, None, 0, None) == ge.GE_OK


def test_plan_schedule_validation():
    lib = ge.lib()
    h = ctypes.c_void_p()
    for sched, tile, waves, status in [(3, 16, 1, ge.GE_ERR_INVALID), (-1, 16, 1, ge.GE_ERR_INVALID),
                                       (2, 16, 4, ge.GE_ERR_INVALID), (2, 8, 1, ge.GE_ERR_INVALID),
                                       (2, 16, 1, ge.GE_OK), (1, 8, 4, ge.GE_OK)]:
        d = ge.GeDesc(n=100000, r=2.0, precision=0, tile=tile, depth=8, waves=waves,
                      schedule=sched)
        st = lib.ge_plan(ctypes.byref(h), ctypes.byref(d))
        assert st == status, (sched, tile, waves)
        if st == ge.GE_OK:
            assert lib.ge_plan_schedule(h) == (2 if sched == 2 else 1)
            lib.ge_destroy(h)
    assert lib.ge_plan_schedule(None) == -1


@pytest.mark.parametrize("prec,depth,src,want", [
    (0, 0, False, (32, 1, 96, 2)), (0, 0, True, (28, 1, 96, 1)),
    (0, 1, False, (2, 1, 1, 1)), (0, 8, True, (4, 1, 8, 1)), (0, 16, False, (8, 1, 16, 1)),
    (0, 32, True, (16, 1, 32, 1)), (0, 64, False, (32, 1, 64, 2)), (0, 64, True, (28, 1, 64, 1)),
    (1, 0, False, (32, 1, 96, 2)), (1, 4, False, (4, 1, 4, 1)), (1, 8, False, (8, 1, 8, 1)),
    (1, 8, True, (4, 1, 8, 1)), (1, 16, True, (16, 1, 16, 1)), (1, 64, True, (32, 1, 64, 1)),
    (1, 0, True, (32, 1, 64, 1)), (1, 32, True, (32, 1, 32, 1)),
    (2, 0, False, (16, 4, 128, 1)), (2, 2, False, (4, 1, 2, 1)), (2, 32, True, (8, 4, 32, 1)),
])
def test_default_tile_follows_depth_and_source(prec, depth, src, want):
    """The library's tile, waves, depth and schedule when only the depth (or
    nothing) is given: narrow rows for shallow launches, wide rows and the
    persistent schedule for deep ones without a source."""
    st, h = _plan(n=1 << 24, precision=prec, depth=depth,
                  src_b=ctypes.c_void_p(0x1000) if src else None)
    assert st == ge.GE_OK
    t, d, w, hal = (ctypes.c_int32() for _ in range(4))
    ge.lib().ge_plan_config(h, ctypes.byref(t), ctypes.byref(d), ctypes.byref(w), ctypes.byref(hal))
    assert (t.value, w.value, d.value, ge.lib().ge_plan_schedule(h)) == want
    ge.lib().ge_destroy(h)


@pytest.mark.parametrize("kw,status", [
    (dict(n=31, k=-1), ge.GE_ERR_INVALID),
    (dict(n=35, k=3), ge.GE_ERR_UNSUPPORTED),
    (dict(n=30, k=2), ge.GE_ERR_INVALID),                 # n + 1 not a multiple of 4
    (dict(n=31, k=4, precision=2), ge.GE_ERR_UNSUPPORTED),
    (dict(n=31, k=4, src_b=ctypes.c_void_p(0x1000)), ge.GE_ERR_UNSUPPORTED),
    (dict(n=31, k=4, tile=16), ge.GE_ERR_INVALID),
    (dict(n=31, k=4, waves=3), ge.GE_ERR_INVALID),
    (dict(n=31, k=4, waves=16), ge.GE_ERR_INVALID),
    (dict(n=32 * 1000 - 1, k=16, depth=46, waves=1), ge.GE_ERR_INVALID),   # halo 25 of 64
    (dict(n=32 * 1000 - 1, k=16, depth=230, waves=4), ge.GE_ERR_INVALID),  # halo 123 of 256
    (dict(n=32 * 1000 - 1, k=16, depth=60), ge.GE_ERR_INVALID),   # halo wider than the window allows
    (dict(n=31, k=4, schedule=3), ge.GE_ERR_INVALID),
])
def test_subdomain_plan_rejects(kw, status):
    st, h = _plan(**kw)
    assert st == status, ge.last_error()
    assert not h.value


def test_subdomain_deep_launches_stay_per_tile():
    """The library takes the persistent sub-domain form only up to the 64
    levels per launch it holds; deeper launches run one workgroup per tile."""
    for depth, sched in ((64, 2), (80, 1)):
        st, h = _plan(n=(1 << 24) - 1, k=16, depth=depth, waves=8)
        assert st == ge.GE_OK, ge.last_error()
        assert ge.lib().ge_plan_schedule(h) == sched
        ge.lib().ge_destroy(h)


def test_subdomain_wide_windows():
    """Windows of 2 or 4 waves keep the halo per side of a single-wave window
    (it depends on the depth only), so deeper launches fit."""
    for waves, depth, halo in ((2, 46, 25), (4, 60, 32), (4, 24, 13)):
        st, h = _plan(n=32 * 1000 - 1, k=16, depth=depth, waves=waves)
        assert st == ge.GE_OK, ge.last_error()
        t, d, w, hal = (ctypes.c_int32() for _ in range(4))
        ge.lib().ge_plan_config(h, ctypes.byref(t), ctypes.byref(d), ctypes.byref(w),
                                ctypes.byref(hal))
        assert (t.value, d.value, w.value, hal.value) == (32, depth, waves, 32 * halo)
        ge.lib().ge_destroy(h)


def test_subdomain_plan_config():
    st, h = _plan(n=32 * 1000 - 1, k=16)
    assert st == ge.GE_OK
    t, d, w, hal = (ctypes.c_int32() for _ in range(4))
    ge.lib().ge_plan_config(h, ctypes.byref(t), ctypes.byref(d), ctypes.byref(w), ctypes.byref(hal))
    # 24 levels (FP64, k = 16): a halo of ceil((24 * 17 + 2) / 32) = 13
    # couples of 32 points; 27 windows, one workgroup per tile
    assert (t.value, d.value, w.value, hal.value) == (32, 24, 1, 416)
    fake = ctypes.c_void_p(0x1000)
    flux = ctypes.c_void_p(0x2000)
    assert ge.lib().ge_step_n(h, fake, ctypes.c_void_p(0x100000), 0, 1, None, None, None, flux,
                              None) == ge.GE_ERR_UNSUPPORTED
    assert ge.lib().ge_plan_schedule(h) == 1
    ge.lib().ge_destroy(h)


@pytest.mark.parametrize("n,schedule,want", [
    (32 * 1000 - 1, 2, 2),      # 27 tiles of 38 couples (24 levels): persistent as asked
    (32 * 100 - 1, 2, 2),       # 3 tiles
    (32 * 70 - 1, 2, 1),        # 2 tiles: one workgroup per tile
    (32 * 64 - 1, 2, 1),        # one window, advanced in place
    (32 * 1000 - 1, 1, 1),
])
def test_subdomain_schedule(n, schedule, want):
    st, h = _plan(n=n, k=16, schedule=schedule)
    assert st == ge.GE_OK
    assert ge.lib().ge_plan_schedule(h) == want
    ge.lib().ge_destroy(h)


@pytest.mark.parametrize("n,prec,k,want", [
    ((1 << 24) - 1, 0, 16, (4, 40, 2)),   # FP64, couples of 32: four waves, persistent
    ((1 << 24) - 1, 1, 16, (8, 48, 1)),   # FP32: eight waves per tile
    ((1 << 24) - 1, 0, 8, (8, 48, 1)),
    ((1 << 24) - 1, 1, 2, (8, 48, 1)),
    (262655, 0, 16, (1, 24, 2)),          # 8208 couples: too few for wide windows
    (262655, 1, 16, (1, 20, 1)),
    (32 * 400000 - 1, 0, 16, (1, 24, 2)),  # 1887 four-wave tiles: 7548 waves
    (32 * 450000 - 1, 0, 16, (4, 40, 2)),  # 2123 tiles of 212 couples: 8492 waves
])
def test_subdomain_library_choice(n, prec, k, want):
    st, h = _plan(n=n, k=k, precision=prec)
    assert st == ge.GE_OK
    t, d, w, hal = (ctypes.c_int32() for _ in range(4))
    ge.lib().ge_plan_config(h, ctypes.byref(t), ctypes.byref(d), ctypes.byref(w), ctypes.byref(hal))
    assert (w.value, d.value, ge.lib().ge_plan_schedule(h)) == want
    ge.lib().ge_destroy(h)


def _d2(**kw):
    d = dict(nx=10, ny=7, rx=1.0, ry=2.0, precision=0)
    d.update(kw)
    return ge.Ge2dDesc(**d)


def test_2d_workspace_bytes():
    assert ge.lib().ge_2d_workspace_bytes(ctypes.byref(_d2())) == 560
    assert ge.lib().ge_2d_workspace_bytes(ctypes.byref(_d2(precision=1))) == 280
    assert ge.lib().ge_2d_workspace_bytes(ctypes.byref(_d2(nx=0))) == 0
    assert ge.lib().ge_2d_workspace_bytes(None) == 0


@pytest.mark.parametrize("kw,args,status", [
    (dict(nx=0), {}, ge.GE_ERR_INVALID),
    (dict(ny=-1), {}, ge.GE_ERR_INVALID),
    (dict(rx=0.0), {}, ge.GE_ERR_INVALID),
    (dict(ry=float("inf")), {}, ge.GE_ERR_INVALID),
    (dict(g_north=float("nan")), {}, ge.GE_ERR_INVALID),
    (dict(precision=2), {}, ge.GE_ERR_UNSUPPORTED),
    (dict(precision=7), {}, ge.GE_ERR_INVALID),
    (dict(nx=1 << 32), {}, ge.GE_ERR_INVALID),
    (dict(depth=3), {}, ge.GE_ERR_INVALID),
    ({}, dict(step0=-1), ge.GE_ERR_INVALID),
    ({}, dict(nsteps=-2), ge.GE_ERR_INVALID),
    ({}, dict(ws=0x100000 + 8), ge.GE_ERR_INVALID),     # overlaps u
    ({}, dict(u=None), ge.GE_ERR_INVALID),
])
def test_2d_rejects(kw, args, status):
    """Argument errors return before anything is enqueued (no device needed)."""
    a = dict(u=0x100000, ws=0x200000, step0=0, nsteps=3)
    a.update(args)
    st = ge.lib().ge_2d_step_n(ctypes.byref(_d2(**kw)), ctypes.c_void_p(a["u"]) if a["u"] else None,
                               ctypes.c_void_p(a["ws"]), a["step0"], a["nsteps"], None)
    assert st == status, ge.last_error()


def test_2d_zero_levels_is_a_no_op():
    assert ge.lib().ge_2d_step_n(ctypes.byref(_d2()), ctypes.c_void_p(0x100000),
                                 ctypes.c_void_p(0x200000), 0, 0, None) == ge.GE_OK
