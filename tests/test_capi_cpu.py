"""CPU-side checks of the C ABI: the library loads, exports every symbol that
include/cute.h declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1210_1833_amd as cute

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    with open(os.path.join(ROOT, "include", "cute.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cute_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(cute.library_path()):
        pytest.fail("libcute.so is not built (run __graft_entry__.build())")
    return cute.load()


def test_exports_every_declared_symbol(lib):
    declared = _declared_functions()
    assert set(cute.EXPORTED) == set(declared), declared
    for name in declared:
        assert hasattr(lib, name), name


def test_status_strings(lib):
    for s in range(6):
        assert lib.cute_status_string(s)
    assert lib.cute_status_string(99) == b"unknown status"


def test_build_grid_rejects_bad_arguments(lib):
    h = ctypes.c_void_p()
    p = cute.GridParams(cute.GEOM_BOX_OPEN, 0.0, 0.0, 0.0, 0, 0)
    x = np.zeros(4)
    # NULL output
    assert lib.cute_build_grid(x.ctypes.data, x.ctypes.data, x.ctypes.data, 4, ctypes.byref(p),
                               None, None) == cute.E_INVALID_ARG
    # negative n
    assert lib.cute_build_grid(x.ctypes.data, x.ctypes.data, x.ctypes.data, -1, ctypes.byref(p),
                               None, ctypes.byref(h)) == cute.E_INVALID_ARG
    # NULL coordinates
    assert lib.cute_build_grid(None, None, None, 4, ctypes.byref(p), None,
                               ctypes.byref(h)) == cute.E_INVALID_ARG
    # periodic box without a size, and r_max >= L/2
    pp = cute.GridParams(cute.GEOM_BOX_PERIODIC, 0.0, 0.0, 0.0, 0, 0)
    assert lib.cute_build_grid(x.ctypes.data, x.ctypes.data, x.ctypes.data, 4, ctypes.byref(pp),
                               None, ctypes.byref(h)) == cute.E_INVALID_ARG
    pp = cute.GridParams(cute.GEOM_BOX_PERIODIC, 10.0, 5.0, 0.0, 0, 0)
    assert lib.cute_build_grid(x.ctypes.data, x.ctypes.data, x.ctypes.data, 4, ctypes.byref(pp),
                               None, ctypes.byref(h)) == cute.E_INVALID_ARG
    # unknown geometry and negative cell size
    pg = cute.GridParams(7, 0.0, 0.0, 0.0, 0, 0)
    assert lib.cute_build_grid(x.ctypes.data, x.ctypes.data, x.ctypes.data, 4, ctypes.byref(pg),
                               None, ctypes.byref(h)) == cute.E_INVALID_ARG
    pc = cute.GridParams(cute.GEOM_BOX_OPEN, 0.0, 0.0, -1.0, 0, 0)
    assert lib.cute_build_grid(x.ctypes.data, x.ctypes.data, x.ctypes.data, 4, ctypes.byref(pc),
                               None, ctypes.byref(h)) == cute.E_INVALID_ARG
    assert lib.cute_last_error()


def test_count_and_estimators_reject_bad_binnings(lib):
    counts = np.zeros(4, dtype=np.uint64)
    good = cute.Binning(cute.BIN_MONO, [0.0, 1.0, 2.0])
    # NULL grid
    assert lib.cute_count_pairs(None, None, ctypes.byref(good.c()), 0, counts.ctypes.data, 0,
                                None, None) == cute.E_INVALID_ARG
    bad = [
        cute.Binning(cute.BIN_MONO, [0.0, 2.0, 1.0]),               # not increasing
        cute.Binning(cute.BIN_MONO, [-1.0, 1.0]),                   # negative
        cute.Binning(cute.BIN_MONO, [0.0, np.inf]),                 # not finite
        cute.Binning(cute.BIN_RMU, [0.0, 1.0], [0.0, 1.5]),         # mu above 1
        cute.Binning(cute.BIN_THETA, [0.0, 4.0]),                   # theta above pi
        cute.Binning(cute.BIN_MONO, [0.0, 1.0], [0.0, 1.0]),        # n2 for MONO
    ]
    dd = np.ones(4, dtype=np.uint64)
    xi = np.zeros(4)
    for b in bad:
        rc = lib.cute_xi_estimate(cute.EST_NATURAL, dd.ctypes.data, None, dd.ctypes.data, 10, 10,
                                  ctypes.byref(b.c()), 0.0,
                                  xi.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        assert rc == cute.E_INVALID_ARG
    sp = cute.Binning(cute.BIN_SIGMAPI, [0.0, 1.0], [0.0, 1.0], los=cute.LOS_Z)
    rc = lib.cute_xi_estimate(cute.EST_NATURAL, dd.ctypes.data, None, dd.ctypes.data, 10, 10,
                              ctypes.byref(sp.c()), 0.0,
                              xi.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert rc == cute.E_UNSUPPORTED
    # LS without DR, BOX on a non-MONO binning, too-small catalogs
    rmu = cute.Binning(cute.BIN_RMU, [0.0, 1.0], [0.0, 1.0])
    assert lib.cute_xi_estimate(cute.EST_LS, dd.ctypes.data, None, dd.ctypes.data, 10, 10,
                                ctypes.byref(good.c()), 0.0,
                                xi.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == cute.E_INVALID_ARG
    assert lib.cute_xi_estimate(cute.EST_BOX, dd.ctypes.data, None, None, 10, 10,
                                ctypes.byref(rmu.c()), 100.0,
                                xi.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == cute.E_INVALID_ARG
    assert lib.cute_xi_estimate(cute.EST_NATURAL, dd.ctypes.data, None, dd.ctypes.data, 1, 10,
                                ctypes.byref(good.c()), 0.0,
                                xi.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == cute.E_INVALID_ARG
    # odd multipole degree
    ells = np.array([1], dtype=np.int32)
    out = np.zeros(1)
    assert lib.cute_xi_multipoles(xi.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  ctypes.byref(rmu.c()), 1,
                                  ells.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                  out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == cute.E_INVALID_ARG


def test_batch_rejects_bad_arguments(lib):
    h = ctypes.c_void_p()
    items = (cute.CBatchItem * 1)()
    # no items, NULL output, NULL grid in an item: all rejected on the host
    assert lib.cute_batch_create(items, 0, cute.PREC_FP32_EDGE, None, ctypes.byref(h)) == cute.E_INVALID_ARG
    assert lib.cute_batch_create(items, 1, cute.PREC_FP32_EDGE, None, None) == cute.E_INVALID_ARG
    assert lib.cute_batch_create(items, 1, cute.PREC_FP32_EDGE, None, ctypes.byref(h)) == cute.E_INVALID_ARG
    assert b"grid a is NULL" in lib.cute_last_error()
    assert lib.cute_batch_run(None, 0, None) == cute.E_INVALID_ARG
    assert lib.cute_batch_layout(None, 0, None, None) == cute.E_INVALID_ARG
    lib.cute_batch_free(None)


def test_tune_grid_rejects_bad_arguments(lib):
    x = np.zeros(4)
    p = cute.GridParams(cute.GEOM_BOX_OPEN, 0.0, 0.0, 0.0, 0, 0)
    b = cute.Binning(cute.BIN_MONO, [0.0, 1.0, 2.0]).c()
    bc, bt = ctypes.c_double(), ctypes.c_int32()
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    bad = np.array([-1.0])
    badt = np.array([65], dtype=np.int32)
    X = (x.ctypes.data, x.ctypes.data, x.ctypes.data, 4)
    # NULL outputs, NULL params, negative side, tile size out of range, too many sides
    assert lib.cute_tune_grid(*X, ctypes.byref(p), ctypes.byref(b), 1, 0, None, 0, None, None,
                              None, None, None) == cute.E_INVALID_ARG
    assert lib.cute_tune_grid(*X, None, ctypes.byref(b), 1, 0, None, 0, None, None,
                              ctypes.byref(bc), ctypes.byref(bt), None) == cute.E_INVALID_ARG
    assert lib.cute_tune_grid(*X, ctypes.byref(p), ctypes.byref(b), 1, 1, bad.ctypes.data_as(dp),
                              0, None, None, ctypes.byref(bc), ctypes.byref(bt),
                              None) == cute.E_INVALID_ARG
    assert lib.cute_tune_grid(*X, ctypes.byref(p), ctypes.byref(b), 1, 0, None, 1,
                              badt.ctypes.data_as(ip), None, ctypes.byref(bc), ctypes.byref(bt),
                              None) == cute.E_INVALID_ARG
    assert lib.cute_tune_grid(*X, ctypes.byref(p), ctypes.byref(b), 1, 65, bad.ctypes.data_as(dp),
                              0, None, None, ctypes.byref(bc), ctypes.byref(bt),
                              None) == cute.E_INVALID_ARG
    # a grid's tile size must be in [0, 64]
    h = ctypes.c_void_p()
    pt = cute.GridParams(cute.GEOM_BOX_OPEN, 0.0, 0.0, 0.0, 0, 65)
    assert lib.cute_build_grid(*X, ctypes.byref(pt), None, ctypes.byref(h)) == cute.E_INVALID_ARG


def test_jackknife_rejects_bad_arguments(lib):
    b = cute.Binning(cute.BIN_MONO, [0.0, 1.0, 2.0]).c()
    reg = np.zeros(4, dtype=np.int32)
    out = np.zeros(8, dtype=np.uint64)
    # NULL grid, then a K out of range (checked before the grid is used)
    assert lib.cute_count_jackknife(None, reg.ctypes.data, 0, 1, ctypes.byref(b), 1,
                                    out.ctypes.data, out.ctypes.data, None, None) == cute.E_INVALID_ARG
    fake = ctypes.c_void_p(1)
    assert lib.cute_count_jackknife(fake, reg.ctypes.data, 0, 0, ctypes.byref(b), 1,
                                    out.ctypes.data, out.ctypes.data, None, None) == cute.E_INVALID_ARG
    assert lib.cute_count_jackknife(fake, None, 0, 4, ctypes.byref(b), 1,
                                    out.ctypes.data, out.ctypes.data, None, None) == cute.E_INVALID_ARG


def test_pixel_map_rejects_bad_arguments(lib):
    x = np.zeros(4)
    X = (x.ctypes.data, x.ctypes.data, x.ctypes.data)
    h = ctypes.c_void_p()
    ps = cute.GridParams(cute.GEOM_SPHERE, 0.0, 0.1, 0.0, 0, 0)
    pb = cute.GridParams(cute.GEOM_BOX_OPEN, 0.0, 0.1, 0.0, 0, 0)
    bad = [
        (X, 4, 16, 32, pb),                  # not SPHERE
        (X, 4, 0, 32, ps),                   # no rings
        (X, 4, 16, 7, ps),                   # fewer than 8 sectors
        (X, 4, 65536, 32768, ps),            # ids would not fit
        (X, -1, 16, 32, ps),                 # negative size
        ((None, None, None), 4, 16, 32, ps),  # NULL coordinates
    ]
    for xyz, n, nc, nph, p in bad:
        assert lib.cute_build_pixel_map(*xyz, n, nc, nph, ctypes.byref(p), None,
                                        ctypes.byref(h)) == cute.E_INVALID_ARG
    assert lib.cute_build_pixel_map(*X, 4, 16, 32, None, None, ctypes.byref(h)) == cute.E_INVALID_ARG
    assert lib.cute_build_pixel_map(*X, 4, 16, 32, ctypes.byref(ps), None, None) == cute.E_INVALID_ARG
    assert lib.cute_pixel_map_read(None, None, None, None) == cute.E_INVALID_ARG


def test_radial_rejects_bad_arguments(lib):
    e = np.linspace(0.0, 0.1, 5)
    z = np.zeros(4)
    out = np.zeros(4, dtype=np.uint64)
    dp = ctypes.POINTER(ctypes.c_double)
    assert lib.cute_count_radial(None, z.ctypes.data, None, None, 0, 0.01, 4, e.ctypes.data_as(dp),
                                 out.ctypes.data, 0, None, None) == cute.E_INVALID_ARG


def test_jackknife_cross_rejects_bad_arguments(lib):
    b = cute.Binning(cute.BIN_MONO, [0.0, 1.0, 2.0]).c()
    reg = np.zeros(4, dtype=np.int32)
    out = np.zeros(8, dtype=np.uint64)
    fake = ctypes.c_void_p(1)
    # NULL grids or labels, and a K out of range, are rejected before a grid is read
    for ga, ra, gb, rb, k in ((None, reg, fake, reg, 2), (fake, None, fake, reg, 2),
                              (fake, reg, None, reg, 2), (fake, reg, fake, None, 2),
                              (fake, reg, fake, reg, 0), (fake, reg, fake, reg, 70000)):
        assert lib.cute_count_jackknife_cross(
            ga, None if ra is None else ra.ctypes.data, gb, None if rb is None else rb.ctypes.data,
            0, k, ctypes.byref(b), 1, out.ctypes.data, out.ctypes.data, None, None) == cute.E_INVALID_ARG


def test_xi_estimate_exact_arithmetic_guard(lib):
    """The 128-bit exact Landy-Szalay evaluation accepts catalogs below 2^31
    points with counts up to their pair totals (the largest values give the
    exact closed form) and rejects anything larger instead of overflowing."""
    from fractions import Fraction
    good = cute.Binning(cute.BIN_MONO, [0.0, 1.0])
    xi = np.zeros(1)
    pxi = xi.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    n = (1 << 31) - 1
    top = n * (n - 1) // 2
    dd = np.array([top], dtype=np.uint64)
    dr = np.array([n * n], dtype=np.uint64)
    rr = np.array([top], dtype=np.uint64)
    assert lib.cute_xi_estimate(cute.EST_LS, dd.ctypes.data, dr.ctypes.data, rr.ctypes.data, n, n,
                                ctypes.byref(good.c()), 0.0, pxi) == cute.OK
    num = n * (n - 1) * top - (n - 1) * (n - 1) * (n * n) + n * (n - 1) * top
    assert xi[0] == float(Fraction(num, n * (n - 1) * top))
    # sizes at 2^31 and counts above their pair totals are refused
    for nd, nr in ((1 << 31, 10), (10, 1 << 31)):
        small = np.array([1], dtype=np.uint64)
        assert lib.cute_xi_estimate(cute.EST_LS, small.ctypes.data, small.ctypes.data,
                                    small.ctypes.data, nd, nr, ctypes.byref(good.c()), 0.0,
                                    pxi) == cute.E_INVALID_ARG
    for name in ("dd", "dr", "rr"):
        c = {"dd": np.array([45], dtype=np.uint64), "dr": np.array([100], dtype=np.uint64),
             "rr": np.array([45], dtype=np.uint64)}
        c[name] = c[name] + np.uint64(1)
        assert lib.cute_xi_estimate(cute.EST_LS, c["dd"].ctypes.data, c["dr"].ctypes.data,
                                    c["rr"].ctypes.data, 10, 10, ctypes.byref(good.c()), 0.0,
                                    pxi) == cute.E_INVALID_ARG, name


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: any other --gpus exits with status 2 and a
    message, before it touches a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "8"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
