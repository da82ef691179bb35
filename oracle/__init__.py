"""CPU FP64 oracle for binned pair counting and the 2PCF estimators.

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg are the only callers. The GPU library never
imports, links or runs anything from here, and this package never imports the
GPU library.

* ``count_pairs``: plain FP64 pair counting (``oracle.c``), the definition of
  the pair count in Sec. 2.2 of the paper evaluated pair by pair.
* ``pixel_map`` and ``count_weighted``: the pixelised angular correlation
  (Sec. 3.4): objects binned into equal-area (cos theta, phi) pixels, and pair
  counts in which each pixel carries its occupancy as a weight.
* ``count_radial``: the radial correlation (Sec. 2.1 and 3.4): pairs within
  an angular aperture, binned by their redshift difference.
* ``estimators``: the natural, Landy-Szalay and periodic-box estimators of
  Sec. 2.2 and the Legendre multipoles of Sec. 2.1, in exact rational
  arithmetic.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

from . import estimators  # noqa: F401  (re-exported)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "liboracle.so")
_lock = threading.Lock()
_lib = None

MONO, RMU, SIGMAPI, THETA = 0, 1, 2, 3
LOS_Z, LOS_MID = 0, 1


class _Binning(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int), ("los", ctypes.c_int), ("periodic", ctypes.c_int),
        ("L", ctypes.c_double),
        ("n1", ctypes.c_int), ("e1", ctypes.POINTER(ctypes.c_double)),
        ("n2", ctypes.c_int), ("e2", ctypes.POINTER(ctypes.c_double)),
    ]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C, OpenMP, no FP contraction)."""
    os.makedirs(_BUILD, exist_ok=True)
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-fexcess-precision=standard",
           "-Wall", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build(force=False)
            lib = ctypes.CDLL(_LIB)
            lib.oracle_count.restype = ctypes.c_int
            lib.oracle_count.argtypes = [
                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                ctypes.c_int, ctypes.POINTER(_Binning), ctypes.c_int, ctypes.c_int,
                ctypes.c_void_p]
            lib.oracle_classify.restype = ctypes.c_int
            lib.oracle_classify.argtypes = [ctypes.POINTER(_Binning), ctypes.c_void_p,
                                            ctypes.c_void_p]
            lib.oracle_rmax.restype = ctypes.c_double
            lib.oracle_rmax.argtypes = [ctypes.POINTER(_Binning)]
            lib.oracle_nbins.restype = ctypes.c_int
            lib.oracle_nbins.argtypes = [ctypes.POINTER(_Binning)]
            lib.oracle_pixel_ids.restype = ctypes.c_int
            lib.oracle_pixel_ids.argtypes = [ctypes.c_void_p] * 3 + [
                ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
            lib.oracle_pixel_centres.restype = ctypes.c_int
            lib.oracle_pixel_centres.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                                 ctypes.c_int] + [ctypes.c_void_p] * 3
            lib.oracle_count_radial.restype = ctypes.c_int
            lib.oracle_count_radial.argtypes = (
                [ctypes.c_void_p] * 4 + [ctypes.c_int64] + [ctypes.c_void_p] * 4
                + [ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_void_p,
                   ctypes.c_int, ctypes.c_void_p])
            lib.oracle_count_jackknife.restype = ctypes.c_int
            lib.oracle_count_jackknife.argtypes = (
                [ctypes.c_void_p] * 3 + [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int,
                                         ctypes.POINTER(_Binning), ctypes.c_int, ctypes.c_void_p,
                                         ctypes.c_void_p])
            lib.oracle_count_weighted.restype = ctypes.c_int
            lib.oracle_count_weighted.argtypes = (
                [ctypes.c_void_p] * 4 + [ctypes.c_int64] + [ctypes.c_void_p] * 4
                + [ctypes.c_int64, ctypes.c_int, ctypes.POINTER(_Binning), ctypes.c_int,
                   ctypes.c_void_p])
            _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Binning:
    """Binning description shared by the oracle's entry points.

    kind: MONO (r), RMU (r, mu), SIGMAPI (sigma, pi) or THETA (radians).
    edges1: n1+1 edges of r | sigma | theta; edges2: n2+1 edges of mu | pi.
    """

    def __init__(self, kind, edges1, edges2=None, los=LOS_Z, periodic=False, L=0.0):
        self.kind = int(kind)
        self.los = int(los)
        self.periodic = bool(periodic)
        self.L = float(L)
        self.edges1 = _f64(edges1)
        self.edges2 = None if edges2 is None else _f64(edges2)

    @property
    def shape(self):
        n1 = len(self.edges1) - 1
        return (n1,) if self.edges2 is None else (n1, len(self.edges2) - 1)

    def _c(self):
        b = _Binning()
        b.kind, b.los, b.periodic, b.L = self.kind, self.los, int(self.periodic), self.L
        b.n1 = len(self.edges1) - 1
        b.e1 = self.edges1.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        if self.edges2 is not None:
            b.n2 = len(self.edges2) - 1
            b.e2 = self.edges2.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        else:
            b.n2 = 0
            b.e2 = ctypes.POINTER(ctypes.c_double)()
        return b


def _xyz(cat):
    if hasattr(cat, "x"):
        return _f64(cat.x), _f64(cat.y), _f64(cat.z)
    a = np.asarray(cat, dtype=np.float64)
    return _f64(a[:, 0]), _f64(a[:, 1]), _f64(a[:, 2])


def count_pairs(a, b, binning: Binning, prune: bool = False, nthreads: int | None = None):
    """Pair counts as uint64, shaped like ``binning.shape``.

    ``b is None``: autocorrelation of ``a`` (unordered pairs i < j).
    Otherwise: cross-correlation, all pairs (i in a, j in b).
    ``prune`` uses the exact band-and-window prune (same counts, fewer pairs
    visited).
    """
    lib = _load()
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    is_auto = b is None
    xb, yb, zb = _xyz(a if is_auto else b)
    xa, ya, za = (xb, yb, zb) if is_auto else _xyz(a)
    cb = binning._c()
    nbins = lib.oracle_nbins(ctypes.byref(cb))
    out = np.zeros(nbins, dtype=np.uint64)
    rc = lib.oracle_count(xa.ctypes.data, ya.ctypes.data, za.ctypes.data, len(xa),
                          xb.ctypes.data, yb.ctypes.data, zb.ctypes.data, len(xb),
                          int(is_auto), ctypes.byref(cb), int(bool(prune)), int(nthreads),
                          out.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_count rejected its arguments (rc=%d)" % rc)
    return out.reshape(binning.shape)


def count_jackknife(cat, region, K: int, binning: Binning, nthreads: int | None = None):
    """Leave-one-region-out autocorrelations: ``(total, jack)`` with ``total``
    the counts of the whole catalog and ``jack[k]`` those of the catalog
    without the points whose ``region`` label is k (labels in [0, K))."""
    lib = _load()
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    x, y, z = _xyz(cat)
    reg = np.ascontiguousarray(region, dtype=np.int32)
    if len(reg) != len(x):
        raise ValueError("one region label per point")
    cb = binning._c()
    nbins = lib.oracle_nbins(ctypes.byref(cb))
    total = np.zeros(nbins, dtype=np.uint64)
    jack = np.zeros((int(K), nbins), dtype=np.uint64)
    rc = lib.oracle_count_jackknife(x.ctypes.data, y.ctypes.data, z.ctypes.data, len(x),
                                    reg.ctypes.data, int(K), ctypes.byref(cb), int(nthreads),
                                    total.ctypes.data, jack.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_count_jackknife rejected its arguments (rc=%d)" % rc)
    return total.reshape(binning.shape), jack.reshape((int(K),) + binning.shape)


def classify(p, q, binning: Binning) -> int:
    """Flattened bin of the ordered pair (p, q), or -1 if it is not counted."""
    lib = _load()
    pp = _f64(p)
    qq = _f64(q)
    cb = binning._c()
    return int(lib.oracle_classify(ctypes.byref(cb), pp.ctypes.data, qq.ctypes.data))


def rmax(binning: Binning) -> float:
    lib = _load()
    cb = binning._c()
    return float(lib.oracle_rmax(ctypes.byref(cb)))


def pixel_ids(cat, n_cth: int, n_phi: int):
    """Pixel id (ring * n_phi + sector) of every unit vector of ``cat``."""
    lib = _load()
    x, y, z = _xyz(cat)
    ids = np.zeros(len(x), dtype=np.int64)
    rc = lib.oracle_pixel_ids(x.ctypes.data, y.ctypes.data, z.ctypes.data, len(x),
                              int(n_cth), int(n_phi), ids.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_pixel_ids rejected its arguments (rc=%d)" % rc)
    return ids


def pixel_centres(ids, n_cth: int, n_phi: int):
    """Centres (x, y, z) of the pixels ``ids`` as FP64 unit vectors."""
    lib = _load()
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    out = [np.zeros(len(ids)) for _ in range(3)]
    rc = lib.oracle_pixel_centres(ids.ctypes.data, len(ids), int(n_cth), int(n_phi),
                                  *[o.ctypes.data for o in out])
    if rc != 0:
        raise ValueError("oracle_pixel_centres rejected its arguments (rc=%d)" % rc)
    return out


class PixelMap:
    """Non-empty pixels of a catalog in ascending id order: ``ids`` (int64),
    ``counts`` (uint32 occupancy) and the centre coordinates ``x, y, z``."""

    def __init__(self, ids, counts, n_cth, n_phi):
        self.ids = ids
        self.counts = counts
        self.n_cth, self.n_phi = n_cth, n_phi
        self.x, self.y, self.z = pixel_centres(ids, n_cth, n_phi)

    def __len__(self):
        return len(self.ids)


def pixel_map(cat, n_cth: int, n_phi: int) -> PixelMap:
    ids, counts = np.unique(pixel_ids(cat, n_cth, n_phi), return_counts=True)
    return PixelMap(ids, counts.astype(np.uint32), n_cth, n_phi)


def count_weighted(a, wa, b, wb, binning: Binning, nthreads: int | None = None):
    """Weighted pair counts (uint64): each pair adds ``wa[i] * wb[j]``.
    ``b is None``: autocorrelation of ``a`` (pairs i < j plus the
    ``wa[i] (wa[i] - 1) / 2`` pairs inside each pixel, at zero separation)."""
    lib = _load()
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    is_auto = b is None
    if is_auto:
        b, wb = a, wa
    xa, ya, za = _xyz(a)
    xb, yb, zb = _xyz(b)
    wa = np.ascontiguousarray(wa, dtype=np.uint32)
    wb = np.ascontiguousarray(wb, dtype=np.uint32)
    if len(wa) != len(xa) or len(wb) != len(xb):
        raise ValueError("one weight per point")
    cb = binning._c()
    out = np.zeros(lib.oracle_nbins(ctypes.byref(cb)), dtype=np.uint64)
    rc = lib.oracle_count_weighted(xa.ctypes.data, ya.ctypes.data, za.ctypes.data, wa.ctypes.data,
                                   len(xa), xb.ctypes.data, yb.ctypes.data, zb.ctypes.data,
                                   wb.ctypes.data, len(xb), int(is_auto), ctypes.byref(cb),
                                   int(nthreads), out.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_count_weighted rejected its arguments (rc=%d)" % rc)
    return out.reshape(binning.shape)


def count_radial(a, ra, b, rb, aperture: float, edges, nthreads: int | None = None):
    """Radial pair counts (uint64, one per bin of ``edges``): pairs of unit
    vectors closer than ``aperture`` radians, binned by |ra[i] - rb[j]|.
    ``b is None``: autocorrelation of ``a`` (pairs i < j)."""
    lib = _load()
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    is_auto = b is None
    if is_auto:
        b, rb = a, ra
    xa, ya, za = _xyz(a)
    xb, yb, zb = _xyz(b)
    ra, rb, e = _f64(ra), _f64(rb), _f64(edges)
    if len(ra) != len(xa) or len(rb) != len(xb):
        raise ValueError("one redshift per point")
    out = np.zeros(len(e) - 1, dtype=np.uint64)
    rc = lib.oracle_count_radial(xa.ctypes.data, ya.ctypes.data, za.ctypes.data, ra.ctypes.data,
                                 len(xa), xb.ctypes.data, yb.ctypes.data, zb.ctypes.data,
                                 rb.ctypes.data, len(xb), int(is_auto), float(aperture),
                                 len(e) - 1, e.ctypes.data, int(nthreads), out.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_count_radial rejected its arguments (rc=%d)" % rc)
    return out
