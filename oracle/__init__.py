"""FP64 CPU oracle for single-dish convolutional gridding -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP path
(``paper_2012_13173_amd``); the two meet only through the seeded input
generators in ``synth``.

What it computes (HCGrid, Wang et al. 2020):

* ``grid_allpairs`` / ``grid_cells`` -- Eq. (1) of Section 2.1: every cell's
  value is the kernel-weighted sum of the samples within the support radius,
  divided by the sum of the weights.  Gaussian kernel of Section 3.6 (iii),
  FP64, compensated sums (``hcg_oracle.c``).
* ``ang2pix`` and the ring tables -- the HEALPix ring scheme of Section 3.2.
* ``sort_keys`` -- the non-descending key-value sort of (pixel, sample index)
  of Section 3.3 step I (a stable library sort: ties keep input order).
* ``ring_csr`` -- the second-level lookup table of Section 3.3 step III: for
  each ring, the position in the sorted sample array where that ring begins,
  followed by an end sentinel.
* ``neighbours`` -- the samples within R of each listed cell (all pairs).
* ``grid_points`` -- Eq. (1) at arbitrary cell centres (the pixel centres of
  a projected WCS map, Section 2.1), with the kernel shapes of Section 3.6
  (iii) -- Gaussian, elliptical Gaussian, Gaussian-tapered sinc -- and
  per-channel flags (a non-finite value leaves its sample out of that channel,
  which then has its own weight sum).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hcg_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")
_lib = None


def build(verbose: bool = False) -> str:
    """Compile the C oracle into ``oracle/liborc.so`` (gcc, OpenMP, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-Wall", _SRC, "-o", _LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Kernel(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32), ("fwhm_deg", ctypes.c_double),
                ("fwhm_minor_deg", ctypes.c_double), ("pa_deg", ctypes.c_double),
                ("sinc_deg", ctypes.c_double), ("taper_deg", ctypes.c_double)]


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("lon0", ctypes.c_double),
                ("lat0", ctypes.c_double), ("dlon", ctypes.c_double), ("dlat", ctypes.c_double)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    i64, f64, vp = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    lib.orc_hpx_npix.restype = i64
    lib.orc_hpx_npix.argtypes = [i64]
    for name in ("orc_hpx_ring_npix", "orc_hpx_ring_start", "orc_hpx_pix2ring"):
        getattr(lib, name).restype = i64
        getattr(lib, name).argtypes = [i64, i64]
    lib.orc_hpx_ring_z.restype = f64
    lib.orc_hpx_ring_z.argtypes = [i64, i64]
    lib.orc_hpx_pix2ang.restype = None
    lib.orc_hpx_pix2ang.argtypes = [i64, i64, ctypes.POINTER(f64), ctypes.POINTER(f64)]
    lib.orc_hpx_ang2pix.restype = i64
    lib.orc_hpx_ang2pix.argtypes = [i64, f64, f64]
    lib.orc_hpx_ang2pix_many.restype = None
    lib.orc_hpx_ang2pix_many.argtypes = [i64, i64, vp, vp, vp]
    lib.orc_sigma_rad.restype = f64
    lib.orc_sigma_rad.argtypes = [f64]
    lib.orc_grid_allpairs.restype = ctypes.c_int
    lib.orc_grid_allpairs.argtypes = [i64, vp, vp, vp, i64, ctypes.POINTER(_Grid), f64, f64,
                                      vp, vp, vp]
    lib.orc_grid_cells.restype = ctypes.c_int
    lib.orc_grid_cells.argtypes = [i64, vp, vp, vp, i64, ctypes.POINTER(_Grid), f64, f64, i64,
                                   vp, vp, vp, vp]
    lib.orc_neighbours.restype = ctypes.c_int
    lib.orc_neighbours.argtypes = [i64, vp, vp, ctypes.POINTER(_Grid), f64, i64, vp, vp, vp, vp]
    lib.orc_grid_points.restype = ctypes.c_int
    lib.orc_grid_points.argtypes = [i64, vp, vp, vp, i64, i64, vp, vp, ctypes.POINTER(_Kernel),
                                    f64, ctypes.c_int, ctypes.c_int, vp, vp, vp]
    lib.orc_set_threads.restype = None
    lib.orc_set_threads.argtypes = [ctypes.c_int]
    lib.orc_max_threads.restype = ctypes.c_int
    lib.orc_max_threads.argtypes = []
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _grid(g) -> _Grid:
    return _Grid(int(g.nx), int(g.ny), float(g.lon0), float(g.lat0), float(g.dlon),
                 float(g.dlat))


def set_threads(n: int) -> None:
    _load().orc_set_threads(int(n))


def max_threads() -> int:
    return int(_load().orc_max_threads())


# --------------------------------------------------------------------------
# HEALPix ring scheme (Section 3.2)
# --------------------------------------------------------------------------

def npix(nside: int) -> int:
    return int(_load().orc_hpx_npix(nside))


def ring_npix(nside: int, ring: int) -> int:
    return int(_load().orc_hpx_ring_npix(nside, ring))


def ring_start(nside: int, ring: int) -> int:
    return int(_load().orc_hpx_ring_start(nside, ring))


def ring_z(nside: int, ring: int) -> float:
    return float(_load().orc_hpx_ring_z(nside, ring))


def pix2ring(nside: int, pix: int) -> int:
    return int(_load().orc_hpx_pix2ring(nside, int(pix)))


def pix2ang(nside: int, pix: int):
    lon, lat = ctypes.c_double(), ctypes.c_double()
    _load().orc_hpx_pix2ang(nside, int(pix), ctypes.byref(lon), ctypes.byref(lat))
    return lon.value, lat.value


def ang2pix(nside: int, lon_deg, lat_deg) -> np.ndarray:
    lon = np.ascontiguousarray(lon_deg, dtype=np.float64).ravel()
    lat = np.ascontiguousarray(lat_deg, dtype=np.float64).ravel()
    out = np.empty(lon.shape[0], dtype=np.int64)
    _load().orc_hpx_ang2pix_many(nside, lon.shape[0], _ptr(lon), _ptr(lat), _ptr(out))
    return out


# --------------------------------------------------------------------------
# Pre-ordering and the ring lookup table (Section 3.3, steps I and III)
# --------------------------------------------------------------------------

def sort_keys(keys: np.ndarray):
    """Non-descending sort of (key, n): returns (sorted keys, permutation).

    A stable library sort: equal keys keep increasing n, which is the order of
    the (key, n) pairs because n is unique.
    """
    keys = np.asarray(keys)
    perm = np.argsort(keys, kind="stable")
    return keys[perm], perm


def ring_csr(nside: int, sorted_pix: np.ndarray, ring_first: int, ring_last: int) -> np.ndarray:
    """Start of every ring ring_first..ring_last in the sorted pixel array.

    Entry r - ring_first is the number of sorted samples whose pixel lies before
    the first pixel of ring r; the final entry (ring_last + 1) is the end
    sentinel.
    """
    starts = np.array([ring_start(nside, r) for r in range(ring_first, ring_last + 1)]
                      + [ring_start(nside, ring_last + 1) if ring_last + 1 <= 4 * nside - 1
                         else npix(nside)], dtype=np.int64)
    return np.searchsorted(np.asarray(sorted_pix, dtype=np.int64), starts, side="left")


# --------------------------------------------------------------------------
# Gridding, Eq. (1)
# --------------------------------------------------------------------------

def sigma_rad(fwhm_deg: float) -> float:
    return float(_load().orc_sigma_rad(fwhm_deg))


def _inputs(lon, lat, spec):
    lon = np.ascontiguousarray(lon, dtype=np.float64).ravel()
    lat = np.ascontiguousarray(lat, dtype=np.float64).ravel()
    spec = np.ascontiguousarray(spec, dtype=np.float32)
    if spec.ndim == 1:
        spec = spec.reshape(-1, 1)
    if spec.shape[0] != lon.shape[0] or lat.shape[0] != lon.shape[0]:
        raise ValueError("lon, lat and spectra rows must have the same length")
    return lon, lat, spec


def grid_allpairs(lon, lat, spec, grid, fwhm_deg: float, support_deg: float):
    """Every (cell, sample) pair tested.  Returns (V [C, ny, nx], W [ny, nx], npairs)."""
    lon, lat, spec = _inputs(lon, lat, spec)
    n, C = spec.shape
    V = np.empty((C, grid.ny, grid.nx), dtype=np.float64)
    W = np.empty((grid.ny, grid.nx), dtype=np.float64)
    npairs = np.zeros(1, dtype=np.int64)
    g = _grid(grid)
    rc = _load().orc_grid_allpairs(n, _ptr(lon), _ptr(lat), _ptr(spec), C, ctypes.byref(g),
                                   fwhm_deg, support_deg, _ptr(V), _ptr(W), _ptr(npairs))
    if rc != 0:
        raise ValueError(f"orc_grid_allpairs failed ({rc})")
    return V, W, int(npairs[0])


def grid_cells(lon, lat, spec, grid, fwhm_deg: float, support_deg: float, cells):
    """Listed cells only (flat index iy*nx+ix), bucketed search.

    Returns (V [ncells, C], W [ncells], npair [ncells]).
    """
    lon, lat, spec = _inputs(lon, lat, spec)
    n, C = spec.shape
    cells = np.ascontiguousarray(cells, dtype=np.int64).ravel()
    V = np.empty((cells.shape[0], C), dtype=np.float64)
    W = np.empty(cells.shape[0], dtype=np.float64)
    npair = np.empty(cells.shape[0], dtype=np.int64)
    g = _grid(grid)
    rc = _load().orc_grid_cells(n, _ptr(lon), _ptr(lat), _ptr(spec), C, ctypes.byref(g),
                                fwhm_deg, support_deg, cells.shape[0], _ptr(cells), _ptr(V),
                                _ptr(W), _ptr(npair))
    if rc != 0:
        raise ValueError(f"orc_grid_cells failed ({rc})")
    return V, W, npair


def neighbours(lon, lat, grid, support_deg: float, cells):
    """For each listed cell, the sorted indices of samples with d <= R (all pairs)."""
    lon = np.ascontiguousarray(lon, dtype=np.float64).ravel()
    lat = np.ascontiguousarray(lat, dtype=np.float64).ravel()
    cells = np.ascontiguousarray(cells, dtype=np.int64).ravel()
    counts = np.empty(cells.shape[0], dtype=np.int64)
    g = _grid(grid)
    lib = _load()
    lib.orc_neighbours(lon.shape[0], _ptr(lon), _ptr(lat), ctypes.byref(g), support_deg,
                       cells.shape[0], _ptr(cells), _ptr(counts), None, None)
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    out = np.empty(int(offsets[-1]), dtype=np.int64)
    lib.orc_neighbours(lon.shape[0], _ptr(lon), _ptr(lat), ctypes.byref(g), support_deg,
                       cells.shape[0], _ptr(cells), _ptr(counts), _ptr(offsets), _ptr(out))
    return [out[offsets[q]:offsets[q + 1]] for q in range(cells.shape[0])]


# --------------------------------------------------------------------------
# Eq. (1) at arbitrary cell centres, kernel shapes and per-channel flags
# --------------------------------------------------------------------------

GAUSS, ELLIPTIC_GAUSS, TAPERED_SINC = 0, 1, 2


class Kernel:
    """A kernel w(g, n) of Section 3.6 (iii) (see ``hcg_oracle.c``):

    * ``Kernel.gauss(fwhm)`` -- exp(-d^2 / 2 sigma^2);
    * ``Kernel.elliptic(fwhm_major, fwhm_minor, pa_deg)`` -- a Gaussian with
      sigmas along the major axis (position angle ``pa_deg`` from north
      through east) and the minor axis, evaluated at the sample's bearing;
    * ``Kernel.tapered_sinc(b, a)`` -- sinc(d / b) exp(-(d / a)^2).
    All widths in degrees."""

    def __init__(self, type_, fwhm=0.0, fwhm_minor=0.0, pa=0.0, sinc=0.0, taper=0.0):
        self.type, self.fwhm, self.fwhm_minor = int(type_), float(fwhm), float(fwhm_minor)
        self.pa, self.sinc, self.taper = float(pa), float(sinc), float(taper)

    @classmethod
    def gauss(cls, fwhm_deg):
        return cls(GAUSS, fwhm=fwhm_deg)

    @classmethod
    def elliptic(cls, fwhm_major_deg, fwhm_minor_deg, pa_deg):
        return cls(ELLIPTIC_GAUSS, fwhm=fwhm_major_deg, fwhm_minor=fwhm_minor_deg, pa=pa_deg)

    @classmethod
    def tapered_sinc(cls, sinc_deg, taper_deg):
        return cls(TAPERED_SINC, sinc=sinc_deg, taper=taper_deg)

    def _c(self) -> _Kernel:
        return _Kernel(self.type, self.fwhm, self.fwhm_minor, self.pa, self.sinc, self.taper)


def grid_points(lon, lat, spec, cell_lon, cell_lat, support_deg: float, kernel: Kernel,
                masked: bool = False, allpairs: bool = False):
    """Eq. (1) at the listed cell centres (degrees; non-finite centres are
    cells without samples).  ``masked``: a non-finite spectrum value flags
    that sample in that channel only, which then has its own weight sum.

    Returns (V [ncells, C], W [ncells] or [ncells, C] when masked, npair [ncells])."""
    lon, lat, spec = _inputs(lon, lat, spec)
    n, C = spec.shape
    cl = np.ascontiguousarray(cell_lon, dtype=np.float64).ravel()
    cb = np.ascontiguousarray(cell_lat, dtype=np.float64).ravel()
    if cl.shape != cb.shape:
        raise ValueError("cell_lon and cell_lat must have the same length")
    V = np.empty((cl.shape[0], C), dtype=np.float64)
    W = np.empty((cl.shape[0], C) if masked else (cl.shape[0],), dtype=np.float64)
    npair = np.empty(cl.shape[0], dtype=np.int64)
    k = kernel._c()
    rc = _load().orc_grid_points(n, _ptr(lon), _ptr(lat), _ptr(spec), C, cl.shape[0], _ptr(cl),
                                 _ptr(cb), ctypes.byref(k), float(support_deg), int(bool(masked)),
                                 int(bool(allpairs)), _ptr(V), _ptr(W), _ptr(npair))
    if rc != 0:
        raise ValueError(f"orc_grid_points failed ({rc})")
    return V, W, npair
