"""Python binding of libhcg.so, the MI355X convolutional gridding library.

Argument marshalling only: every step of the gridding path runs in the HIP
kernels of ``csrc/`` behind the C ABI of ``include/hcg.h``.  PyTorch provides
device memory and streams.  The binding raises if the compiled library is
missing; there is no fallback implementation.

Names mirror the C ABI: ``hcg_plan``, ``hcg_grid``, ``hcg_destroy``,
``hcg_quantize``, ``hcg_plan_batch``, ``hcg_grid_batch``, ``hcg_ang2pix``,
``hcg_sort_keys``, ``hcg_get_plan_info``, ``hcg_export``,
``hcg_get_plan_stats``.
"""
from __future__ import annotations

import ctypes
import math
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhcg.so")

HCG_OK, HCG_E_ARG, HCG_E_NOMEM, HCG_E_DEVICE, HCG_E_UNSUPPORTED, HCG_E_STATE = range(6)
(HCG_F32, HCG_BF16, HCG_BF16_SPLIT, HCG_F16_SCALED, HCG_FP8E4M3_SCALED,
 HCG_FP8E4M3_SPLIT) = range(6)
HCG_ARR_KEYS, HCG_ARR_PERM, HCG_ARR_RING_CSR, HCG_ARR_TILE_NRANGES, HCG_ARR_TILE_RANGES = range(5)
HCG_KERNEL_GAUSS, HCG_KERNEL_ELLIPTIC_GAUSS, HCG_KERNEL_TAPERED_SINC = range(3)
HCG_PROJ_CAR, HCG_PROJ_SFL, HCG_PROJ_SIN, HCG_PROJ_TAN = range(4)
HCG_BATCH_PERSISTENT, HCG_BATCH_ITEMS = 1, 2
PROJECTIONS = {"CAR": HCG_PROJ_CAR, "SFL": HCG_PROJ_SFL, "SIN": HCG_PROJ_SIN, "TAN": HCG_PROJ_TAN}
STATUS_NAMES = {0: "HCG_OK", 1: "HCG_E_ARG", 2: "HCG_E_NOMEM", 3: "HCG_E_DEVICE",
                4: "HCG_E_UNSUPPORTED", 5: "HCG_E_STATE"}


class HcgError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class GridDescC(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("lon0_deg", ctypes.c_double),
                ("lat0_deg", ctypes.c_double), ("dlon_deg", ctypes.c_double),
                ("dlat_deg", ctypes.c_double)]


class OptsC(ctypes.Structure):
    _fields_ = [("nside", ctypes.c_int32), ("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32),
                ("coarsen", ctypes.c_int32), ("chan_tile", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


class KernelC(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32), ("fwhm_deg", ctypes.c_double),
                ("fwhm_minor_deg", ctypes.c_double), ("pa_deg", ctypes.c_double),
                ("sinc_deg", ctypes.c_double), ("taper_deg", ctypes.c_double)]


class CellCentresC(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("lon_deg", ctypes.c_void_p),
                ("lat_deg", ctypes.c_void_p)]


class WcsC(ctypes.Structure):
    _fields_ = [("proj", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("lonpole_set", ctypes.c_int32), ("crpix1", ctypes.c_double),
                ("crpix2", ctypes.c_double), ("cdelt1", ctypes.c_double),
                ("cdelt2", ctypes.c_double), ("crval1", ctypes.c_double),
                ("crval2", ctypes.c_double), ("lonpole", ctypes.c_double),
                ("latpole", ctypes.c_double)]


class PlanInfoC(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nside", ctypes.c_int32), ("key_bits", ctypes.c_int32),
                ("pix_base", ctypes.c_uint32), ("pix_max", ctypes.c_uint32),
                ("ring_first", ctypes.c_int32), ("ring_last", ctypes.c_int32),
                ("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32),
                ("ntiles_x", ctypes.c_int32), ("ntiles_y", ctypes.c_int32),
                ("max_ranges", ctypes.c_int32), ("sort_passes", ctypes.c_int32),
                ("sigma_rad", ctypes.c_double), ("support_rad", ctypes.c_double)]


class PlanStatsC(ctypes.Structure):
    _fields_ = [("pairs", ctypes.c_int64), ("candidates", ctypes.c_int64),
                ("cells", ctypes.c_int64)]


class FieldDescC(ctypes.Structure):
    _fields_ = [("lon_deg", ctypes.c_void_p), ("lat_deg", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("grid", GridDescC), ("fwhm_deg", ctypes.c_double),
                ("support_deg", ctypes.c_double)]


class FieldDataC(ctypes.Structure):
    _fields_ = [("spectra", ctypes.c_void_p), ("nchan", ctypes.c_int64),
                ("dtype", ctypes.c_int32), ("chan_scale", ctypes.c_void_p),
                ("cube", ctypes.c_void_p), ("weights", ctypes.c_void_p)]


class BatchInfoC(ctypes.Structure):
    _fields_ = [("nfields", ctypes.c_int32), ("chan_slab", ctypes.c_int32),
                ("cost_order", ctypes.c_int32), ("tuned", ctypes.c_int32),
                ("graph_captured", ctypes.c_int32), ("persistent_blocks", ctypes.c_int32),
                ("items", ctypes.c_int64), ("tune_ms", ctypes.c_double * 8),
                ("launch", ctypes.c_int32), ("reserved", ctypes.c_int32)]


EXPORTED = ["hcg_plan", "hcg_grid", "hcg_destroy", "hcg_last_error", "hcg_get_plan_info",
            "hcg_export", "hcg_export_size", "hcg_get_plan_stats", "hcg_ang2pix",
            "hcg_sort_keys", "hcg_quantize", "hcg_plan_batch", "hcg_grid_batch",
            "hcg_destroy_batch", "hcg_get_batch_info", "hcg_quantize_packed", "hcg_grid_packed",
            "hcg_packed_bytes", "hcg_grid_host", "hcg_grid_rowthreads", "hcg_plan_ex",
            "hcg_grid_masked", "hcg_wcs_centres", "hcg_grid_noalloc", "hcg_batch_get_plan"]

_lib = None


def load(path: str = LIB_PATH):
    """Loads libhcg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2012_13173_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i64, i32, f64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    lib.hcg_plan.argtypes = [ctypes.POINTER(vp), vp, vp, i64, ctypes.POINTER(GridDescC), f64, f64,
                             ctypes.POINTER(OptsC), vp]
    lib.hcg_grid.argtypes = [vp, vp, i64, ctypes.c_int, vp, vp, vp, vp]
    lib.hcg_grid_noalloc.argtypes = [vp, vp, i64, ctypes.c_int, vp, vp, vp, vp]
    lib.hcg_plan_ex.argtypes = [ctypes.POINTER(vp), vp, vp, i64, ctypes.POINTER(GridDescC),
                                ctypes.POINTER(CellCentresC), ctypes.POINTER(KernelC), f64,
                                ctypes.POINTER(OptsC), vp]
    lib.hcg_grid_masked.argtypes = [vp, vp, i64, vp, vp, vp]
    lib.hcg_wcs_centres.argtypes = [ctypes.POINTER(WcsC), vp, vp, vp]
    lib.hcg_destroy.argtypes = [vp]
    lib.hcg_last_error.restype = ctypes.c_char_p
    lib.hcg_last_error.argtypes = []
    lib.hcg_get_plan_info.argtypes = [vp, ctypes.POINTER(PlanInfoC)]
    lib.hcg_export.argtypes = [vp, ctypes.c_int, vp, i64, vp]
    lib.hcg_export_size.argtypes = [vp, ctypes.c_int, ctypes.POINTER(i64)]
    lib.hcg_get_plan_stats.argtypes = [vp, ctypes.POINTER(PlanStatsC), vp]
    lib.hcg_ang2pix.argtypes = [vp, vp, i64, i32, vp, vp]
    lib.hcg_sort_keys.argtypes = [vp, i64, i32, vp, vp, vp]
    lib.hcg_quantize.argtypes = [vp, i64, i64, ctypes.c_int, vp, vp, vp]
    lib.hcg_quantize_packed.argtypes = [vp, vp, i64, ctypes.c_int, vp, vp, vp]
    lib.hcg_grid_packed.argtypes = [vp, vp, i64, ctypes.c_int, vp, vp, vp, vp]
    lib.hcg_packed_bytes.argtypes = [vp, i64, ctypes.c_int, ctypes.POINTER(i64)]
    lib.hcg_grid_host.argtypes = [vp, vp, i64, ctypes.c_int, vp, i64, vp, vp, vp]
    lib.hcg_grid_rowthreads.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, vp, vp, vp]
    lib.hcg_plan_batch.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(FieldDescC),
                                   ctypes.POINTER(OptsC), vp]
    lib.hcg_grid_batch.argtypes = [vp, ctypes.POINTER(FieldDataC), vp]
    lib.hcg_destroy_batch.argtypes = [vp]
    lib.hcg_get_batch_info.argtypes = [vp, ctypes.POINTER(BatchInfoC)]
    lib.hcg_batch_get_plan.argtypes = [vp, i32, ctypes.POINTER(vp)]
    for name in EXPORTED:
        if name != "hcg_last_error":
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(st: int, where: str) -> None:
    if st != HCG_OK:
        raise HcgError(st, where, load().hcg_last_error().decode())


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dptr(t, dtype, name):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor")
    return ctypes.c_void_p(t.data_ptr())


def grid_desc(g) -> GridDescC:
    return GridDescC(int(g.nx), int(g.ny), float(g.lon0), float(g.lat0), float(g.dlon),
                     float(g.dlat))


class Plan:
    """Owns an hcg_plan_t; destroyed explicitly or on garbage collection."""

    def __init__(self, handle: ctypes.c_void_p, grid, n: int):
        self.handle = handle
        self.grid = grid
        self.n = int(n)

    def info(self) -> dict:
        out = PlanInfoC()
        _check(load().hcg_get_plan_info(self.handle, ctypes.byref(out)), "hcg_get_plan_info")
        return {k: getattr(out, k) for k, _ in PlanInfoC._fields_}

    def export(self, which: int, stream=None) -> torch.Tensor:
        nbytes = ctypes.c_int64()
        _check(load().hcg_export_size(self.handle, which, ctypes.byref(nbytes)), "hcg_export_size")
        dst = torch.empty(nbytes.value // 4, dtype=torch.int32, device="cuda")
        _check(load().hcg_export(self.handle, which, ctypes.c_void_p(dst.data_ptr()), nbytes.value,
                                 _stream(stream)), "hcg_export")
        return dst

    def stats(self, stream=None) -> dict:
        out = PlanStatsC()
        _check(load().hcg_get_plan_stats(self.handle, ctypes.byref(out), _stream(stream)),
               "hcg_get_plan_stats")
        return {k: getattr(out, k) for k, _ in PlanStatsC._fields_}

    def destroy(self) -> None:
        if self.handle is not None and load() is not None:
            h, self.handle = self.handle, None
            _check(load().hcg_destroy(h), "hcg_destroy")

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def hcg_plan(lon: torch.Tensor, lat: torch.Tensor, grid, fwhm_deg: float, support_deg: float,
             nside: int = 0, stream=None) -> Plan:
    """Builds a plan from device float64 lon/lat (degrees) for ``grid``."""
    lib = load()
    n = int(lon.shape[0])
    if int(lat.shape[0]) != n:
        raise ValueError("lon and lat must have the same length")
    handle = ctypes.c_void_p()
    g = grid_desc(grid)
    opts = OptsC(int(nside), 0, 0, 0, 0, 0)
    st = lib.hcg_plan(ctypes.byref(handle), _dptr(lon, torch.float64, "lon"),
                      _dptr(lat, torch.float64, "lat"), n, ctypes.byref(g), float(fwhm_deg),
                      float(support_deg), ctypes.byref(opts), _stream(stream))
    _check(st, "hcg_plan")
    return Plan(handle, grid, n)


class Kernel:
    """A kernel shape of ``hcg_plan_ex`` (widths in degrees):
    ``Kernel.gauss(fwhm)``, ``Kernel.elliptic(fwhm_major, fwhm_minor, pa_deg)``,
    ``Kernel.tapered_sinc(sinc_deg, taper_deg)``."""

    def __init__(self, type_, fwhm=0.0, fwhm_minor=0.0, pa=0.0, sinc=0.0, taper=0.0):
        self.c = KernelC(int(type_), float(fwhm), float(fwhm_minor), float(pa), float(sinc),
                         float(taper))

    @classmethod
    def gauss(cls, fwhm_deg):
        return cls(HCG_KERNEL_GAUSS, fwhm=fwhm_deg)

    @classmethod
    def elliptic(cls, fwhm_major_deg, fwhm_minor_deg, pa_deg):
        return cls(HCG_KERNEL_ELLIPTIC_GAUSS, fwhm=fwhm_major_deg, fwhm_minor=fwhm_minor_deg,
                   pa=pa_deg)

    @classmethod
    def tapered_sinc(cls, sinc_deg, taper_deg):
        return cls(HCG_KERNEL_TAPERED_SINC, sinc=sinc_deg, taper=taper_deg)


class CellGrid:
    """Shape of a target given by cell centres (what ``Plan.grid`` needs)."""

    def __init__(self, nx: int, ny: int):
        self.nx, self.ny = int(nx), int(ny)


def hcg_plan_ex(lon: torch.Tensor, lat: torch.Tensor, kernel: Kernel, support_deg: float,
                grid=None, cell_lon=None, cell_lat=None, nside: int = 0, stream=None) -> Plan:
    """Plan for any kernel shape, on a linear ``grid`` or on cell centres
    ``cell_lon`` / ``cell_lat`` (device float64 [ny, nx], degrees)."""
    lib = load()
    n = int(lon.shape[0])
    if int(lat.shape[0]) != n:
        raise ValueError("lon and lat must have the same length")
    if (grid is None) == (cell_lon is None):
        raise ValueError("give exactly one of grid and cell_lon / cell_lat")
    handle = ctypes.c_void_p()
    opts = OptsC(int(nside), 0, 0, 0, 0, 0)
    if grid is not None:
        g = grid_desc(grid)
        st = lib.hcg_plan_ex(ctypes.byref(handle), _dptr(lon, torch.float64, "lon"),
                             _dptr(lat, torch.float64, "lat"), n, ctypes.byref(g), None,
                             ctypes.byref(kernel.c), float(support_deg), ctypes.byref(opts),
                             _stream(stream))
        shape = grid
    else:
        if cell_lon.dim() != 2 or tuple(cell_lat.shape) != tuple(cell_lon.shape):
            raise ValueError("cell_lon and cell_lat must be [ny, nx] of the same shape")
        ny, nx = (int(x) for x in cell_lon.shape)
        cc = CellCentresC(nx, ny, _dptr(cell_lon, torch.float64, "cell_lon"),
                          _dptr(cell_lat, torch.float64, "cell_lat"))
        st = lib.hcg_plan_ex(ctypes.byref(handle), _dptr(lon, torch.float64, "lon"),
                             _dptr(lat, torch.float64, "lat"), n, None, ctypes.byref(cc),
                             ctypes.byref(kernel.c), float(support_deg), ctypes.byref(opts),
                             _stream(stream))
        shape = CellGrid(nx, ny)
    _check(st, "hcg_plan_ex")
    return Plan(handle, shape, n)


def hcg_wcs_centres(proj, nx: int, ny: int, crpix, cdelt, crval, lonpole=None, latpole=90.0,
                    device="cuda", stream=None):
    """World coordinates (degrees) of the pixel centres of a CAR / SFL / SIN /
    TAN map: device float64 (lon [ny, nx], lat [ny, nx])."""
    p = PROJECTIONS[proj.upper()] if isinstance(proj, str) else int(proj)
    w = WcsC(p, int(nx), int(ny), 0 if lonpole is None else 1, float(crpix[0]), float(crpix[1]),
             float(cdelt[0]), float(cdelt[1]), float(crval[0]), float(crval[1]),
             0.0 if lonpole is None else float(lonpole), float(latpole))
    lon = torch.empty((int(ny), int(nx)), dtype=torch.float64, device=device)
    lat = torch.empty_like(lon)
    _check(load().hcg_wcs_centres(ctypes.byref(w), ctypes.c_void_p(lon.data_ptr()),
                                  ctypes.c_void_p(lat.data_ptr()), _stream(stream)),
           "hcg_wcs_centres")
    return lon, lat


def hcg_grid_masked(plan: Plan, spectra: torch.Tensor, cube: torch.Tensor, chan_weights=None,
                    stream=None) -> None:
    """Eq. (1) with per-channel flags: non-finite values of ``spectra`` [n, C]
    (float32) are left out of their channel; ``cube`` [C, ny, nx] gets V and
    ``chan_weights`` [C, ny, nx] (or None) each channel's W."""
    if spectra.dim() != 2 or int(spectra.shape[0]) != plan.n:
        raise ValueError(f"spectra must be [{plan.n}, nchan]")
    C = int(spectra.shape[1])
    g = plan.grid
    if tuple(cube.shape) != (C, g.ny, g.nx):
        raise ValueError(f"cube must be [{C}, {g.ny}, {g.nx}]")
    if chan_weights is not None and tuple(chan_weights.shape) != (C, g.ny, g.nx):
        raise ValueError(f"chan_weights must be [{C}, {g.ny}, {g.nx}]")
    st = load().hcg_grid_masked(plan.handle, _dptr(spectra, torch.float32, "spectra"), C,
                                _dptr(cube, torch.float32, "cube"),
                                _dptr(chan_weights, torch.float32, "chan_weights"),
                                _stream(stream))
    _check(st, "hcg_grid_masked")


# storage dtype of each form's spectra and the shape prefix of its buffer
_FORM_STORAGE = {HCG_F32: (torch.float32, ()), HCG_BF16: (torch.bfloat16, ()),
                 HCG_BF16_SPLIT: (torch.bfloat16, (2,)), HCG_F16_SCALED: (torch.float16, ()),
                 HCG_FP8E4M3_SCALED: (torch.uint8, ()), HCG_FP8E4M3_SPLIT: (torch.uint8, (2,))}


def hcg_grid(plan: Plan, spectra: torch.Tensor, cube: torch.Tensor, weights=None,
             dtype: int = HCG_F32, chan_scale=None, stream=None) -> None:
    """Grids ``spectra`` ([n, C], or [2, n, C] for the split forms) into
    ``cube`` [C, ny, nx] (and ``weights`` [ny, nx])."""
    _grid_call("hcg_grid", plan, spectra, cube, weights, dtype, chan_scale, stream)


def hcg_grid_noalloc(plan: Plan, spectra: torch.Tensor, cube: torch.Tensor, weights=None,
                     dtype: int = HCG_F32, chan_scale=None, stream=None) -> None:
    """``hcg_grid`` through the entry point that allocates no device memory
    (its scratch is a static device array shared by every call on a device:
    calls that overlap on one device race)."""
    _grid_call("hcg_grid_noalloc", plan, spectra, cube, weights, dtype, chan_scale, stream)


def _grid_call(name, plan, spectra, cube, weights, dtype, chan_scale, stream):
    sdt, prefix = _FORM_STORAGE[dtype]
    if spectra.dim() != 2 + len(prefix) or tuple(spectra.shape[:len(prefix)]) != prefix:
        raise ValueError(f"spectra must be [{', '.join(map(str, prefix + ('n', 'nchan')))}]")
    if int(spectra.shape[-2]) != plan.n:
        raise ValueError(f"spectra has {int(spectra.shape[-2])} rows, the plan {plan.n} samples")
    C = int(spectra.shape[-1])
    g = plan.grid
    if tuple(cube.shape) != (C, g.ny, g.nx):
        raise ValueError(f"cube must be [{C}, {g.ny}, {g.nx}]")
    if weights is not None and tuple(weights.shape) != (g.ny, g.nx):
        raise ValueError(f"weights must be [{g.ny}, {g.nx}]")
    sp = _dptr(spectra, sdt, "spectra")
    st = getattr(load(), name)(plan.handle, sp, C, int(dtype),
                               _dptr(chan_scale, torch.float32, "chan_scale"),
                               _dptr(cube, torch.float32, "cube"),
                               _dptr(weights, torch.float32, "weights"), _stream(stream))
    _check(st, name)


def _hptr(t, name, dtype=torch.float32):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cpu":
        raise TypeError(f"{name} must be a CPU tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor")
    return ctypes.c_void_p(t.data_ptr())


def hcg_grid_host(plan: Plan, spectra: torch.Tensor, cube: torch.Tensor, weights=None,
                  slab: int = 0, dtype: int = HCG_F32, chan_scale=None, stream=None) -> None:
    """Grids host spectra ([n, C], or [2, n, C] for the split forms, in the
    storage of ``dtype``) into the host cube [C, ny, nx] (and weights
    [ny, nx]) in channel slabs streamed through the device; ``chan_scale`` is
    a host float32 [C] for the scaled forms.  Synchronous.  Page-locked
    tensors (``pin_memory()``) let the copies overlap the gridding."""
    sdt, prefix = _FORM_STORAGE[dtype]
    if spectra.dim() != 2 + len(prefix) or tuple(spectra.shape[:len(prefix)]) != prefix:
        raise ValueError(f"spectra must be [{', '.join(map(str, prefix + ('n', 'nchan')))}]")
    n, C = int(spectra.shape[-2]), int(spectra.shape[-1])
    if n != plan.n:
        raise ValueError(f"spectra has {n} rows, the plan {plan.n} samples")
    g = plan.grid
    if tuple(cube.shape) != (C, g.ny, g.nx):
        raise ValueError(f"cube must be [{C}, {g.ny}, {g.nx}]")
    if weights is not None and tuple(weights.shape) != (g.ny, g.nx):
        raise ValueError(f"weights must be [{g.ny}, {g.nx}]")
    if chan_scale is not None and tuple(chan_scale.shape) != (C,):
        raise ValueError(f"chan_scale must be [{C}]")
    st = load().hcg_grid_host(plan.handle, _hptr(spectra, "spectra", sdt), C, int(dtype),
                              _hptr(chan_scale, "chan_scale"), int(slab), _hptr(cube, "cube"),
                              _hptr(weights, "weights"), _stream(stream))
    _check(st, "hcg_grid_host")


def hcg_grid_rowthreads(plan: Plan, spectra: torch.Tensor, out: torch.Tensor, weights=None,
                        gamma: int = 1, block: int = 64, stream=None) -> None:
    """The paper's thread-per-row-cells gather on one channel: ``spectra`` [n]
    into ``out`` [ny, nx] (and ``weights`` [ny, nx]), ``gamma`` cells per
    thread, ``block`` threads per block."""
    g = plan.grid
    if spectra.dim() != 1 or int(spectra.shape[0]) != plan.n:
        raise ValueError("spectra must be [n] with the plan's sample count")
    if tuple(out.shape) != (g.ny, g.nx):
        raise ValueError(f"out must be [{g.ny}, {g.nx}]")
    if weights is not None and tuple(weights.shape) != (g.ny, g.nx):
        raise ValueError(f"weights must be [{g.ny}, {g.nx}]")
    st = load().hcg_grid_rowthreads(plan.handle, _dptr(spectra, torch.float32, "spectra"),
                                    int(gamma), int(block), _dptr(out, torch.float32, "out"),
                                    _dptr(weights, torch.float32, "weights"), _stream(stream))
    _check(st, "hcg_grid_rowthreads")


def hcg_quantize(spectra: torch.Tensor, dtype: int, stream=None):
    """Encodes float32 spectra [n, C] for a low-precision form.

    Returns (encoded tensor in the form's storage dtype, chan_scale or None)."""
    n, C = (int(x) for x in spectra.shape)
    sdt, prefix = _FORM_STORAGE[dtype]
    out = torch.empty(prefix + (n, C), dtype=sdt, device=spectra.device)
    scaled = dtype in (HCG_F16_SCALED, HCG_FP8E4M3_SCALED, HCG_FP8E4M3_SPLIT)
    scale = torch.empty(C, dtype=torch.float32, device=spectra.device) if scaled else None
    st = load().hcg_quantize(_dptr(spectra, torch.float32, "spectra"), n, C, int(dtype),
                             ctypes.c_void_p(out.data_ptr()),
                             _dptr(scale, torch.float32, "chan_scale"), _stream(stream))
    _check(st, "hcg_quantize")
    return out, scale


def _packed_shape(plan: Plan, C: int, dtype: int):
    sdt, prefix = _FORM_STORAGE[dtype]
    if dtype == HCG_F32:
        raise ValueError("plan-ordered spectra are a low-precision form")
    n = plan.n
    planes = prefix[0] if prefix else 1
    nbytes = ctypes.c_int64()
    _check(load().hcg_packed_bytes(plan.handle, C, int(dtype), ctypes.byref(nbytes)),
           "hcg_packed_bytes")
    shape = (planes, (n + 7) // 8, (C + 15) // 16 * 16, 8)
    assert nbytes.value == math.prod(shape) * torch.empty((), dtype=sdt).element_size()
    return sdt, shape, n


def hcg_quantize_packed(plan: Plan, spectra: torch.Tensor, dtype: int, stream=None):
    """Encodes float32 spectra [n, C] (in the sample order given to the plan)
    for a low-precision form in the plan's sorted order: [planes, ceil(n/8), Cp,
    8] with Cp = C rounded up to 16, the 8 sorted samples of a group
    contiguous per channel (zero padding past n and C).

    Returns (encoded tensor, chan_scale or None)."""
    n, C = (int(x) for x in spectra.shape)
    sdt, shape, pn = _packed_shape(plan, C, dtype)
    if n != pn:
        raise ValueError(f"spectra has {n} rows, the plan {pn} samples")
    out = torch.empty(shape, dtype=sdt, device=spectra.device)
    scaled = dtype in (HCG_F16_SCALED, HCG_FP8E4M3_SCALED, HCG_FP8E4M3_SPLIT)
    scale = torch.empty(C, dtype=torch.float32, device=spectra.device) if scaled else None
    st = load().hcg_quantize_packed(plan.handle, _dptr(spectra, torch.float32, "spectra"), C,
                                    int(dtype), ctypes.c_void_p(out.data_ptr()),
                                    _dptr(scale, torch.float32, "chan_scale"), _stream(stream))
    _check(st, "hcg_quantize_packed")
    return out, scale


def hcg_grid_packed(plan: Plan, packed: torch.Tensor, cube: torch.Tensor, weights=None,
                    dtype: int = HCG_F16_SCALED, chan_scale=None, stream=None) -> None:
    """Grids plan-ordered spectra (from ``hcg_quantize_packed``) into ``cube``
    [C, ny, nx] (and ``weights`` [ny, nx])."""
    C = int(cube.shape[0])
    sdt, shape, _ = _packed_shape(plan, max(C, 1), dtype)
    if tuple(packed.shape) != shape:
        raise ValueError(f"packed spectra must be {list(shape)}")
    g = plan.grid
    if tuple(cube.shape) != (C, g.ny, g.nx):
        raise ValueError(f"cube must be [{C}, {g.ny}, {g.nx}]")
    if weights is not None and tuple(weights.shape) != (g.ny, g.nx):
        raise ValueError(f"weights must be [{g.ny}, {g.nx}]")
    st = load().hcg_grid_packed(plan.handle, _dptr(packed, sdt, "packed"), C, int(dtype),
                                _dptr(chan_scale, torch.float32, "chan_scale"),
                                _dptr(cube, torch.float32, "cube"),
                                _dptr(weights, torch.float32, "weights"), _stream(stream))
    _check(st, "hcg_grid_packed")


def hcg_destroy(plan: Plan) -> None:
    plan.destroy()


def hcg_ang2pix(lon: torch.Tensor, lat: torch.Tensor, nside: int, stream=None) -> torch.Tensor:
    """Device HEALPix ring pixel (uint32 stored in an int32 tensor)."""
    n = int(lon.shape[0])
    pix = torch.empty(n, dtype=torch.int32, device=lon.device)
    st = load().hcg_ang2pix(_dptr(lon, torch.float64, "lon"), _dptr(lat, torch.float64, "lat"), n,
                            int(nside), ctypes.c_void_p(pix.data_ptr()), _stream(stream))
    _check(st, "hcg_ang2pix")
    return pix


def hcg_sort_keys(keys: torch.Tensor, key_bits: int, stream=None):
    """Stable radix sort of uint32 keys held in an int32 tensor -> (keys, perm)."""
    n = int(keys.shape[0])
    ko = torch.empty_like(keys)
    po = torch.empty_like(keys)
    st = load().hcg_sort_keys(_dptr(keys, torch.int32, "keys"), n, int(key_bits),
                              ctypes.c_void_p(ko.data_ptr()), ctypes.c_void_p(po.data_ptr()),
                              _stream(stream))
    _check(st, "hcg_sort_keys")
    return ko, po


class BorrowedPlan(Plan):
    """A batch's plan of one field (hcg_batch_get_plan): valid while the batch
    lives; destroying it is left to the batch."""

    def destroy(self) -> None:
        self.handle = None


class Batch:
    """Owns an hcg_batch_t (one plan per field)."""

    def __init__(self, handle: ctypes.c_void_p, grids, ns):
        self.handle = handle
        self.grids = grids
        self.ns = [int(n) for n in ns]

    def plan(self, field: int) -> BorrowedPlan:
        h = ctypes.c_void_p()
        _check(load().hcg_batch_get_plan(self.handle, int(field), ctypes.byref(h)),
               "hcg_batch_get_plan")
        return BorrowedPlan(h, self.grids[field], self.ns[field])

    def info(self) -> dict:
        out = BatchInfoC()
        _check(load().hcg_get_batch_info(self.handle, ctypes.byref(out)), "hcg_get_batch_info")
        d = {k: getattr(out, k) for k, _ in BatchInfoC._fields_}
        d["tune_ms"] = list(out.tune_ms)
        return d

    def destroy(self) -> None:
        if self.handle is not None:
            h, self.handle = self.handle, None
            _check(load().hcg_destroy_batch(h), "hcg_destroy_batch")

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def hcg_plan_batch(fields, chan_tile: int = 0, nside: int = 0, launch: str = "auto",
                   stream=None) -> Batch:
    """``fields``: sequence of (lon, lat, grid, fwhm_deg, support_deg), lon/lat
    device float64 tensors (read during the call only).  ``launch``: "auto"
    (autotuned), "persistent" or "items" (HCG_BATCH_PERSISTENT /
    HCG_BATCH_ITEMS)."""
    flags = {"auto": 0, "persistent": HCG_BATCH_PERSISTENT, "items": HCG_BATCH_ITEMS}[launch]
    arr = (FieldDescC * len(fields))()
    for i, (lon, lat, grid, fwhm, support) in enumerate(fields):
        if int(lat.shape[0]) != int(lon.shape[0]):
            raise ValueError(f"field {i}: lon and lat differ in length")
        arr[i] = FieldDescC(_dptr(lon, torch.float64, "lon"), _dptr(lat, torch.float64, "lat"),
                            int(lon.shape[0]), grid_desc(grid), float(fwhm), float(support))
    opts = OptsC(int(nside), 0, 0, 0, int(chan_tile), flags)
    handle = ctypes.c_void_p()
    _check(load().hcg_plan_batch(ctypes.byref(handle), len(fields), arr, ctypes.byref(opts),
                                 _stream(stream)), "hcg_plan_batch")
    return Batch(handle, [f[2] for f in fields], [int(f[0].shape[0]) for f in fields])


def hcg_grid_batch(batch: Batch, spectra, cubes, weights=None, dtypes=None, chan_scales=None,
                   stream=None) -> None:
    """Grids every field: ``spectra[i]`` ([n_i, C_i], or [2, n_i, C_i] for the
    split forms, in the storage of ``dtypes[i]``, FP32 by default) into
    ``cubes[i]`` [C_i, ny_i, nx_i] (and ``weights[i]`` [ny_i, nx_i] or None);
    ``chan_scales[i]`` for the scaled forms.  The tensors must stay alive
    until the work has run."""
    nf = len(batch.grids)
    if len(spectra) != nf or len(cubes) != nf:
        raise ValueError(f"need {nf} spectra and cubes")
    weights = weights if weights is not None else [None] * nf
    dtypes = dtypes if dtypes is not None else [HCG_F32] * nf
    chan_scales = chan_scales if chan_scales is not None else [None] * nf
    arr = (FieldDataC * nf)()
    for i in range(nf):
        g, sp, cb, dt = batch.grids[i], spectra[i], cubes[i], int(dtypes[i])
        sdt, prefix = _FORM_STORAGE[dt]
        if (sp.dim() != 2 + len(prefix) or tuple(sp.shape[:len(prefix)]) != prefix
                or int(sp.shape[-2]) != batch.ns[i]):
            raise ValueError(f"field {i}: spectra must be "
                             f"[{', '.join(map(str, prefix + (batch.ns[i], 'nchan')))}]")
        C = int(sp.shape[-1])
        if tuple(cb.shape) != (C, g.ny, g.nx):
            raise ValueError(f"field {i}: cube must be [{C}, {g.ny}, {g.nx}]")
        if weights[i] is not None and tuple(weights[i].shape) != (g.ny, g.nx):
            raise ValueError(f"field {i}: weights must be [{g.ny}, {g.nx}]")
        arr[i] = FieldDataC(_dptr(sp, sdt, "spectra"), C, dt,
                            _dptr(chan_scales[i], torch.float32, "chan_scale"),
                            _dptr(cb, torch.float32, "cube"),
                            _dptr(weights[i], torch.float32, "weights"))
    _check(load().hcg_grid_batch(batch.handle, arr, _stream(stream)), "hcg_grid_batch")


def u32(t: torch.Tensor):
    """int32 tensor holding uint32 values -> int64 numpy array."""
    return t.cpu().numpy().view("uint32").astype("int64")
