"""The gridding entry point that allocates nothing (hcg_grid_noalloc),
through the C ABI: on two calls in a row, the second with a smaller input,
its maps equal hcg_grid's bit for bit (the same kernels and the same split
of the candidate lists, with the partial sums in the library's static scratch
array instead of stream-ordered memory) and the FP64 oracle's within the FP32
tolerance of Eq. (1).  The first call's larger map leaves partial sums in the
scratch array; the second must not see them."""
import numpy as np
import pytest
import torch

import oracle
import paper_2012_13173_amd as hcg
import synth
from tests.gridcheck import assert_cube_close, assert_weights_close

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
TOL_F32 = 1e-5


def _bits(t):
    return t.contiguous().view(torch.int32).cpu().numpy()


def _both(w):
    """hcg_grid and hcg_grid_noalloc on one plan of ``w``; returns the maps of
    each (cube, W) as numpy arrays."""
    plan = hcg.hcg_plan(w.lon.to(DEV), w.lat.to(DEV), w.grid, w.fwhm_deg, w.support_deg,
                        nside=w.nside)
    spec = w.spectra.to(DEV).contiguous()
    shape = (w.nchan, w.grid.ny, w.grid.nx)
    cube_a = torch.empty(shape, dtype=torch.float32, device=DEV)
    W_a = torch.empty(shape[1:], dtype=torch.float32, device=DEV)
    # filled with a value no cell takes, so that a cell left unwritten shows
    cube_b = torch.full(shape, 12345.0, dtype=torch.float32, device=DEV)
    W_b = torch.full(shape[1:], -1.0, dtype=torch.float32, device=DEV)
    hcg.hcg_grid(plan, spec, cube_a, W_a)
    hcg.hcg_grid_noalloc(plan, spec, cube_b, W_b)
    torch.cuda.synchronize()
    info = plan.info()
    plan.destroy()
    assert np.array_equal(_bits(cube_a), _bits(cube_b)), "hcg_grid_noalloc differs from hcg_grid"
    assert np.array_equal(_bits(W_a), _bits(W_b)), "weight maps differ"
    return cube_b.cpu().numpy(), W_b.cpu().numpy(), info


def _against_oracle(w, V, W, what):
    Vr, Wr, _ = oracle.grid_allpairs(w.lon.numpy(), w.lat.numpy(), w.spectra.numpy(), w.grid,
                                     w.fwhm_deg, w.support_deg)
    assert_cube_close(V, Vr, TOL_F32, what)
    assert_weights_close(W, Wr)


def test_noalloc_equals_hcg_grid_on_two_calls_in_a_row():
    # first call: 120 x 120 cells of 0.5' = 225 tiles, so each tile's
    # candidates are split over 10 workgroups whose partial sums (5 channels
    # + W) go to the scratch array
    w1 = synth.small_cube(n=40_000, nchan=5, nx=120, ny=120, cell_arcmin=0.5, seed=951)
    print("call 1: 40,000 samples x 5 channels -> 120 x 120", flush=True)
    V1, W1, info1 = _both(w1)
    assert info1["ntiles_x"] * info1["ntiles_y"] == 225
    _against_oracle(w1, V1, W1, "noalloc call 1")
    # second call, smaller: 10,000 samples x 1 channel -> 60 x 60 (64 tiles,
    # split 32 ways): fewer partial-sum slots than the first call left behind
    w2 = synth.point_source_field()
    print("call 2: 10,000 samples x 1 channel -> 60 x 60", flush=True)
    V2, W2, info2 = _both(w2)
    assert info2["ntiles_x"] * info2["ntiles_y"] == 64
    _against_oracle(w2, V2, W2, "noalloc call 2")


def test_noalloc_many_channel_and_precision_forms():
    # the matrix-core forms use no scratch; the entry point runs them as
    # hcg_grid does (FP32, then an FP16 x channel-scale encoding)
    w = synth.small_cube(n=20_000, nchan=40, seed=953)
    print("matrix-core forms: 20,000 samples x 40 channels -> 45 x 37", flush=True)
    V, W, _ = _both(w)
    _against_oracle(w, V, W, "noalloc FP32 matrix-core form")
    plan = hcg.hcg_plan(w.lon.to(DEV), w.lat.to(DEV), w.grid, w.fwhm_deg, w.support_deg,
                        nside=w.nside)
    enc, scale = hcg.hcg_quantize(w.spectra.to(DEV).contiguous(), hcg.HCG_F16_SCALED)
    shape = (w.nchan, w.grid.ny, w.grid.nx)
    a = torch.empty(shape, dtype=torch.float32, device=DEV)
    b = torch.empty(shape, dtype=torch.float32, device=DEV)
    hcg.hcg_grid(plan, enc, a, dtype=hcg.HCG_F16_SCALED, chan_scale=scale)
    hcg.hcg_grid_noalloc(plan, enc, b, dtype=hcg.HCG_F16_SCALED, chan_scale=scale)
    torch.cuda.synchronize()
    plan.destroy()
    assert np.array_equal(_bits(a), _bits(b))


def test_noalloc_argument_errors():
    lib = hcg.load()
    import ctypes
    vp = ctypes.c_void_p
    assert lib.hcg_grid_noalloc(None, vp(1), 4, hcg.HCG_F32, None, vp(1), None, None) == hcg.HCG_E_ARG
    assert lib.hcg_grid_noalloc(vp(12345), vp(1), 4, hcg.HCG_F32, None, vp(1), None,
                                None) == hcg.HCG_E_STATE
    w = synth.point_source_field(n=2_000)
    plan = hcg.hcg_plan(w.lon.to(DEV), w.lat.to(DEV), w.grid, w.fwhm_deg, w.support_deg,
                        nside=w.nside)
    spec = w.spectra.to(DEV).contiguous()
    cube = torch.empty((1, w.grid.ny, w.grid.nx), dtype=torch.float32, device=DEV)
    assert lib.hcg_grid_noalloc(plan.handle, vp(spec.data_ptr()), 0, hcg.HCG_F32, None,
                                vp(cube.data_ptr()), None, None) == hcg.HCG_E_ARG
    assert lib.hcg_grid_noalloc(plan.handle, vp(spec.data_ptr()), 1, 99, None,
                                vp(cube.data_ptr()), None, None) == hcg.HCG_E_UNSUPPORTED
    assert b"hcg_grid_noalloc" in lib.hcg_last_error()
    with pytest.raises(ValueError):
        hcg.hcg_grid_noalloc(plan, spec[:-1], cube)
    plan.destroy()
