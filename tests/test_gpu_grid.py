"""GPU parity of hcg_grid (Eq. (1)) against the FP64 oracle, through the C ABI.

The FP32 form must agree with the oracle to 1e-5 per channel in relative L2
norm over cells with W > 0 (NaN patterns equal), and the W map to 1e-6 per
cell.  Cases span several tiles, ragged tile and channel tails, both
accumulation kernels (one lane per cell for C <= 8, the matrix-core
contraction for more), longitude wrap, the polar-cap boundary and empty
cells."""
import numpy as np
import pytest
import torch

import oracle
import paper_2012_13173_amd as hcg
import synth
from synth import GridDesc
from tests.gridcheck import assert_cube_close, assert_weights_close, run_gpu, run_oracle

pytestmark = pytest.mark.gpu
TOL_F32 = 1e-5


def test_point_source_field_parity():
    w = synth.point_source_field()
    V, W = run_gpu(w)
    Vr, Wr, _ = run_oracle(w)
    assert_cube_close(V, Vr, TOL_F32, "point sources")
    assert_weights_close(W, Wr)


@pytest.mark.parametrize("nchan", [1, 2, 3, 8, 9, 64, 67, 256, 300, 513])
def test_channel_counts(nchan):
    w = synth.small_cube(n=12_000, nchan=nchan, nx=29, ny=19)
    V, W = run_gpu(w)
    Vr, Wr, _ = run_oracle(w)
    assert_cube_close(V, Vr, TOL_F32, f"C={nchan}")
    assert_weights_close(W, Wr)


@pytest.mark.parametrize("kw", [
    dict(lon_c=0.05, nx=40, ny=21, name="ra_wrap"),
    dict(lon_c=359.9, nx=33, ny=17, name="ra_wrap_high"),
    dict(lat_c=41.8, nx=30, ny=50, cell_arcmin=1.0, name="cap_boundary"),
    dict(lat_c=75.0, lon_c=300.0, nx=24, ny=24, name="polar_cap"),
    dict(lat_c=-60.0, nx=24, ny=9, name="south"),
    # support 6.4 deg: the distances beyond the chord series (arcsine branch)
    dict(fwhm_arcmin=300.0, cell_arcmin=60.0, nx=20, ny=20, pad_arcmin=400.0,
         name="wide_support"),
])
def test_geometry_cases(kw):
    w = synth.small_cube(n=20_000, nchan=20, **kw)
    V, W = run_gpu(w)
    Vr, Wr, _ = run_oracle(w)
    assert_cube_close(V, Vr, TOL_F32, kw["name"])
    assert_weights_close(W, Wr)


def test_empty_cells_and_partial_coverage():
    # the grid sticks out of the sampled area: outer cells have W = 0, V = NaN
    w = synth.small_cube(n=8000, nchan=70, nx=50, ny=44, pad_arcmin=-6.0)
    V, W = run_gpu(w)
    Vr, Wr, _ = run_oracle(w)
    assert (Wr == 0).sum() > 100
    assert_cube_close(V, Vr, TOL_F32, "partial coverage")
    assert_weights_close(W, Wr)


def test_constant_input_gives_constant_map():
    w = synth.small_cube(n=15_000, nchan=96, nx=31, ny=23)
    w.spectra[:] = 2.5
    V, W = run_gpu(w)
    ok = W > 0
    assert ok.all()
    np.testing.assert_allclose(V[:, ok], 2.5, rtol=1e-5)


def test_input_order_does_not_matter():
    w = synth.small_cube(n=15_000, nchan=80, nx=31, ny=23)
    V1, W1 = run_gpu(w)
    p = torch.randperm(w.n, generator=torch.Generator().manual_seed(9))
    w2 = synth.Workload(w.name, w.lon[p], w.lat[p], w.spectra[p], w.grid, w.fwhm_deg,
                        w.support_deg, w.nside)
    V2, W2 = run_gpu(w2)
    np.testing.assert_allclose(V2, V1, rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(W2, W1, rtol=1e-6)


def test_nside_does_not_change_the_map():
    w = synth.small_cube(n=10_000, nchan=33, nx=20, ny=20)
    Va, Wa = run_gpu(w, nside=1024)
    Vb, Wb = run_gpu(w, nside=16384)
    Vr, Wr, _ = run_oracle(w)
    assert_cube_close(Va, Vr, TOL_F32, "nside 1024")
    assert_cube_close(Vb, Vr, TOL_F32, "nside 16384")
    assert_weights_close(Wa, Wr)


def test_plan_reuse_and_stream():
    w = synth.small_cube(n=10_000, nchan=40, nx=20, ny=20)
    dev = torch.device("cuda:0")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan = hcg.hcg_plan(w.lon.to(dev), w.lat.to(dev), w.grid, w.fwhm_deg, w.support_deg,
                            stream=s)
        Vr, Wr, _ = run_oracle(w)
        for sl in (slice(0, 40), slice(5, 17), slice(39, 40)):
            spec = w.spectra[:, sl].contiguous().to(dev)
            cube = torch.empty((spec.shape[1], 20, 20), dtype=torch.float32, device=dev)
            hcg.hcg_grid(plan, spec, cube, None, stream=s)
            s.synchronize()
            assert_cube_close(cube.cpu().numpy(), Vr[sl], TOL_F32, f"slab {sl}")
    plan.destroy()


def test_repeated_plans_reuse_memory_and_agree():
    # plans and their scratch come from the library's pool: forty plan +
    # grid + destroy cycles (the second half on another stream, the
    # few-channel gather's partial sums included) leave the device's free
    # memory where the first cycle left it, up to the pool's retained bytes,
    # and every cycle gives the same map bit for bit
    dev = torch.device("cuda:0")
    w = synth.small_cube(n=400_000, nchan=3, nx=60, ny=50, seed=77)
    lon, lat, spec = w.lon.to(dev), w.lat.to(dev), w.spectra.to(dev).contiguous()
    s2 = torch.cuda.Stream()
    first, free_after_first = None, None
    for i in range(40):
        st = None if i < 20 else s2
        with torch.cuda.stream(st if st is not None else torch.cuda.current_stream()):
            plan = hcg.hcg_plan(lon, lat, w.grid, w.fwhm_deg, w.support_deg, nside=w.nside,
                                stream=st)
            cube = torch.empty((3, 50, 60), dtype=torch.float32, device=dev)
            hcg.hcg_grid(plan, spec, cube, None, stream=st)
            torch.cuda.synchronize()
            plan.destroy()
        if first is None:
            first = cube.cpu().numpy()
            free_after_first = torch.cuda.mem_get_info()[0]
        else:
            assert np.array_equal(cube.cpu().numpy(), first, equal_nan=True), i
        del cube
    torch.cuda.synchronize()
    drop = free_after_first - torch.cuda.mem_get_info()[0]
    print(f"free device memory after 40 cycles: {drop / 2**20:.1f} MiB less than after the first",
          flush=True)
    assert drop <= (2 << 30) + (64 << 20)


def test_grid_argument_errors():
    w = synth.small_cube(n=2000, nchan=4, nx=8, ny=8)
    dev = torch.device("cuda:0")
    plan = hcg.hcg_plan(w.lon.to(dev), w.lat.to(dev), w.grid, w.fwhm_deg, w.support_deg)
    spec = w.spectra.to(dev)
    cube = torch.empty((4, 8, 8), dtype=torch.float32, device=dev)
    lib = hcg.load()
    import ctypes
    vp = ctypes.c_void_p
    assert lib.hcg_grid(plan.handle, None, 4, 0, None, vp(cube.data_ptr()), None, None) == hcg.HCG_E_ARG
    assert lib.hcg_grid(plan.handle, vp(spec.data_ptr()), 0, 0, None, vp(cube.data_ptr()), None, None) == hcg.HCG_E_ARG
    assert lib.hcg_grid(plan.handle, vp(spec.data_ptr()), 4, 7, None, vp(cube.data_ptr()), None, None) == hcg.HCG_E_UNSUPPORTED
    # chan_scale is required by the scaled forms and refused by the others
    assert lib.hcg_grid(plan.handle, vp(spec.data_ptr()), 4, hcg.HCG_F16_SCALED, None, vp(cube.data_ptr()), None, None) == hcg.HCG_E_ARG
    assert lib.hcg_grid(plan.handle, vp(spec.data_ptr()), 4, hcg.HCG_F32, vp(spec.data_ptr()), vp(cube.data_ptr()), None, None) == hcg.HCG_E_ARG
    plan.destroy()
    assert lib.hcg_grid(plan.handle, vp(spec.data_ptr()), 4, 0, None, vp(cube.data_ptr()), None, None) in (hcg.HCG_E_ARG, hcg.HCG_E_STATE)


@pytest.mark.parametrize("n", [1, 5, 9, 64])
@pytest.mark.parametrize("nchan", [1, 40])
def test_tiny_sample_counts(n, nchan):
    # a handful of samples: most cells are empty, the candidate lists are
    # shorter than one staged block (and than one group of 8 sorted samples)
    w = synth.small_cube(n=n, nchan=nchan, nx=12, ny=10, cell_arcmin=1.0, pad_arcmin=-1.0,
                         seed=300 + n)
    V, W = run_gpu(w)
    Vr, Wr, _ = run_oracle(w)
    assert_cube_close(V, Vr, TOL_F32, f"n={n} C={nchan}")
    assert_weights_close(W, Wr)
