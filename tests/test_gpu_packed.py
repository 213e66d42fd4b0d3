"""GPU parity of the plan-ordered low-precision path (hcg_quantize_packed +
hcg_grid_packed) through the C ABI: the encoding is the input-order encoding
of hcg_quantize permuted into the plan's sorted order and grouped 8 samples
per channel (bit-exact), and the gridded cubes meet the same per-form
budgets against the FP64 oracle as the input-order forms.  Cases cover
sample counts that are not a multiple of 8, ragged channel tails, longitude
wrap, the polar cap, partial coverage and the argument checks."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2012_13173_amd as hcg
import synth
from tests.gridcheck import assert_cube_close, assert_weights_close, run_oracle

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")

# per-form budgets, as for the input-order forms
FORMS = {
    "f16_scaled": (hcg.HCG_F16_SCALED, 1e-3),
    "bf16_split": (hcg.HCG_BF16_SPLIT, 5e-5),
    "fp8e4m3_split": (hcg.HCG_FP8E4M3_SPLIT, 1e-2),
    "bf16": (hcg.HCG_BF16, 1e-2),
    "fp8e4m3_scaled": (hcg.HCG_FP8E4M3_SCALED, 1e-1),
}


def _plan(w):
    return hcg.hcg_plan(w.lon.to(DEV), w.lat.to(DEV), w.grid, w.fwhm_deg, w.support_deg,
                        nside=w.nside)


def _grid_packed(w, plan, form):
    spec = w.spectra.to(DEV).contiguous()
    packed, scale = hcg.hcg_quantize_packed(plan, spec, form)
    cube = torch.empty((w.nchan, w.grid.ny, w.grid.nx), dtype=torch.float32, device=DEV)
    W = torch.empty((w.grid.ny, w.grid.nx), dtype=torch.float32, device=DEV)
    hcg.hcg_grid_packed(plan, packed, cube, W, dtype=form, chan_scale=scale)
    torch.cuda.synchronize()
    return cube.cpu().numpy(), W.cpu().numpy()


@pytest.mark.parametrize("n,nchan", [(12_001, 67), (12_007, 300), (12_000, 16), (9_999, 1024),
                                    (8_003, 1)])
def test_packed_encoding_is_the_sorted_grouped_encoding(n, nchan):
    w = synth.small_cube(n=n, nchan=nchan, nx=21, ny=17)
    plan = _plan(w)
    perm = hcg.u32(plan.export(hcg.HCG_ARR_PERM)).astype(np.int64)
    spec = w.spectra.to(DEV).contiguous()
    groups = (n + 7) // 8
    for name, (form, _) in FORMS.items():
        enc, scale = hcg.hcg_quantize(spec, form)
        packed, pscale = hcg.hcg_quantize_packed(plan, spec, form)
        if scale is not None:
            assert torch.equal(pscale, scale), name
        planes = enc if enc.dim() == 3 else enc.unsqueeze(0)
        idx = torch.from_numpy(perm).to(DEV)
        cp = (nchan + 15) // 16 * 16
        want = torch.zeros((planes.shape[0], groups * 8, cp), dtype=enc.dtype, device=DEV)
        want[:, :n, :nchan] = planes.index_select(1, idx)
        want = want.view(planes.shape[0], groups, 8, cp).transpose(2, 3).contiguous()
        assert tuple(packed.shape) == tuple(want.shape), name
        assert torch.equal(packed.view(torch.uint8), want.view(torch.uint8)), name
    plan.destroy()


@pytest.mark.parametrize("n,nchan", [(15_001, 300), (15_003, 67), (14_999, 1024), (15_000, 20),
                                    (15_005, 3), (15_002, 1)])
def test_packed_forms_against_oracle(n, nchan):
    w = synth.small_cube(n=n, nchan=nchan, nx=29, ny=19)
    Vr, Wr, _ = run_oracle(w)
    plan = _plan(w)
    for name, (form, tol) in FORMS.items():
        V, W = _grid_packed(w, plan, form)
        e = assert_cube_close(V, Vr, tol, f"packed {name} C={nchan}")
        print(f"packed {name:>15s} C={nchan:5d}: max {e.max():.2e} median {np.median(e):.2e}")
        assert_weights_close(W, Wr)
    plan.destroy()


def test_packed_equals_input_order_up_to_rounding_order():
    w = synth.small_cube(n=15_005, nchan=192, nx=29, ny=19)
    plan = _plan(w)
    spec = w.spectra.to(DEV).contiguous()
    for name, (form, _) in FORMS.items():
        V1, W1 = _grid_packed(w, plan, form)
        enc, scale = hcg.hcg_quantize(spec, form)
        cube = torch.empty_like(torch.from_numpy(V1), device=DEV)
        W = torch.empty((w.grid.ny, w.grid.nx), dtype=torch.float32, device=DEV)
        hcg.hcg_grid(plan, enc, cube, W, dtype=form, chan_scale=scale)
        V2 = cube.cpu().numpy()
        assert np.array_equal(np.isnan(V1), np.isnan(V2)), name
        ok = ~np.isnan(V2)
        # the same rounded products, summed in another order in FP32
        np.testing.assert_allclose(V1[ok], V2[ok], rtol=2e-5, atol=2e-5 * np.abs(V2[ok]).max(),
                                   err_msg=name)
        np.testing.assert_allclose(W1, W.cpu().numpy(), rtol=1e-6)
    plan.destroy()


@pytest.mark.parametrize("kw", [
    dict(lon_c=0.05, nx=40, ny=21, name="ra_wrap"),
    dict(lat_c=75.0, lon_c=300.0, nx=24, ny=24, name="polar_cap"),
    dict(nx=50, ny=44, pad_arcmin=-6.0, name="partial_coverage"),
    dict(fwhm_arcmin=300.0, cell_arcmin=60.0, nx=20, ny=20, pad_arcmin=400.0,
         name="wide_support"),
])
def test_packed_geometry_cases(kw):
    w = synth.small_cube(n=20_003, nchan=40, **kw)
    Vr, Wr, _ = run_oracle(w)
    plan = _plan(w)
    for form, tol in ((hcg.HCG_F16_SCALED, 1e-3), (hcg.HCG_FP8E4M3_SPLIT, 1e-2)):
        V, W = _grid_packed(w, plan, form)
        assert_cube_close(V, Vr, tol, kw["name"])
        assert_weights_close(W, Wr)
    plan.destroy()


def test_packed_constant_input_is_exact():
    w = synth.small_cube(n=12_005, nchan=64, nx=21, ny=13)
    w.spectra[:] = 2.5
    plan = _plan(w)
    for name, (form, _) in FORMS.items():
        V, W = _grid_packed(w, plan, form)
        assert (W > 0).all()
        np.testing.assert_allclose(V, 2.5, rtol=1e-5, err_msg=name)
    plan.destroy()


def test_packed_argument_errors():
    w = synth.small_cube(n=2001, nchan=16, nx=8, ny=8)
    plan = _plan(w)
    spec = w.spectra.to(DEV).contiguous()
    lib = hcg.load()
    cube = torch.empty((16, 8, 8), dtype=torch.float32, device=DEV)
    packed, scale = hcg.hcg_quantize_packed(plan, spec, hcg.HCG_F16_SCALED)
    vp = ctypes.c_void_p
    stream = vp(torch.cuda.current_stream().cuda_stream)
    # FP32 has no plan-ordered form
    st = lib.hcg_grid_packed(plan.handle, vp(packed.data_ptr()), 16, hcg.HCG_F32, None,
                             vp(cube.data_ptr()), None, stream)
    assert st == hcg.HCG_E_ARG
    # scale missing / given wrongly
    st = lib.hcg_grid_packed(plan.handle, vp(packed.data_ptr()), 16, hcg.HCG_F16_SCALED, None,
                             vp(cube.data_ptr()), None, stream)
    assert st == hcg.HCG_E_ARG
    st = lib.hcg_grid_packed(plan.handle, vp(packed.data_ptr()), 16, hcg.HCG_BF16,
                             vp(scale.data_ptr()), vp(cube.data_ptr()), None, stream)
    assert st == hcg.HCG_E_ARG
    # a misaligned buffer is refused before any launch
    st = lib.hcg_grid_packed(plan.handle, vp(packed.data_ptr() + 2), 16, hcg.HCG_F16_SCALED,
                             vp(scale.data_ptr()), vp(cube.data_ptr()), None, stream)
    assert st == hcg.HCG_E_ARG
    out = torch.empty(packed.numel() * 2 + 64, dtype=torch.uint8, device=DEV)
    st = lib.hcg_quantize_packed(plan.handle, vp(spec.data_ptr()), 16, hcg.HCG_F16_SCALED,
                                 vp(out.data_ptr() + 4), vp(scale.data_ptr()), stream)
    assert st == hcg.HCG_E_ARG
    with pytest.raises(ValueError):
        hcg.hcg_quantize_packed(plan, spec[:-1].contiguous(), hcg.HCG_F16_SCALED)
    with pytest.raises(ValueError):
        hcg.hcg_grid_packed(plan, packed[:, :-1].contiguous(), cube, dtype=hcg.HCG_F16_SCALED,
                            chan_scale=scale)
    nbytes = ctypes.c_int64()
    assert lib.hcg_packed_bytes(plan.handle, 16, hcg.HCG_F32, ctypes.byref(nbytes)) == hcg.HCG_E_ARG
    assert lib.hcg_packed_bytes(plan.handle, 16, hcg.HCG_FP8E4M3_SPLIT,
                                ctypes.byref(nbytes)) == hcg.HCG_OK
    assert nbytes.value == 2 * ((2001 + 7) // 8) * 8 * 16
    assert lib.hcg_packed_bytes(plan.handle, 17, hcg.HCG_BF16, ctypes.byref(nbytes)) == hcg.HCG_OK
    assert nbytes.value == 2 * ((2001 + 7) // 8) * 8 * 32
    torch.cuda.synchronize()
    plan.destroy()


@pytest.mark.parametrize("n", [1, 5, 9, 64])
def test_packed_tiny_sample_counts(n):
    w = synth.small_cube(n=n, nchan=24, nx=12, ny=10, cell_arcmin=1.0, pad_arcmin=-1.0,
                         seed=400 + n)
    Vr, Wr, _ = run_oracle(w)
    plan = _plan(w)
    for name, (form, tol) in FORMS.items():
        V, W = _grid_packed(w, plan, form)
        assert_cube_close(V, Vr, tol, f"packed {name} n={n}")
        assert_weights_close(W, Wr)
    plan.destroy()
