"""GPU parity of hcg_grid_host: spectra and cube in host memory, gridded in
channel slabs streamed through the device (the copy/compute overlap on
streams that Section 5 names as future work).

Each streamed slab must equal, bit for bit, hcg_grid run on the device over
the same channels (the same kernels on the same inputs), and the whole cube
must agree with the FP64 oracle to the FP32 bound of 1e-5.  Cases: ragged last
slab, one-channel slabs, a slab wider than the cube, pageable and page-locked
host memory, W omitted, and a full-size sample count with sampled cells.

The low-precision storage forms stream the same way (one or two planes of
16- or 8-bit elements, per-channel scales in host memory): each slab equals
hcg_grid on the device over the same encoded channels and scales, and the cube
meets the form's error budget against the oracle on the FP32 master spectra
(the budgets of the precision tests: FP16 x scale 1e-3, BF16 hi+lo 5e-5, FP8
hi+lo 1e-2, plain BF16 1e-2, FP8 x scale 1e-1)."""
import numpy as np
import pytest
import torch

import paper_2012_13173_amd as hcg
import synth
from tests.gridcheck import (assert_cube_close, assert_weights_close, gather_cells, run_oracle,
                             sample_cells, sampled_oracle)

pytestmark = pytest.mark.gpu
TOL_F32 = 1e-5
DEV = torch.device("cuda:0")
LP_FORMS = [(hcg.HCG_BF16, 1e-2), (hcg.HCG_BF16_SPLIT, 5e-5), (hcg.HCG_F16_SCALED, 1e-3),
            (hcg.HCG_FP8E4M3_SCALED, 1e-1), (hcg.HCG_FP8E4M3_SPLIT, 1e-2)]


def _plan(w):
    dev = torch.device("cuda:0")
    return hcg.hcg_plan(w.lon.to(dev), w.lat.to(dev), w.grid, w.fwhm_deg, w.support_deg,
                        nside=w.nside)


def _host(shape, pinned):
    t = torch.empty(shape, dtype=torch.float32, pin_memory=pinned)
    t.fill_(-7.0)  # every element must be overwritten
    return t


def _device_slabs(plan, w, slab):
    """hcg_grid on the device, one call per slab of channels."""
    dev = torch.device("cuda:0")
    C, g = w.nchan, w.grid
    cs = slab if slab else C
    V = np.empty((C, g.ny, g.nx), dtype=np.float32)
    W = torch.empty((g.ny, g.nx), dtype=torch.float32, device=dev)
    for c0 in range(0, C, cs):
        cn = min(cs, C - c0)
        spec = w.spectra[:, c0:c0 + cn].contiguous().to(dev)
        cube = torch.empty((cn, g.ny, g.nx), dtype=torch.float32, device=dev)
        hcg.hcg_grid(plan, spec, cube, W if c0 == 0 else None)
        V[c0:c0 + cn] = cube.cpu().numpy()
    torch.cuda.synchronize()
    return V, W.cpu().numpy()


def _encoded(w, form, pinned):
    """The form's encoding of the spectra (hcg_quantize on the device), on the
    device and as a host copy, with its scales."""
    enc, scale = hcg.hcg_quantize(w.spectra.to(DEV).contiguous(), form)
    torch.cuda.synchronize()
    enc_h = enc.cpu()
    if pinned:
        enc_h = enc_h.pin_memory()
    return enc, scale, enc_h, (scale.cpu() if scale is not None else None)


def _device_slabs_form(plan, w, enc, scale, form, slab):
    """hcg_grid on the device over each slab of encoded channels."""
    C, g = w.nchan, w.grid
    cs = slab if slab else C
    V = np.empty((C, g.ny, g.nx), dtype=np.float32)
    W = torch.empty((g.ny, g.nx), dtype=torch.float32, device=DEV)
    for c0 in range(0, C, cs):
        cn = min(cs, C - c0)
        spec = enc[..., c0:c0 + cn].contiguous()
        sc = scale[c0:c0 + cn].contiguous() if scale is not None else None
        cube = torch.empty((cn, g.ny, g.nx), dtype=torch.float32, device=DEV)
        hcg.hcg_grid(plan, spec, cube, W if c0 == 0 else None, dtype=form, chan_scale=sc)
        V[c0:c0 + cn] = cube.cpu().numpy()
    torch.cuda.synchronize()
    return V, W.cpu().numpy()


def _streamed(plan, w, slab, pinned=True, with_weights=True, pinned_out=None):
    g = w.grid
    pinned_out = pinned if pinned_out is None else pinned_out
    spec = w.spectra.contiguous()
    if pinned:
        spec = spec.pin_memory()
    cube = _host((w.nchan, g.ny, g.nx), pinned_out)
    W = _host((g.ny, g.nx), pinned_out) if with_weights else None
    hcg.hcg_grid_host(plan, spec, cube, W, slab=slab)
    return cube.numpy(), (W.numpy() if with_weights else None)


@pytest.mark.parametrize("nchan,slab,pinned,pinned_out", [
    (300, 64, True, True),     # 4 full slabs and a ragged one of 44 channels
    (300, 64, False, False),   # the same through the library's page-locked chunks
    (300, 64, True, False),    # page-locked spectra, pageable cube
    (300, 64, False, True),    # pageable spectra, page-locked cube
    (37, 1, True, True),       # one channel per slab (the one-lane-per-cell kernel)
    (70, 9, True, True),       # slabs that switch between the two accumulation kernels
    (70, 9, False, False),
    (20, 0, True, True),       # default slab, wider than the cube
    (20, 0, False, False),     # one slab of whole rows: contiguous packing
    (600, 300, True, True),    # slabs above 256 channels
])
def test_streamed_equals_device_slabs(nchan, slab, pinned, pinned_out):
    w = synth.small_cube(n=12_000, nchan=nchan, nx=29, ny=19)
    plan = _plan(w)
    V, W = _streamed(plan, w, slab, pinned, pinned_out=pinned_out)
    Vd, Wd = _device_slabs(plan, w, slab if slab else 512)
    plan.destroy()
    assert np.array_equal(V, Vd, equal_nan=True), "streamed cube differs from hcg_grid"
    assert np.array_equal(W, Wd)
    Vr, Wr, _ = run_oracle(w)
    assert_cube_close(V, Vr, TOL_F32, f"C={nchan} slab={slab}")
    assert_weights_close(W, Wr)


@pytest.mark.parametrize("form,tol", LP_FORMS)
@pytest.mark.parametrize("pinned,slab", [(True, 32), (False, 32), (False, 0)])
def test_streamed_forms_equal_device_slabs(form, tol, pinned, slab):
    # 70 channels in slabs of 32: two full slabs and a ragged one of 6 (rows
    # read one element at a time); slab 0: one slab of whole rows
    w = synth.small_cube(n=12_000, nchan=70, nx=29, ny=19)
    plan = _plan(w)
    g = w.grid
    enc, scale, enc_h, scale_h = _encoded(w, form, pinned)
    cube = _host((w.nchan, g.ny, g.nx), pinned)
    W = _host((g.ny, g.nx), pinned)
    hcg.hcg_grid_host(plan, enc_h, cube, W, slab=slab, dtype=form, chan_scale=scale_h)
    Vd, Wd = _device_slabs_form(plan, w, enc, scale, form, slab if slab else 512)
    plan.destroy()
    V = cube.numpy()
    assert np.array_equal(V, Vd, equal_nan=True), f"form {form}: streamed cube differs from hcg_grid"
    assert np.array_equal(W.numpy(), Wd)
    Vr, Wr, _ = run_oracle(w)
    assert_cube_close(V, Vr, tol, f"form {form} slab={slab} pinned={pinned}")
    assert_weights_close(W.numpy(), Wr)


def test_streamed_without_weights_and_repeated():
    w = synth.small_cube(n=9000, nchan=50, nx=23, ny=31, lat_c=-60.0)
    plan = _plan(w)
    V1, _ = _streamed(plan, w, 16, with_weights=False)
    V2, W2 = _streamed(plan, w, 7)
    plan.destroy()
    Vr, Wr, _ = run_oracle(w)
    assert_cube_close(V1, Vr, TOL_F32, "no W")
    assert_cube_close(V2, Vr, TOL_F32, "slab 7")
    assert_weights_close(W2, Wr)


def test_streamed_after_work_on_the_stream():
    # work queued earlier on the caller's stream (the plan build) comes first
    w = synth.small_cube(n=10_000, nchan=33, nx=20, ny=20)
    s = torch.cuda.Stream()
    dev = torch.device("cuda:0")
    with torch.cuda.stream(s):
        plan = hcg.hcg_plan(w.lon.to(dev), w.lat.to(dev), w.grid, w.fwhm_deg, w.support_deg,
                            nside=w.nside, stream=s)
        cube = _host((w.nchan, w.grid.ny, w.grid.nx), True)
        hcg.hcg_grid_host(plan, w.spectra.pin_memory(), cube, None, slab=8, stream=s)
    plan.destroy()
    Vr, _, _ = run_oracle(w)
    assert_cube_close(cube.numpy(), Vr, TOL_F32, "plan on a side stream")


def test_argument_errors():
    w = synth.small_cube(n=2000, nchan=4, nx=8, ny=8)
    plan = _plan(w)
    g = w.grid
    cube = torch.empty((4, g.ny, g.nx), dtype=torch.float32)
    with pytest.raises(TypeError):
        hcg.hcg_grid_host(plan, w.spectra.cuda(), cube)
    with pytest.raises(ValueError):
        hcg.hcg_grid_host(plan, w.spectra[:100].contiguous(), cube)
    with pytest.raises(ValueError):
        hcg.hcg_grid_host(plan, w.spectra, cube[:3].contiguous())
    with pytest.raises(hcg.HcgError):
        hcg.hcg_grid_host(plan, w.spectra, cube, slab=-1)
    enc, scale, enc_h, scale_h = _encoded(w, hcg.HCG_F16_SCALED, False)
    with pytest.raises(hcg.HcgError, match="chan_scale is required"):
        hcg.hcg_grid_host(plan, enc_h, cube, dtype=hcg.HCG_F16_SCALED)
    with pytest.raises(hcg.HcgError, match="chan_scale must be NULL"):
        hcg.hcg_grid_host(plan, w.spectra, cube, chan_scale=scale_h)
    with pytest.raises(TypeError):  # scales in device memory
        hcg.hcg_grid_host(plan, enc_h, cube, dtype=hcg.HCG_F16_SCALED, chan_scale=scale)
    with pytest.raises(TypeError):  # FP32 spectra given for a 16-bit form
        hcg.hcg_grid_host(plan, w.spectra, cube, dtype=hcg.HCG_F16_SCALED, chan_scale=scale_h)
    with pytest.raises(ValueError):  # one plane given for a split form
        hcg.hcg_grid_host(plan, enc_h, cube, dtype=hcg.HCG_BF16_SPLIT)
    plan.destroy()


def test_device_pointer_refused():
    # the C ABI itself rejects device memory given as host memory
    import ctypes
    w = synth.small_cube(n=2000, nchan=4, nx=8, ny=8)
    plan = _plan(w)
    spec_d = w.spectra.cuda()
    cube = torch.empty((4, 8, 8), dtype=torch.float32)
    lib = hcg.load()
    st = lib.hcg_grid_host(plan.handle, ctypes.c_void_p(spec_d.data_ptr()), 4, hcg.HCG_F32,
                           None, 0, ctypes.c_void_p(cube.data_ptr()), None, None)
    assert st == hcg.HCG_E_ARG and b"device pointer" in lib.hcg_last_error()
    # the scales of a scaled form, given in device memory
    enc_h = torch.zeros((2000, 4), dtype=torch.float16)
    scale_d = torch.ones(4, dtype=torch.float32, device=DEV)
    st = lib.hcg_grid_host(plan.handle, ctypes.c_void_p(enc_h.data_ptr()), 4,
                           hcg.HCG_F16_SCALED, ctypes.c_void_p(scale_d.data_ptr()), 0,
                           ctypes.c_void_p(cube.data_ptr()), None, None)
    assert st == hcg.HCG_E_ARG and b"device pointer" in lib.hcg_last_error()
    # an unknown form
    st = lib.hcg_grid_host(plan.handle, ctypes.c_void_p(enc_h.data_ptr()), 4, 99, None, 0,
                           ctypes.c_void_p(cube.data_ptr()), None, None)
    assert st == hcg.HCG_E_UNSUPPORTED
    plan.destroy()


def test_full_size_sample_count_sampled():
    """The 9.12M-sample drift scan (64 channels) streamed from page-locked
    memory in slabs of 16, and from pageable memory in slabs of 48 (27 packed
    chunks in per slab, two chunks out): slabs equal to hcg_grid on the
    device, sampled cells against the oracle."""
    dev = torch.device("cuda:0")
    w = synth.drift_scan_cube(40, 12_000, 64, 600, 0.5, 3.0, synth.SEED0 + 1, device=dev,
                              name="drift_scan_600x600_c64")
    print(f"{w.name}: {w.n} samples x {w.nchan} channels", flush=True)
    plan = _plan(w)
    g = w.grid
    spec = w.spectra.cpu().pin_memory()
    cube = _host((w.nchan, g.ny, g.nx), True)
    W = _host((g.ny, g.nx), True)
    hcg.hcg_grid_host(plan, spec, cube, W, slab=16)
    del spec
    Vd, Wd = _device_slabs(plan, w, 16)
    assert np.array_equal(cube.numpy(), Vd, equal_nan=True)
    assert np.array_equal(W.numpy(), Wd)
    spec = w.spectra.cpu()
    cube_p = _host((w.nchan, g.ny, g.nx), False)
    W_p = _host((g.ny, g.nx), False)
    hcg.hcg_grid_host(plan, spec, cube_p, W_p, slab=48)
    del spec
    Vd, _ = _device_slabs(plan, w, 48)
    plan.destroy()
    assert np.array_equal(cube_p.numpy(), Vd, equal_nan=True)
    assert np.array_equal(W_p.numpy(), Wd)
    del cube_p, W_p
    groups = sample_cells(g, seed=3, patches=3, patch=8)
    cells = np.concatenate(groups)
    ref = [sampled_oracle(w, c) for c in groups]
    Vr = np.concatenate([v for v, _ in ref])
    Wr = np.concatenate([x for _, x in ref])
    Vg, Wg = gather_cells(cube, W, cells)
    assert_cube_close(Vg.T, Vr.T, TOL_F32, "drift scan, sampled")
    assert_weights_close(Wg, Wr)


def test_full_size_sample_count_forms_sampled():
    """The 9.12M-sample drift scan (64 channels) streamed in two stored
    forms: FP16 x scale from page-locked memory in slabs of 16, BF16 hi+lo
    (two planes) from pageable memory in slabs of 48 (each plane packed
    through the library's chunks).  Slabs equal hcg_grid on the device;
    sampled cells meet the form's budget against the oracle."""
    w = synth.drift_scan_cube(40, 12_000, 64, 600, 0.5, 3.0, synth.SEED0 + 1, device=DEV,
                              name="drift_scan_600x600_c64")
    print(f"{w.name}: {w.n} samples x {w.nchan} channels", flush=True)
    plan = _plan(w)
    g = w.grid
    groups = sample_cells(g, seed=5, patches=3, patch=8)
    cells = np.concatenate(groups)
    ref = [sampled_oracle(w, c) for c in groups]
    Vr = np.concatenate([v for v, _ in ref])
    Wr = np.concatenate([x for _, x in ref])
    for form, tol, pinned, slab in [(hcg.HCG_F16_SCALED, 1e-3, True, 16),
                                    (hcg.HCG_BF16_SPLIT, 5e-5, False, 48)]:
        print(f"form {form}, pinned {pinned}, slab {slab}", flush=True)
        enc, scale, enc_h, scale_h = _encoded(w, form, pinned)
        cube = _host((w.nchan, g.ny, g.nx), pinned)
        W = _host((g.ny, g.nx), pinned)
        hcg.hcg_grid_host(plan, enc_h, cube, W, slab=slab, dtype=form, chan_scale=scale_h)
        del enc_h
        Vd, Wd = _device_slabs_form(plan, w, enc, scale, form, slab)
        del enc
        assert np.array_equal(cube.numpy(), Vd, equal_nan=True), f"form {form}"
        assert np.array_equal(W.numpy(), Wd)
        del Vd
        Vg, Wg = gather_cells(cube, W, cells)
        assert_cube_close(Vg.T, Vr.T, tol, f"drift scan, form {form}, sampled")
        assert_weights_close(Wg, Wr)
    plan.destroy()
