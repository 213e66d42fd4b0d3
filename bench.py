"""Throughput benchmark of the gridding hot path on one MI355X.

Workload: the 19-beam drift-scan map -- 40 strips x 19 beams x 12,000 samples
(9,120,000 samples) x 1,024 float32 channels gridded onto 600 x 600 cells of
0.5' with a Gaussian kernel of FWHM 3', support 3 sigma, HEALPix nside 8192.
Inputs are synthesised on the GPU (seeded) and resident in HBM before timing.

One step = hcg_plan (ang2pix, radix sort, trig, ring table, tile ranges) +
hcg_grid (weights + channel accumulation + normalisation) + hcg_destroy.
The metric is sample*channel updates per second, N * C / t_step.

Printed: one JSON line with the metric, a roofline record of the dominant
kernel (the gather, timed with HIP events on its stream) and the FP64 CPU
oracle timed on a bounded sample of the same workload.  The same line carries
the low-precision forms on this workload and, under "c2", the many-channel
drift scan (1,976,000 samples x 8,192 channels -> 400 x 400) on which the
metric's "FP32 gather vs BF16-MFMA at <= 1e-3" is stated: the FP32 gather,
FP16 x channel scale and BF16 hi+lo, each with its per-channel error against
the oracle, whether it meets its budget, and its encoding time.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import paper_2012_13173_amd as hcg  # noqa: E402
import synth  # noqa: E402

MFMA_FP32_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0
# error budgets per form (largest per-channel relative L2 against the oracle):
# FP32 1e-5; the 16-bit matrix-core forms 1e-3; the FP8 forms 1e-2
BUDGET = {"f32": 1e-5, "bf16": 1e-3, "f16_scaled": 1e-3, "bf16_split": 1e-3,
          "fp8e4m3_scaled": 1e-2, "fp8e4m3_split": 1e-2}
# bytes per spectrum element stored by each form (planes x element size)
ELEM_BYTES = {"f32": 4, "bf16": 2, "f16_scaled": 2, "bf16_split": 4, "fp8e4m3_scaled": 1,
              "fp8e4m3_split": 2}
# The paper's context (Section 1): about 21 CPU-hours per TB of raw data on a
# 16-core CPU; 1 TB of FP32 values is 2.5e11 sample*channel values.
PAPER_CONTEXT = {"cpu_hours_per_TB": 21.0, "cpu_cores": 16,
                 "sample_channel_updates_per_s": 2.5e11 / (21.0 * 3600.0),
                 "note": "context only (the paper's multi-core CPU gridding of FAST data, "
                         "wall-clock reading; not a measurement of this build)"}
# the sources the gather kernels are compiled from: a traffic record taken on
# other versions of them is not used
GATHER_SRCS = [os.path.join(ROOT, "paper_2012_13173_amd", "csrc", f)
               for f in ("gather.hip", "gather_tile.h", "sphere.h", "hcg_internal.h")]


def gather_source_sha256():
    import hashlib
    h = hashlib.sha256()
    for path in GATHER_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload, kernel="f32"):
    """HBM bytes per gather launch of ``kernel`` (a key of the summary's
    "kernels": "f32" or a form name) from the committed counter summary
    (profiles/traffic_<workload>.json: FETCH_SIZE x its copy-kernel factor +
    WRITE_SIZE), or None if it was taken on another version of the kernel
    source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("gather_source_sha256") != gather_source_sha256():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return float(k["hbm_bytes_per_launch"]) if k else None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def oracle_sample(w, budget_s=15.0, patch=32, max_patches=40, seed=7):
    """Runs the FP64 oracle on seeded patches of patch x patch cells (all
    channels) until ~budget_s of wall time; returns the cells, the oracle's
    values on them and the time it took (the CPU baseline leg)."""
    import oracle
    cores = len(os.sched_getaffinity(0))
    oracle.set_threads(cores)
    g = w.grid
    lon = w.lon.cpu().numpy()
    lat = w.lat.cpu().numpy()
    rng = np.random.default_rng(seed)
    t_total, cells, refs, pairs = 0.0, [], [], []
    R = w.support_deg
    for _ in range(max_patches):
        x0 = int(rng.integers(0, g.nx - patch + 1))
        y0 = int(rng.integers(0, g.ny - patch + 1))
        ix, iy = np.meshgrid(np.arange(x0, x0 + patch), np.arange(y0, y0 + patch))
        c = (iy * g.nx + ix).ravel()
        clon = g.lon0 + (np.array([x0, x0 + patch - 1]) - (g.nx - 1) / 2) * g.dlon
        clat = g.lat0 + (np.array([y0, y0 + patch - 1]) - (g.ny - 1) / 2) * g.dlat
        m = 1.5 * R
        coslat = math.cos(math.radians(max(abs(clat[0]), abs(clat[1])) + m))
        sel = np.nonzero((lat >= clat.min() - m) & (lat <= clat.max() + m)
                         & (lon >= clon.min() - m / coslat) & (lon <= clon.max() + m / coslat))[0]
        rows = w.spectra.index_select(0, torch.from_numpy(sel).to(w.spectra.device)).cpu().numpy()
        t0 = time.perf_counter()
        V, W, npair = oracle.grid_cells(lon[sel], lat[sel], rows, g, w.fwhm_deg, R, c)
        t_total += time.perf_counter() - t0
        cells.append(c)
        refs.append(V)
        pairs.append(npair)
        if t_total >= budget_s:
            break
    return {"cells": np.concatenate(cells), "V": np.concatenate(refs), "t": t_total,
            "pairs": int(np.concatenate(pairs).sum()), "cores": cores, "patch": patch,
            "patches": len(cells)}


def cpu_baseline(w, samp, total_pairs):
    """The oracle's rate on the sample, extrapolated to the whole grid by pair
    work: t_sample x (sum over all cells of their samples within R) / (the
    same sum over the sampled cells)."""
    g = w.grid
    done = samp["cells"].size
    t_full = samp["t"] * total_pairs / max(samp["pairs"], 1)
    return {"value": w.n * w.nchan / t_full, "unit": "sample*channel updates/s",
            "cores": samp["cores"], "kind": "oracle",
            "sample": f"{done} of {g.ncells} cells ({samp['patches']} random "
                      f"{samp['patch']}x{samp['patch']}-cell patches, {samp['pairs']} of "
                      f"{total_pairs} pairs within R), all {w.nchan} channels, FP64 bucketed "
                      f"oracle, {samp['t']:.1f} s measured, whole-grid time extrapolated by "
                      f"pair count ({t_full:.0f} s)"}


def sampled_errors(cube, samp):
    """Per-channel relative L2 error of a GPU cube [C, ny, nx] against the
    oracle on the sampled cells (NaN patterns must agree)."""
    V = samp["V"]
    idx = torch.from_numpy(samp["cells"]).to(cube.device)
    gv = cube.reshape(cube.shape[0], -1).index_select(1, idx).cpu().numpy().astype(np.float64).T
    ok = ~np.isnan(V)
    assert np.array_equal(ok, ~np.isnan(gv)), "NaN patterns differ from the oracle"
    d = np.where(ok, gv - V, 0.0)
    r = np.where(ok, V, 0.0)
    return np.sqrt((d * d).sum(0) / (r * r).sum(0))


FORM_CODE = {"bf16": hcg.HCG_BF16, "f16_scaled": hcg.HCG_F16_SCALED,
             "bf16_split": hcg.HCG_BF16_SPLIT, "fp8e4m3_scaled": hcg.HCG_FP8E4M3_SCALED,
             "fp8e4m3_split": hcg.HCG_FP8E4M3_SPLIT}


def algorithmic_bytes(w, form, packed):
    """Bytes a gather launch must move at least: the spectra once (in the
    form's storage, plan-ordered encodings with their padding to groups of 8
    samples and 16 channels), the sorted unit vectors and permutation once
    (36 B per sample) and the cube once."""
    C = w.nchan
    if packed:
        spec = ELEM_BYTES[form] * 8 * ((w.n + 7) // 8) * ((C + 15) // 16 * 16)
    else:
        spec = ELEM_BYTES[form] * w.n * C
    return float(spec + 36 * w.n + 4 * C * w.grid.ncells)


def time_events(run, reps=3):
    stream = torch.cuda.current_stream()
    run()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    for a, b in evs:
        a.record(stream)
        run()
        b.record(stream)
    torch.cuda.synchronize()
    return float(np.mean([a.elapsed_time(b) for a, b in evs]))


def run_forms(w, order_forms, packed_forms, grid_avg, samp, errs):
    """The matrix-core precision forms on one plan of ``w``: input-order
    encodings (hcg_quantize + hcg_grid) and plan-ordered ones
    (hcg_quantize_packed + hcg_grid_packed); gather times by HIP events,
    encoding times beside, errors against the oracle sample into ``errs``."""
    g = w.grid
    dev = w.spectra.device
    stream = torch.cuda.current_stream()
    updates = w.n * w.nchan
    plan = hcg.hcg_plan(w.lon, w.lat, g, w.fwhm_deg, w.support_deg, nside=w.nside)
    out_cube = torch.empty((w.nchan, g.ny, g.nx), dtype=torch.float32, device=dev)
    forms = {}

    def rates(rec, form, packed, ms):
        alg = algorithmic_bytes(w, form, packed)
        rec["algorithmic_hbm_bytes"] = alg
        rec["hbm_frac_of_peak_algorithmic"] = alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS

    for name in order_forms:
        form = FORM_CODE[name]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        enc, scale = hcg.hcg_quantize(w.spectra, form)
        e1.record(stream)
        ms = time_events(lambda: hcg.hcg_grid(plan, enc, out_cube, dtype=form, chan_scale=scale))
        enc_ms = e0.elapsed_time(e1)
        forms[name] = {"grid_ms": ms, "encode_ms": enc_ms,
                       "grid_updates_per_s": updates / (ms * 1e-3),
                       "speedup_vs_f32_grid": grid_avg / ms,
                       "speedup_vs_f32_grid_incl_encode": grid_avg / (ms + enc_ms)}
        rates(forms[name], name, False, ms)
        del enc
        if samp is not None:
            errs[name] = sampled_errors(out_cube, samp)
        log(f"form {name}: gather {ms:.2f} ms ({grid_avg / ms:.2f}x the FP32 gather), "
            f"encode {enc_ms:.2f} ms")
    # the same forms encoded once in the plan's sorted order
    for name in packed_forms:
        form = FORM_CODE[name]
        enc, scale = hcg.hcg_quantize_packed(plan, w.spectra, form)
        del enc, scale  # the timed call below reuses the cached allocation
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        enc, scale = hcg.hcg_quantize_packed(plan, w.spectra, form)
        e1.record(stream)
        ms = time_events(lambda: hcg.hcg_grid_packed(plan, enc, out_cube, dtype=form,
                                                     chan_scale=scale))
        enc_ms = e0.elapsed_time(e1)
        key = "packed_" + name
        forms[key] = {"grid_ms": ms, "encode_ms": enc_ms,
                      "grid_updates_per_s": updates / (ms * 1e-3),
                      "speedup_vs_f32_grid": grid_avg / ms,
                      "speedup_vs_f32_grid_incl_encode": grid_avg / (ms + enc_ms)}
        rates(forms[key], name, True, ms)
        hbm = measured_traffic(w.name, key)
        if hbm:
            forms[key]["measured_hbm_bytes_per_launch"] = hbm
            forms[key]["measured_hbm_GBps"] = hbm / (ms * 1e-3) / 1e9
        del enc
        if samp is not None:
            errs[key] = sampled_errors(out_cube, samp)
        log(f"plan-ordered form {name}: gather {ms:.2f} ms ({grid_avg / ms:.2f}x the FP32 "
            f"gather), encode {enc_ms:.2f} ms")
    plan.destroy()
    del out_cube
    return forms


def add_errors(forms, errs):
    """Per-form error record: largest and median per-channel relative L2 on
    the oracle sample, and whether the largest meets the form's budget."""
    for k, e in errs.items():
        rec = forms.setdefault(k, {})
        base = k[len("packed_"):] if k.startswith("packed_") else k
        rec["rel_l2_max_over_channels"] = float(e.max())
        rec["rel_l2_median_over_channels"] = float(np.median(e))
        rec["budget"] = BUDGET[base]
        rec["meets_budget"] = bool(e.max() <= BUDGET[base])


def run_c2(oracle_budget_s=8.0):
    """The metric's many-channel configuration: 1,976,000 samples x 8,192
    channels -> 400 x 400 cells (the FP32 gather, FP16 x channel scale, BF16
    and BF16 hi+lo, input order and plan-ordered), every form against the
    oracle on sampled cells."""
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    w = synth.drift_scan_8192(device=dev)
    torch.cuda.synchronize()
    log(f"c2: synthesised {w.n} samples x {w.nchan} channels in {time.perf_counter() - t0:.1f} s")
    g = w.grid
    plan = hcg.hcg_plan(w.lon, w.lat, g, w.fwhm_deg, w.support_deg, nside=w.nside)
    stats = plan.stats()
    cube = torch.empty((w.nchan, g.ny, g.nx), dtype=torch.float32, device=dev)
    ms = time_events(lambda: hcg.hcg_grid(plan, w.spectra, cube))
    plan.destroy()
    updates = w.n * w.nchan
    log(f"c2: FP32 gather {ms:.2f} ms")
    errs = {}
    samp = None
    if oracle_budget_s > 0:
        samp = oracle_sample(w, budget_s=oracle_budget_s, patch=16)
        errs["f32"] = sampled_errors(cube, samp)
    del cube
    torch.cuda.empty_cache()
    forms = {"f32": {"grid_ms": ms, "grid_updates_per_s": updates / (ms * 1e-3),
                     "pair_updates_per_s": stats["pairs"] * w.nchan / (ms * 1e-3),
                     "tflops": 2.0 * stats["pairs"] * w.nchan / (ms * 1e-3) / 1e12}}
    forms.update(run_forms(w, ["f16_scaled", "bf16_split", "bf16"],
                           ["f16_scaled", "bf16_split", "bf16"], ms, samp, errs))
    add_errors(forms, errs)
    best = None
    for k, r in forms.items():
        if k != "f32" and r.get("meets_budget") and BUDGET.get(k.replace("packed_", "")) == 1e-3:
            if best is None or r["grid_ms"] < forms[best]["grid_ms"]:
                best = k
    out = {"workload": w.name, "n_samples": w.n, "nchan": w.nchan, "grid": [g.nx, g.ny],
           "pairs": stats["pairs"], "forms": forms,
           "fastest_form_within_1e-3": best,
           "speedup_of_fastest_within_1e-3": (ms / forms[best]["grid_ms"]) if best else None}
    if samp is not None:
        out["oracle_sample"] = (f"{samp['cells'].size} cells ({samp['patches']} patches of "
                                f"16x16), all {w.nchan} channels")
    del w
    torch.cuda.empty_cache()
    return out


def run_host_stream(w, slabs, samp, pageable_slab=256):
    """hcg_grid_host with the spectra and the cube in host memory: wall time
    per cube (plan built beforehand, not timed) and the host-to-device rate it
    implies, beside the rate of one plain 4 GiB page-locked host-to-device
    copy (the bound of the stream).  Page-locked: the first channels that fit
    20 GB of spectra (torch rounds page-locked blocks up to a power of two, and
    the page-locked total is limited), once per slab width; pageable: the
    whole cube, once; spectra stored as FP16 x per-channel scale (half the
    host bytes), page-locked, the same channels, once per slab width."""
    g = w.grid
    dev = w.spectra.device
    nch = int(min(w.nchan, max(16, 20e9 // (4 * w.n) // 16 * 16)))
    t0 = time.perf_counter()
    spec_h = torch.empty((w.n, nch), dtype=torch.float32, pin_memory=True)
    spec_h.copy_(w.spectra[:, :nch])
    cube_h = torch.empty((nch, g.ny, g.nx), dtype=torch.float32, pin_memory=True)
    W_h = torch.empty((g.ny, g.nx), dtype=torch.float32, pin_memory=True)
    log(f"host stream: page-locked copy of {nch} channels made in "
        f"{time.perf_counter() - t0:.1f} s")
    chunk = min(spec_h.numel(), 1 << 30)
    dst = torch.empty(chunk, dtype=torch.float32, device=dev)
    src = spec_h.view(-1)[:chunk]
    dst.copy_(src, non_blocking=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        dst.copy_(src, non_blocking=True)
    torch.cuda.synchronize()
    copy_gbs = 3 * 4.0 * chunk / (time.perf_counter() - t0) / 1e9
    del dst
    samp_h = None
    if samp is not None:
        samp_h = dict(samp, V=samp["V"][:, :nch])
    plan = hcg.hcg_plan(w.lon, w.lat, g, w.fwhm_deg, w.support_deg, nside=w.nside)

    def timed(spec, cube, W, cs, reps, dtype=hcg.HCG_F32, scale=None):
        hcg.hcg_grid_host(plan, spec, cube, W, slab=cs, dtype=dtype, chan_scale=scale)
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            hcg.hcg_grid_host(plan, spec, cube, W, slab=cs, dtype=dtype, chan_scale=scale)
            ts.append(time.perf_counter() - t0)
        ms = 1e3 * float(np.mean(ts))
        C = spec.shape[-1]
        h2d = float(spec.element_size() * spec.numel())
        return {"nchan": C, "slab": cs, "ms": ms, "updates_per_s": w.n * C / (ms * 1e-3),
                "h2d_bytes": h2d, "d2h_bytes": 4.0 * C * g.ncells,
                "h2d_GBps": h2d / (ms * 1e-3) / 1e9,
                "frac_of_plain_copy": h2d / (ms * 1e-3) / 1e9 / copy_gbs}

    out = {"plain_h2d_copy_GBps": copy_gbs, "page_locked": [], "pageable": None}
    for cs in slabs:
        rec = timed(spec_h, cube_h, W_h, cs, 2)
        if samp_h is not None:
            rec["rel_l2_max_over_channels"] = float(sampled_errors(cube_h, samp_h).max())
        out["page_locked"].append(rec)
        log(f"host stream, page-locked, slabs of {cs}: {rec['ms']:.1f} ms per {nch}-channel "
            f"cube, host-to-device {rec['h2d_GBps']:.1f} GB/s (plain copy {copy_gbs:.1f} GB/s)")
    del spec_h
    # the same channels stored as FP16 x scale (encoded on the device, copied
    # to page-locked memory outside the timed calls)
    enc, scale = hcg.hcg_quantize(w.spectra[:, :nch].contiguous(), hcg.HCG_F16_SCALED)
    enc_h = torch.empty(tuple(enc.shape), dtype=enc.dtype, pin_memory=True)
    enc_h.copy_(enc)
    scale_h = scale.cpu()
    del enc, scale
    torch.cuda.empty_cache()
    out["page_locked_f16_scaled"] = []
    for cs in slabs:
        rec = timed(enc_h, cube_h, W_h, cs, 2, hcg.HCG_F16_SCALED, scale_h)
        if samp_h is not None:
            rec["rel_l2_max_over_channels"] = float(sampled_errors(cube_h, samp_h).max())
        out["page_locked_f16_scaled"].append(rec)
        log(f"host stream, page-locked FP16 x scale, slabs of {cs}: {rec['ms']:.1f} ms per "
            f"{nch}-channel cube, host-to-device {rec['h2d_GBps']:.1f} GB/s")
    del enc_h, cube_h
    if pageable_slab:
        t0 = time.perf_counter()
        spec_p = w.spectra.cpu()
        cube_p = torch.empty((w.nchan, g.ny, g.nx), dtype=torch.float32)
        log(f"host stream: pageable copy of {w.nchan} channels made in "
            f"{time.perf_counter() - t0:.1f} s")
        rec = timed(spec_p, cube_p, W_h, pageable_slab, 1)
        if samp is not None:
            rec["rel_l2_max_over_channels"] = float(sampled_errors(cube_p, samp).max())
        out["pageable"] = rec
        log(f"host stream, pageable, slabs of {pageable_slab}: {rec['ms']:.1f} ms per "
            f"{w.nchan}-channel cube, host-to-device {rec['h2d_GBps']:.1f} GB/s")
        del spec_p, cube_p
    plan.destroy()
    return out


def sweep_points(name):
    """(label, paper_field kwargs) of the paper's scaling experiments
    (Section 4.2): e2 coarsening at 10^8 samples on 5 deg x 5 deg over cell
    sizes; e3 input volume 10^3 .. 3.6 x 10^8 on 5 deg x 5 deg, 90 x 90;
    e4 field size 0.1 .. 60 deg at 10^5 samples per square degree, 200" cells."""
    if name == "e2":
        return [(f'cell {c:g}"', dict(n=100_000_000, side_deg=5.0, cell_arcsec=c))
                for c in (200.0, 100.0, 50.0, 25.0)]
    if name == "e3":
        return [(f"N {n:.2g}", dict(n=n, side_deg=5.0))
                for n in (1_000, 10_000, 100_000, 1_000_000, 10_000_000, 100_000_000,
                          360_000_000)]
    return [(f"field {d:g} deg", dict(n=int(round(1e5 * d * d)), side_deg=d))
            for d in (0.1, 0.5, 1.0, 2.0, 5.0, 10.0, 20.0, 40.0, 60.0)]


def run_sweep(args):
    """Plan, the tile gather (hcg_grid, one channel) and the paper's
    thread-per-row-cells gather (hcg_grid_rowthreads, gamma 1..3, 64 and
    256 threads per block) on each point of a sweep; the maps of the two
    gathers are compared.  One JSON line."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()

    def timed(fn, reps=3):
        fn()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(reps)]
        for a, b in evs:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        return float(np.mean([a.elapsed_time(b) for a, b in evs]))

    rows = []
    for label, kw in sweep_points(args.sweep):
        w = synth.paper_field(device=dev, **kw)
        g = w.grid
        spec = w.spectra[:, 0].contiguous()
        V = torch.empty((g.ny, g.nx), dtype=torch.float32, device=dev)
        Vt = torch.empty((1, g.ny, g.nx), dtype=torch.float32, device=dev)
        plan_ms = timed(lambda: hcg.hcg_plan(w.lon, w.lat, g, w.fwhm_deg, w.support_deg,
                                             nside=w.nside).destroy(), reps=2)
        plan = hcg.hcg_plan(w.lon, w.lat, g, w.fwhm_deg, w.support_deg, nside=w.nside)
        stats = plan.stats()
        rec = {"point": label, "n": w.n, "grid": [g.nx, g.ny], "side_deg": kw["side_deg"],
               "pairs": stats["pairs"], "candidates": stats["candidates"], "plan_ms": plan_ms,
               "tile_gather_ms": timed(lambda: hcg.hcg_grid(plan, spec[:, None], Vt))}
        log(f"  {label}: plan {plan_ms:.2f} ms, tile gather {rec['tile_gather_ms']:.3f} ms")
        ok = ~torch.isnan(Vt[0])
        scale = float(Vt[0][ok].abs().max()) if bool(ok.any()) else 1.0
        paper = {}
        for gamma in (1, 2, 3):
            for block in (64, 256):
                ms = timed(lambda: hcg.hcg_grid_rowthreads(plan, spec, V, gamma=gamma,
                                                           block=block))
                same = bool(torch.equal(torch.isnan(V), ~ok))
                diff = float((V[ok] - Vt[0][ok]).abs().max()) / scale if bool(ok.any()) else 0.0
                paper[f"gamma{gamma}_block{block}"] = {"ms": ms, "nan_same": same,
                                                       "max_rel_diff": diff}
                log(f"  {label}: paper scheme gamma {gamma} block {block}: {ms:.3f} ms")
        rec["paper_scheme"] = paper
        best = min(paper.values(), key=lambda r: r["ms"])["ms"]
        rec["paper_best_ms"] = best
        rec["tile_speedup_vs_paper_best"] = best / rec["tile_gather_ms"]
        plan.destroy()
        rows.append(rec)
        log(f"{args.sweep} {label}: N {w.n}, {g.nx}x{g.ny}, plan {plan_ms:.2f} ms, tile gather "
            f"{rec['tile_gather_ms']:.3f} ms, paper scheme best {best:.3f} ms")
        del w, spec, V, Vt
        torch.cuda.empty_cache()
    print(json.dumps({"sweep": args.sweep, "unit": "ms", "kernel_fwhm_arcsec": 300.0,
                      "support_sigma": 3.0, "rows": rows}), flush=True)


def run_batch(args):
    """64 independent fields of uneven size: one batched launch (persistent
    kernel, hipGraph replay, autotuned) against 64 separate plan + grid calls
    on the same buffers."""
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    ws = synth.batch_fields(device=dev)
    torch.cuda.synchronize()
    tot_in = sum(w.n * w.nchan for w in ws)
    log(f"synthesised {len(ws)} fields, {tot_in:.4g} sample*channels in "
        f"{time.perf_counter() - t0:.1f} s")
    cubes = [torch.empty((w.nchan, w.grid.ny, w.grid.nx), device=dev) for w in ws]
    wts = [torch.empty((w.grid.ny, w.grid.nx), device=dev) for w in ws]
    stream = torch.cuda.current_stream()

    def separate():
        for w, c, W in zip(ws, cubes, wts):
            p = hcg.hcg_plan(w.lon, w.lat, w.grid, w.fwhm_deg, w.support_deg, nside=w.nside)
            hcg.hcg_grid(p, w.spectra, c, W)
            p.destroy()

    fields = [(w.lon, w.lat, w.grid, w.fwhm_deg, w.support_deg) for w in ws]
    spectra = [w.spectra for w in ws]

    def batched(b=None):
        own = b is None
        if own:
            b = hcg.hcg_plan_batch(fields)
        hcg.hcg_grid_batch(b, spectra, cubes, wts)
        if own:
            b.destroy()

    def timed(fn, steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t) / steps

    import tempfile
    os.environ.setdefault("HCG_TUNE_CACHE", os.path.join(tempfile.mkdtemp(), "hcg_tune.txt"))
    separate()  # warm-up, and reference slices (first and last channel of each field)
    torch.cuda.synchronize()
    ref = [torch.stack([c[0], c[-1]]).clone() if w.nchan > 8 else None
           for w, c in zip(ws, cubes)]
    ms_sep = timed(separate, args.steps)
    log(f"64 separate plan+grid calls: {ms_sep:.1f} ms")
    b = hcg.hcg_plan_batch(fields)
    hcg.hcg_grid_batch(b, spectra, cubes, wts)  # tunes and captures
    info = b.info()
    torch.cuda.synchronize()
    def eq_nan(a, b):
        return bool(((a == b) | (torch.isnan(a) & torch.isnan(b))).all())
    same = all(eq_nan(torch.stack([c[0], c[-1]]), r) for c, r in zip(cubes, ref)
               if r is not None)
    ms_grid_b = timed(lambda: batched(b), args.steps)
    b.destroy()
    del ref
    plans = [hcg.hcg_plan(w.lon, w.lat, w.grid, w.fwhm_deg, w.support_deg, nside=w.nside)
             for w in ws]

    def grids_only():
        for p, w, c, W in zip(plans, ws, cubes, wts):
            hcg.hcg_grid(p, w.spectra, c, W)
    ms_grid_sep = timed(grids_only, args.steps)
    for p in plans:
        p.destroy()
    ms_bat = timed(batched, args.steps)
    log(f"batched plan+grid: {ms_bat:.1f} ms; grid only: batched {ms_grid_b:.1f} ms vs "
        f"separate {ms_grid_sep:.1f} ms; autotuner {info['tune_ms']} -> slab "
        f"{info['chan_slab']}, cost order {info['cost_order']}, launch {info['launch']}; identical to separate: {same}")
    out = {
        "metric": "sample*channel updates/s, FP32 gather vs BF16-MFMA at <=1e-3 rel err",
        "value": tot_in / (ms_bat * 1e-3), "unit": "sample*channel updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": ms_bat, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded fields: uniform positions, N(0,1) + lines / point sources)",
        "config": {"workload": "batch_64_fields", "fields": len(ws),
                   "sample_channels": tot_in, "output_cells_channels":
                   sum(w.grid.ncells * w.nchan for w in ws), "parallelism": "single GPU"},
        "separate_calls_ms_per_step": ms_sep,
        "batched_grid_ms": ms_grid_b, "separate_grid_ms": ms_grid_sep,
        "speedup_batched_vs_separate": ms_sep / ms_bat,
        "autotune": {"tune_ms": info["tune_ms"], "chan_slab": info["chan_slab"],
                     "launch": ["persistent", "work items"][info["launch"]],
                     "cost_order": info["cost_order"], "items": info["items"],
                     "persistent_blocks": info["persistent_blocks"]},
        "batched_equals_separate_for_C_gt_8": same,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the low-precision forms")
    ap.add_argument("--no-c2", action="store_true",
                    help="skip the 8,192-channel leg of the default workload")
    ap.add_argument("--workload", default="drift_scan",
                    choices=["drift_scan", "drift_scan_8192", "large", "batch"],
                    help="drift_scan: 9.12M samples x 1024 channels -> 600 x 600 (default); "
                         "drift_scan_8192: 1.976M x 8192 -> 400 x 400; large: 20.064M x 1024 -> "
                         "3000 x 3000; batch: 64 fields")
    ap.add_argument("--sweep", choices=["e2", "e3", "e4"],
                    help="instead of the benchmark: the paper's coarsening (e2), input-volume "
                         "(e3) or field-size (e4) sweep, tile gather against the paper's scheme")
    ap.add_argument("--host-stream", default="",
                    help="comma-separated slab widths: also time hcg_grid_host (spectra and "
                         "cube in page-locked host memory) for each")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run a kernel that reads 1 GiB and writes 1 GiB first (reference "
                         "for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU; --gpus must be 1 (sharding across GPUs is "
              "described, not built)", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.sweep:
        run_sweep(args)
        return
    if args.workload == "batch":
        run_batch(args)
        return
    t0 = time.perf_counter()
    make = {"drift_scan": synth.drift_scan_1024, "drift_scan_8192": synth.drift_scan_8192,
            "large": synth.drift_scan_large}[args.workload]
    w = make(device=dev)
    torch.cuda.synchronize()
    log(f"synthesised {w.n} samples x {w.nchan} channels in {time.perf_counter() - t0:.1f} s")
    g = w.grid
    stream = torch.cuda.current_stream()
    if args.calib_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 2.0, out=dst)  # one elementwise kernel: 1 GiB in, 1 GiB out
        torch.cuda.synchronize()
        del src, dst
    cube = torch.empty((w.nchan, g.ny, g.nx), dtype=torch.float32, device=dev)
    wmap = torch.empty((g.ny, g.nx), dtype=torch.float32, device=dev)

    # exact pair work of this workload (not timed)
    plan = hcg.hcg_plan(w.lon, w.lat, g, w.fwhm_deg, w.support_deg, nside=w.nside)
    stats = plan.stats()
    info = plan.info()
    plan.destroy()
    log(f"plan: nside {info['nside']}, {info['sort_passes']} sort passes, "
        f"{stats['pairs']:.4g} pairs, {stats['candidates']:.4g} candidates")

    def step(evs=None):
        p = hcg.hcg_plan(w.lon, w.lat, g, w.fwhm_deg, w.support_deg, nside=w.nside)
        if evs is not None:
            evs[0].record(stream)
        hcg.hcg_grid(p, w.spectra, cube, wmap)
        if evs is not None:
            evs[1].record(stream)
        p.destroy()

    for i in range(args.warmup):
        step()
        log(f"warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(events[i])
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t0
    grid_ms = [a.elapsed_time(b) for a, b in events]
    ms_step = 1e3 * t_total / args.steps
    grid_avg = float(np.mean(grid_ms))
    log(f"{args.steps} steps: {ms_step:.2f} ms/step, gather {grid_avg:.2f} ms (min "
        f"{min(grid_ms):.2f})")

    updates = w.n * w.nchan
    value = updates / (ms_step * 1e-3)

    # the oracle on sampled cells: the CPU baseline, and the reference for the
    # errors of every form (computed right after each form, whose cube is then
    # freed)
    samp = None
    errs = {}
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        samp = oracle_sample(w)
        errs["f32"] = sampled_errors(cube, samp)
        log(f"oracle sample: {samp['cells'].size} cells in {time.perf_counter() - t0:.1f} s")

    host_stream = None
    if args.host_stream:
        host_stream = run_host_stream(w, [int(x) for x in args.host_stream.split(",")], samp)

    # the matrix-core precision forms on the same plan (encoding timed beside)
    order_forms = {
        "drift_scan": ["bf16", "f16_scaled", "bf16_split", "fp8e4m3_scaled", "fp8e4m3_split"],
        "drift_scan_8192": ["bf16", "f16_scaled", "bf16_split"],
        "large": ["fp8e4m3_scaled", "fp8e4m3_split"],
    }[args.workload]
    packed_forms = {
        "drift_scan": ["f16_scaled", "bf16_split", "fp8e4m3_split", "bf16", "fp8e4m3_scaled"],
        "drift_scan_8192": ["f16_scaled", "bf16_split", "bf16"],
        "large": ["fp8e4m3_split", "fp8e4m3_scaled", "f16_scaled"],
    }[args.workload]
    forms = {}
    if not args.no_forms:
        if samp is not None and args.workload != "drift_scan":
            del cube  # the FP32 cube's errors are taken; make room for the forms' cubes
            torch.cuda.empty_cache()
        forms = run_forms(w, order_forms, packed_forms, grid_avg, samp, errs)
    flops = 2.0 * stats["pairs"] * w.nchan
    achieved = flops / (grid_avg * 1e-3) / 1e12
    traffic = measured_traffic(w.name)
    out = {
        "metric": "sample*channel updates/s, FP32 gather vs BF16-MFMA at <=1e-3 rel err",
        "value": value,
        "unit": "sample*channel updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded 19-beam drift scan, N(0,1) spectra + 32 lines)",
        "config": {"workload": w.name, "n_samples": w.n, "nchan": w.nchan, "grid": [g.nx, g.ny],
                   "cell_arcmin": g.dlon * 60, "fwhm_arcmin": w.fwhm_deg * 60,
                   "support_sigma": 3.0, "nside": w.nside, "parallelism": "single GPU"},
        "plan_ms": ms_step - grid_avg,
        "grid_ms": grid_avg,
        "grid_only_updates_per_s": updates / (grid_avg * 1e-3),
        "pair_updates_per_s": stats["pairs"] * w.nchan / (grid_avg * 1e-3),
        "pairs": stats["pairs"],
        "candidates": stats["candidates"],
        "roofline": {"kernel": "hcg::k_gather_mfma<0, 2, true, false, false, false, false> "
                               "(FP32, 512-channel slabs, input order, narrow support)",
                     "bound": "mfma", "achieved": achieved,
                     "peak": MFMA_FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / MFMA_FP32_PEAK_TFLOPS, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE x 2.0 + "
                                     "WRITE_SIZE, see profiles/)",
                     "traffic_GBps": (traffic / (grid_avg * 1e-3) / 1e9) if traffic else None,
                     "algorithmic_flops_per_launch": flops},
    }
    out["paper_context"] = PAPER_CONTEXT
    if samp is not None:
        cb = cpu_baseline(w, samp, stats["pairs"])
        out["cpu_baseline"] = cb
        forms.setdefault("f32", {"grid_ms": grid_avg, "grid_updates_per_s":
                                 updates / (grid_avg * 1e-3), "speedup_vs_f32_grid": 1.0})
        add_errors(forms, errs)
        log(f"cpu baseline {cb['value']:.3g} /s on {cb['cores']} cores ({samp['t']:.1f} s); "
            "sampled errors " + ", ".join(f"{k} {e.max():.2e}" for k, e in errs.items()))
    if forms:
        out["forms"] = forms
    if host_stream:
        out["host_stream"] = host_stream
    if args.workload == "drift_scan" and not args.no_c2:
        del w, wmap
        cube = None
        torch.cuda.empty_cache()
        out["c2"] = run_c2(0.0 if args.no_cpu_baseline else 8.0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
