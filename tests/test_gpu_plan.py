"""GPU parity of the plan steps against the oracle, through the C ABI:
HEALPix pixels and the sort order bit-exact, the ring lookup table exact, and
every sample within R of a cell covered by its tile's candidate ranges."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2012_13173_amd as hcg
import synth
from synth import GridDesc

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _pix_gpu(lon, lat, ns):
    p = hcg.hcg_ang2pix(torch.as_tensor(lon, dtype=torch.float64, device=DEV),
                        torch.as_tensor(lat, dtype=torch.float64, device=DEV), ns)
    return hcg.u32(p)


def _edge_points(ns):
    """Pixel centres, points on ring-centre latitudes, z = +-2/3, poles,
    longitudes 0 / 360 / negative, and uniform points on the sphere."""
    rng = np.random.default_rng(ns)
    pts = []
    for p in rng.integers(0, 12 * ns * ns, 2000):
        pts.append(oracle.pix2ang(ns, int(p)))
    for i in rng.integers(1, 4 * ns, 500):
        z = oracle.ring_z(ns, int(i))
        pts.append((rng.uniform(-360, 720), math.degrees(math.asin(z))))
    z23 = math.degrees(math.asin(2.0 / 3.0))
    for lon in (0.0, 360.0, -0.0, -1e-300, 359.99999999999994, -720.0, 45.0, 90.0, 1e9):
        for lat in (90.0, -90.0, 0.0, z23, -z23, np.nextafter(z23, 0), np.nextafter(z23, 90),
                    30.0, -89.999999):
            pts.append((lon, lat))
    lon = rng.uniform(-180, 540, 200_000)
    lat = np.degrees(np.arcsin(rng.uniform(-1, 1, 200_000)))
    a = np.array(pts)
    return np.concatenate([a[:, 0], lon]), np.concatenate([a[:, 1], lat])


@pytest.mark.parametrize("ns", [1, 2, 64, 4096, 8192, 16384])
def test_ang2pix_bit_exact(ns):
    lon, lat = _edge_points(ns)
    ref = oracle.ang2pix(ns, lon, lat)
    got = _pix_gpu(lon, lat, ns)
    bad = np.nonzero(ref != got)[0]
    assert bad.size == 0, f"{bad.size} pixels differ, first at lon={lon[bad[0]]!r} lat={lat[bad[0]]!r}"


def test_ang2pix_rejects_bad_coordinates():
    for lon, lat in ((0.0, 90.5), (float("nan"), 0.0), (0.0, float("inf")), (float("inf"), 1.0)):
        with pytest.raises(hcg.HcgError) as e:
            _pix_gpu([1.0, lon], [2.0, lat], 64)
        assert e.value.status == hcg.HCG_E_ARG


@pytest.mark.parametrize("n,bits,mode", [
    (1, 8, "rand"), (2, 32, "rand"), (4095, 12, "rand"), (4096, 9, "rand"), (4097, 24, "rand"),
    (100_003, 7, "rand"), (100_003, 32, "rand"), (250_000, 17, "ties"), (70_001, 20, "sorted"),
    (70_001, 20, "reversed"), (50_000, 1, "rand"), (33_333, 16, "const")])
def test_radix_sort_is_stable_and_exact(n, bits, mode):
    rng = np.random.default_rng(n + bits)
    hi = (1 << bits)
    if mode == "rand":
        k = rng.integers(0, hi, n, dtype=np.uint64)
    elif mode == "ties":
        k = rng.integers(0, 37, n, dtype=np.uint64) * (hi // 64)
    elif mode == "sorted":
        k = np.sort(rng.integers(0, hi, n, dtype=np.uint64))
    elif mode == "reversed":
        k = np.sort(rng.integers(0, hi, n, dtype=np.uint64))[::-1].copy()
    else:
        k = np.full(n, hi - 1, dtype=np.uint64)
    k32 = k.astype(np.uint32)
    kt = torch.from_numpy(k32.view(np.int32).copy()).to(DEV)
    ko, po = hcg.hcg_sort_keys(kt, bits)
    sk, perm = oracle.sort_keys(k32)
    assert np.array_equal(hcg.u32(ko), sk.astype(np.int64))
    assert np.array_equal(hcg.u32(po), perm.astype(np.int64))
    assert np.array_equal(hcg.u32(kt), k32.astype(np.int64))  # input untouched


def _plan_arrays(w):
    dev = torch.device(DEV)
    plan = hcg.hcg_plan(w.lon.to(dev), w.lat.to(dev), w.grid, w.fwhm_deg, w.support_deg,
                        nside=w.nside)
    info = plan.info()
    keys = hcg.u32(plan.export(hcg.HCG_ARR_KEYS))
    perm = hcg.u32(plan.export(hcg.HCG_ARR_PERM))
    csr = hcg.u32(plan.export(hcg.HCG_ARR_RING_CSR))
    nr = hcg.u32(plan.export(hcg.HCG_ARR_TILE_NRANGES))
    rg = hcg.u32(plan.export(hcg.HCG_ARR_TILE_RANGES)).reshape(-1, info["max_ranges"], 2)
    torch.cuda.synchronize()
    return plan, info, keys, perm, csr, nr, rg


def _plan_cases():
    return [
        ("point_sources", lambda: synth.point_source_field()),
        ("small_cube", lambda: synth.small_cube(n=30_000, nchan=3)),
        ("ra_wrap", lambda: synth.small_cube(n=20_000, nchan=2, lon_c=0.05, nx=40, ny=21,
                                              name="ra_wrap")),
        ("cap_boundary", lambda: synth.small_cube(n=20_000, nchan=2, lat_c=41.8, nx=30, ny=50,
                                                   cell_arcmin=1.0, name="cap_boundary")),
        ("polar_cap", lambda: synth.small_cube(n=20_000, nchan=2, lat_c=75.0, lon_c=300.0,
                                                nx=24, ny=24, name="polar_cap")),
    ]


@pytest.mark.parametrize("name,make", _plan_cases())
def test_plan_keys_sort_csr_and_ranges(name, make):
    w = make()
    plan, info, keys, perm, csr, nr, rg = _plan_arrays(w)
    lon, lat = w.lon.numpy(), w.lat.numpy()
    pix = oracle.ang2pix(w.nside, lon, lat)
    # a1 + a2: keys and stable order bit-exact
    assert info["pix_base"] == pix.min() and info["pix_max"] == pix.max()
    sk, operm = oracle.sort_keys(pix)
    assert np.array_equal(perm, operm)
    assert np.array_equal(keys + info["pix_base"], sk)
    # a4: ring lookup table
    assert info["ring_first"] == oracle.pix2ring(w.nside, int(pix.min()))
    assert info["ring_last"] == oracle.pix2ring(w.nside, int(pix.max()))
    ocsr = oracle.ring_csr(w.nside, sk, info["ring_first"], info["ring_last"])
    ocsr[-1] = len(sk)
    assert np.array_equal(csr, ocsr)
    # a5: every sample within R of a cell is a candidate of that cell's tile
    g = w.grid
    inv = np.empty_like(operm)
    inv[operm] = np.arange(operm.shape[0])
    cells = np.arange(g.ncells)
    nb = oracle.neighbours(lon, lat, g, w.support_deg, cells)
    ntx = info["ntiles_x"]
    missing = 0
    cand_total = 0
    for t in range(info["ntiles_x"] * info["ntiles_y"]):
        tx, ty = t % ntx, t // ntx
        mask = np.zeros(w.n, dtype=bool)
        for a, b in rg[t, :nr[t]]:
            assert a < b and b <= w.n
            mask[a:b] = True
        cand_total += int(mask.sum())
        for iy in range(ty * 8, min(g.ny, ty * 8 + 8)):
            for ix in range(tx * 8, min(g.nx, tx * 8 + 8)):
                need = inv[nb[iy * g.nx + ix]]
                missing += int((~mask[need]).sum())
    assert missing == 0
    st = plan.stats()
    assert st["candidates"] == cand_total
    assert st["pairs"] == sum(len(x) for x in nb)
    plan.destroy()


def test_plan_rejects_bad_samples_and_frees():
    dev = torch.device(DEV)
    g = GridDesc(16, 16, 180.0, 30.0, 1 / 60, 1 / 60)
    lon = torch.full((100,), 180.0, dtype=torch.float64, device=dev)
    lat = torch.full((100,), 30.0, dtype=torch.float64, device=dev)
    lat[57] = float("nan")
    with pytest.raises(hcg.HcgError) as e:
        hcg.hcg_plan(lon, lat, g, 0.05, 0.06)
    assert e.value.status == hcg.HCG_E_ARG
    lat[57] = -91.0
    with pytest.raises(hcg.HcgError):
        hcg.hcg_plan(lon, lat, g, 0.05, 0.06)
    lat[57] = 30.0
    p = hcg.hcg_plan(lon, lat, g, 0.05, 0.06)
    h = p.handle
    p.destroy()
    assert hcg.load().hcg_destroy(h) == hcg.HCG_E_STATE
