"""Seeded synthetic inputs for gridding: sample positions, spectra and target grids.

This package holds no gridding arithmetic.  It makes the inputs that both the
HIP path and the CPU oracle consume: coordinate-uniform random fields with
Gaussian noise and point sources (the test data recipe of HCGrid's Section 4,
after Cygrid), and 19-beam drift-scan sampling patterns shaped like FAST's
multibeam survey mode (Section 1: ~1.15' Dec spacing of the 19 tracks from a
23.4 deg rotation, up to 10 samples per second).

Everything is drawn from ``torch.Generator`` seeded explicitly, on the device
asked for; a workload drawn on the CPU and copied to the GPU gives both sides
the same bytes.  Sky signals (point sources, spectral lines) use a flat-sky
Gaussian profile around their centre; they are test signal, not the method.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import torch

ARCMIN = 1.0 / 60.0
ARCSEC = 1.0 / 3600.0
FWHM_TO_SIGMA = 1.0 / (2.0 * math.sqrt(2.0 * math.log(2.0)))


@dataclass(frozen=True)
class GridDesc:
    """Linear lon/lat target grid; cell (ix, iy) is centred at
    lon0 + (ix - (nx-1)/2) dlon, lat0 + (iy - (ny-1)/2) dlat (degrees)."""
    nx: int
    ny: int
    lon0: float
    lat0: float
    dlon: float
    dlat: float

    @property
    def ncells(self) -> int:
        return self.nx * self.ny


@dataclass
class Workload:
    name: str
    lon: torch.Tensor            # [N] float64 degrees
    lat: torch.Tensor            # [N] float64 degrees
    spectra: torch.Tensor        # [N, C] float32, channel-fastest
    grid: GridDesc
    fwhm_deg: float
    support_deg: float
    nside: int
    sources: list = field(default_factory=list)  # (lon, lat, ...) of injected signals

    @property
    def n(self) -> int:
        return int(self.lon.shape[0])

    @property
    def nchan(self) -> int:
        return int(self.spectra.shape[1])

    def to(self, device) -> "Workload":
        return Workload(self.name, self.lon.to(device), self.lat.to(device),
                        self.spectra.to(device), self.grid, self.fwhm_deg, self.support_deg,
                        self.nside, list(self.sources))


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def _uniform(g, n, lo, hi, device):
    return lo + (hi - lo) * torch.rand(n, generator=g, dtype=torch.float64, device=device)


def uniform_positions(n, lon_c, lat_c, width_deg, height_deg, seed, device="cpu"):
    """Coordinate-uniform positions in [lon_c +- w/2) x [lat_c +- h/2)."""
    g = _gen(seed, device)
    lon = _uniform(g, n, lon_c - width_deg / 2, lon_c + width_deg / 2, device)
    lat = _uniform(g, n, lat_c - height_deg / 2, lat_c + height_deg / 2, device)
    return lon, lat


def hex19_offsets_arcmin(rotation_deg: float = 23.4, dec_step_arcmin: float = 1.15):
    """On-sky (east, north) offsets of a 19-beam hexagonal feed rotated by
    ``rotation_deg``.  The lattice spacing is chosen so that the two lattice
    directions project onto Dec in steps of 2 and ~5 units of dec_step."""
    th = math.radians(rotation_deg)
    a = 2.0 * dec_step_arcmin / math.sin(th)
    pts = []
    for m in range(-2, 3):
        for n in range(-2, 3):
            if abs(m + n) <= 2:
                x = a * (m + 0.5 * n)
                y = a * (math.sqrt(3.0) / 2.0) * n
                pts.append((x * math.cos(th) - y * math.sin(th),
                            x * math.sin(th) + y * math.cos(th)))
    return pts


def drift_scan_positions(nstrips, strip_spacing_arcmin, dec_c, ra_start, nsamp, step_arcsec,
                         device="cpu"):
    """19-beam drift-scan tracks: ``nstrips`` strips centred on Dec
    dec_c + (k - (nstrips-1)/2) * spacing; each beam takes ``nsamp`` samples
    stepping ``step_arcsec`` of RA from ``ra_start`` (RA offsets of the beams
    are divided by cos Dec).  Deterministic; returns float64 lon, lat."""
    beams = hex19_offsets_arcmin()
    ks = torch.arange(nstrips, dtype=torch.float64, device=device)
    dec_strip = dec_c + (ks - 0.5 * (nstrips - 1)) * strip_spacing_arcmin * ARCMIN
    j = torch.arange(nsamp, dtype=torch.float64, device=device)
    ra_track = ra_start + j * step_arcsec * ARCSEC
    bx = torch.tensor([b[0] for b in beams], dtype=torch.float64, device=device) * ARCMIN
    by = torch.tensor([b[1] for b in beams], dtype=torch.float64, device=device) * ARCMIN
    dec_beam = dec_strip[:, None] + by[None, :]                        # [S, 19]
    ra_off = bx[None, :] / torch.cos(torch.deg2rad(dec_beam))          # [S, 19]
    lat = dec_beam[:, :, None].expand(nstrips, 19, nsamp)
    lon = ra_track[None, None, :] + ra_off[:, :, None]
    return lon.reshape(-1).contiguous(), lat.reshape(-1).contiguous()


def _flat_offsets_deg(lon, lat, lon_s, lat_s):
    dx = (lon - lon_s) * math.cos(math.radians(lat_s))
    dy = lat - lat_s
    return dx, dy


def add_point_sources(values, lon, lat, n_src, amp, fwhm_deg, lon_c, lat_c, width, height,
                      seed, device):
    """Adds ``n_src`` circular Gaussian sources of peak ``amp`` at seeded
    centres inset by 2 FWHM from the field edge; returns their centres."""
    g = _gen(seed, "cpu")
    inset = 2.0 * fwhm_deg
    cl = lon_c - width / 2 + inset + (width - 2 * inset) * torch.rand(n_src, generator=g,
                                                                     dtype=torch.float64)
    cb = lat_c - height / 2 + inset + (height - 2 * inset) * torch.rand(n_src, generator=g,
                                                                       dtype=torch.float64)
    sig = fwhm_deg * FWHM_TO_SIGMA
    out = []
    for s in range(n_src):
        dx, dy = _flat_offsets_deg(lon, lat, float(cl[s]), float(cb[s]))
        values += (amp * torch.exp(-(dx * dx + dy * dy) / (2 * sig * sig))).to(values.dtype)
        out.append((float(cl[s]), float(cb[s]), float(amp), float(fwhm_deg)))
    return out


def add_lines(spectra, lon, lat, n_lines, lon_c, lat_c, width, height, fwhm_sp_deg, seed):
    """Adds ``n_lines`` Gaussian-profile spectral lines: spatial FWHM
    ``fwhm_sp_deg``, peak U[1, 10], centre channel U[0, C), spectral FWHM
    U[4, 64] channels (capped at C/4).  Touches only samples within 3 spatial
    FWHM and channels within 4 spectral sigma."""
    C = spectra.shape[1]
    g = _gen(seed, "cpu")
    inset = 2.0 * fwhm_sp_deg
    u = torch.rand((n_lines, 5), generator=g, dtype=torch.float64)
    sig_sp = fwhm_sp_deg * FWHM_TO_SIGMA
    out = []
    for i in range(n_lines):
        cl = lon_c - width / 2 + inset + (width - 2 * inset) * float(u[i, 0])
        cb = lat_c - height / 2 + inset + (height - 2 * inset) * float(u[i, 1])
        amp = 1.0 + 9.0 * float(u[i, 2])
        c0 = C * float(u[i, 3])
        fw = min(4.0 + 60.0 * float(u[i, 4]), max(C / 4.0, 1.0))
        sch = fw * FWHM_TO_SIGMA
        dx, dy = _flat_offsets_deg(lon, lat, cl, cb)
        r2 = dx * dx + dy * dy
        idx = torch.nonzero(r2 < (3.0 * fwhm_sp_deg) ** 2).flatten()
        lo = max(0, int(math.floor(c0 - 4 * sch)))
        hi = min(C, int(math.ceil(c0 + 4 * sch)) + 1)
        if idx.numel() and hi > lo:
            sp = amp * torch.exp(-r2[idx] / (2 * sig_sp * sig_sp))
            ch = torch.arange(lo, hi, dtype=torch.float64, device=spectra.device)
            prof = torch.exp(-((ch - c0) ** 2) / (2 * sch * sch))
            spectra[idx, lo:hi] += (sp[:, None] * prof[None, :]).to(spectra.dtype)
        out.append((cl, cb, amp, c0, fw))
    return out


def nside_for(fwhm_deg: float) -> int:
    """Smallest power of two whose mean HEALPix pixel size is at most half the
    kernel sigma (the 'hpx_max_resolution ~ sigma_kernel/2' rule for a 3 sigma
    support, Section 3.6 (iii)); capped at 16384."""
    sig = math.radians(fwhm_deg * FWHM_TO_SIGMA)
    ns = 1
    while ns < 16384 and math.sqrt(4 * math.pi / (12.0 * ns * ns)) > sig / 2:
        ns *= 2
    return ns


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

SEED0 = 13173


def point_source_field(n=10_000, nchan=1, seed=SEED0, device="cpu", side_deg=1.0,
                       cell_arcmin=1.0, fwhm_arcmin=3.0, n_src=5, amp=10.0, lon_c=180.0,
                       lat_c=30.0, nside=4096, support_sigma=3.0) -> Workload:
    """Uniform random positions in a side x side field, N(0,1) values plus
    ``n_src`` point sources of FWHM 3'.  Defaults: 10,000 samples on 1 deg x 1 deg
    at (180, 30), 60 x 60 cells of 1', kernel FWHM 3', support 3 sigma, nside 4096."""
    lon, lat = uniform_positions(n, lon_c, lat_c, side_deg, side_deg, seed, device)
    g = _gen(seed + 1, device)
    spec = torch.randn((n, nchan), generator=g, dtype=torch.float32, device=device)
    vals = torch.zeros(n, dtype=torch.float64, device=device)
    src = add_point_sources(vals, lon, lat, n_src, amp, 3.0 * ARCMIN, lon_c, lat_c, side_deg,
                            side_deg, seed + 2, device)
    spec += vals.to(torch.float32)[:, None]
    ncell = int(round(side_deg / (cell_arcmin * ARCMIN)))
    grid = GridDesc(ncell, ncell, lon_c, lat_c, cell_arcmin * ARCMIN, cell_arcmin * ARCMIN)
    fwhm = fwhm_arcmin * ARCMIN
    return Workload("point_sources", lon, lat, spec, grid, fwhm,
                    support_sigma * fwhm * FWHM_TO_SIGMA, nside, src)


def drift_scan_cube(nstrips, nsamp, nchan, grid_n, cell_arcmin, fwhm_arcmin, seed,
                    device="cpu", lon_c=180.0, lat_c=30.0, n_lines=32, beam_fwhm_arcmin=2.9,
                    step_arcsec=1.5, support_sigma=3.0, nside=None, name="drift_scan",
                    noise=True) -> Workload:
    """19-beam drift scan covering the grid: ``nstrips`` strips spread over the
    grid's Dec extent, ``nsamp`` samples per beam at ``step_arcsec`` of RA,
    spectra N(0,1) plus ``n_lines`` spectral lines of spatial FWHM 2.9'."""
    side = grid_n * cell_arcmin * ARCMIN
    ra_len = nsamp * step_arcsec * ARCSEC
    lon, lat = drift_scan_positions(nstrips, side * 60.0 / nstrips, lat_c, lon_c - ra_len / 2,
                                    nsamp, step_arcsec, device)
    n = lon.shape[0]
    g = _gen(seed, device)
    if noise:
        spec = torch.randn((n, nchan), generator=g, dtype=torch.float32, device=device)
    else:
        spec = torch.zeros((n, nchan), dtype=torch.float32, device=device)
    src = add_lines(spec, lon, lat, n_lines, lon_c, lat_c, side, side,
                    beam_fwhm_arcmin * ARCMIN, seed + 1)
    grid = GridDesc(grid_n, grid_n, lon_c, lat_c, cell_arcmin * ARCMIN, cell_arcmin * ARCMIN)
    fwhm = fwhm_arcmin * ARCMIN
    return Workload(name, lon, lat, spec, grid, fwhm, support_sigma * fwhm * FWHM_TO_SIGMA,
                    nside if nside else nside_for(fwhm), src)


def drift_scan_1024(device="cpu", seed=SEED0 + 1) -> Workload:
    """Drift-scan map: 40 strips x 19 beams x 12,000 samples (5 deg of RA at
    1.5" steps) = 9,120,000 samples x 1,024 float32 channels; 600 x 600 cells
    of 0.5', kernel FWHM 3', support 3 sigma, nside 8192."""
    return drift_scan_cube(40, 12_000, 1024, 600, 0.5, 3.0, seed, device,
                           name="drift_scan_600x600_c1024")


def drift_scan_8192(device="cpu", seed=SEED0 + 2) -> Workload:
    """Drift-scan cube: 13 strips x 19 beams x 8,000 samples = 1,976,000 samples
    x 8,192 channels; 400 x 400 cells of 0.5', kernel FWHM 3', support 3 sigma."""
    return drift_scan_cube(13, 8_000, 8192, 400, 0.5, 3.0, seed, device,
                           name="drift_scan_400x400_c8192")


def drift_scan_large(device="cpu", seed=SEED0 + 4) -> Workload:
    """Large cube: 44 strips x 19 beams x 24,000 samples = 20,064,000 samples x
    1,024 channels on 10 deg x 10 deg; 3000 x 3000 cells of 0.2', FWHM 2.9'."""
    return drift_scan_cube(44, 24_000, 1024, 3000, 0.2, 2.9, seed, device,
                           name="drift_scan_3000x3000_c1024")


def small_cube(n=20_000, nchan=67, nx=45, ny=37, cell_arcmin=0.75, fwhm_arcmin=3.0,
               seed=SEED0 + 100, device="cpu", lon_c=180.0, lat_c=30.0, nside=None,
               pad_arcmin=4.0, name="small_cube", support_sigma=3.0) -> Workload:
    """Uniform positions covering the grid plus ``pad_arcmin`` on every side,
    N(0,1) spectra with a few lines: a multi-tile, ragged-edge parity case.
    The support radius is ``support_sigma`` kernel sigmas."""
    w = nx * cell_arcmin * ARCMIN + 2 * pad_arcmin * ARCMIN
    h = ny * cell_arcmin * ARCMIN + 2 * pad_arcmin * ARCMIN
    lon, lat = uniform_positions(n, lon_c, lat_c, w, h, seed, device)
    g = _gen(seed + 1, device)
    spec = torch.randn((n, nchan), generator=g, dtype=torch.float32, device=device)
    src = add_lines(spec, lon, lat, 4, lon_c, lat_c, w, h, 2.9 * ARCMIN, seed + 2)
    grid = GridDesc(nx, ny, lon_c, lat_c, cell_arcmin * ARCMIN, cell_arcmin * ARCMIN)
    fwhm = fwhm_arcmin * ARCMIN
    return Workload(name, lon, lat, spec, grid, fwhm, support_sigma * fwhm * FWHM_TO_SIGMA,
                    nside if nside else nside_for(fwhm), src)


def paper_field(n, side_deg=5.0, cell_arcsec=200.0, fwhm_arcsec=300.0, seed=SEED0 + 200,
                device="cpu", lon_c=180.0, lat_c=30.0, name=None) -> Workload:
    """The simulation of the paper's experiments (Section 4): one N(0,1) value
    at each of n coordinate-uniform random positions in a side x side field,
    gridded onto side / cell cells per axis (5 deg at 200" = 90 x 90), kernel
    FWHM 300", support 3 sigma, nside by the sigma/2 rule."""
    lon, lat = uniform_positions(n, lon_c, lat_c, side_deg, side_deg, seed, device)
    g = _gen(seed + 1, device)
    spec = torch.randn((n, 1), generator=g, dtype=torch.float32, device=device)
    ncell = max(1, int(round(side_deg * 3600.0 / cell_arcsec)))
    cell = cell_arcsec / 3600.0
    grid = GridDesc(ncell, ncell, lon_c, lat_c, cell, cell)
    fwhm = fwhm_arcsec / 3600.0
    return Workload(name or f"paper_field_{side_deg:g}deg_n{n}", lon, lat, spec, grid, fwhm,
                    3.0 * fwhm * FWHM_TO_SIGMA, nside_for(fwhm), [])


def batch_field_params(nfields=64, seed=SEED0 + 3):
    """Per-field draws of the batched configuration: sample count log-uniform
    in [1e4, 2e6], channels in {1, 64, 512, 2048}, square grid side uniform in
    [100, 1500] cells, kernel FWHM uniform in [2', 6'], cell = FWHM / 3,
    centre RA uniform in [0, 360), Dec uniform in [-20, 20]."""
    g = _gen(seed, "cpu")
    u = torch.rand((nfields, 6), generator=g, dtype=torch.float64)
    chans = (1, 64, 512, 2048)
    out = []
    for f in range(nfields):
        n = int(round(math.exp(math.log(1e4) + (math.log(2e6) - math.log(1e4)) * float(u[f, 0]))))
        C = chans[min(3, int(4 * float(u[f, 1])))]
        side = 100 + min(1400, int(1401 * float(u[f, 2])))
        fwhm = 2.0 + 4.0 * float(u[f, 3])  # arcmin
        out.append({"n": n, "nchan": C, "side": side, "fwhm_arcmin": fwhm,
                    "cell_arcmin": fwhm / 3.0, "lon_c": 360.0 * float(u[f, 4]),
                    "lat_c": -20.0 + 40.0 * float(u[f, 5])})
    return out


def batch_fields(device="cpu", nfields=64, seed=SEED0 + 3, params=None):
    """The batched configuration: ``nfields`` independent fields of uniform
    random positions over their grid, N(0,1) spectra plus 4 lines (or 3 point
    sources for one channel), support 3 sigma, nside by the sigma/2 rule."""
    params = params if params is not None else batch_field_params(nfields, seed)
    ws = []
    for f, p in enumerate(params):
        cell = p["cell_arcmin"] * ARCMIN
        side_deg = p["side"] * cell
        # coordinate extent of the grid in longitude shrinks the sky span at
        # high |Dec|; keep the field inside the grid's coordinate box
        lon, lat = uniform_positions(p["n"], p["lon_c"], p["lat_c"], side_deg, side_deg,
                                     seed + 1000 + f, device)
        gg = _gen(seed + 2000 + f, device)
        spec = torch.randn((p["n"], p["nchan"]), generator=gg, dtype=torch.float32, device=device)
        fwhm = p["fwhm_arcmin"] * ARCMIN
        if p["nchan"] > 1:
            src = add_lines(spec, lon, lat, 4, p["lon_c"], p["lat_c"], side_deg, side_deg,
                            2.0 * fwhm, seed + 3000 + f)
        else:
            vals = torch.zeros(p["n"], dtype=torch.float64, device=device)
            src = add_point_sources(vals, lon, lat, 3, 10.0, fwhm, p["lon_c"], p["lat_c"],
                                    side_deg, side_deg, seed + 3000 + f, device)
            spec += vals.to(torch.float32)[:, None]
        grid = GridDesc(p["side"], p["side"], p["lon_c"], p["lat_c"], cell, cell)
        ws.append(Workload(f"field{f:02d}", lon, lat, spec, grid, fwhm,
                           3.0 * fwhm * FWHM_TO_SIGMA, nside_for(fwhm), src))
    return ws
