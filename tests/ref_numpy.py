"""A third, independent implementation of Eq. (1) in NumPy, for tiny inputs.

It measures angles through the chord between unit vectors,
d = 2 asin(|u - v| / 2), instead of the haversine form used by the C oracle,
so a wrong sign, factor or index in either distance shows up as a mismatch.
"""
import numpy as np

DEG = np.pi / 180.0


def unit(lon_deg, lat_deg):
    lon = np.asarray(lon_deg, dtype=np.float64) * DEG
    lat = np.asarray(lat_deg, dtype=np.float64) * DEG
    return np.stack([np.cos(lat) * np.cos(lon), np.cos(lat) * np.sin(lon), np.sin(lat)], -1)


def cell_centres(grid):
    ix = np.arange(grid.nx, dtype=np.float64)
    iy = np.arange(grid.ny, dtype=np.float64)
    clon = grid.lon0 + (ix - 0.5 * (grid.nx - 1)) * grid.dlon
    clat = grid.lat0 + (iy - 0.5 * (grid.ny - 1)) * grid.dlat
    CL, CB = np.meshgrid(clon, clat)  # [ny, nx]
    return CL.ravel(), CB.ravel()


def distances(grid, lon, lat):
    """[G, N] great-circle distances in radians (chord form)."""
    CL, CB = cell_centres(grid)
    u = unit(CL, CB)[:, None, :]
    v = unit(lon, lat)[None, :, :]
    chord = np.sqrt(((u - v) ** 2).sum(-1))
    return 2.0 * np.arcsin(np.minimum(chord / 2.0, 1.0))


def weights(grid, lon, lat, fwhm_deg, support_deg):
    d = distances(grid, lon, lat)
    sig = fwhm_deg * DEG / (2.0 * np.sqrt(2.0 * np.log(2.0)))
    w = np.exp(-d * d / (2.0 * sig * sig))
    w[d > support_deg * DEG] = 0.0
    return w, d


def grid(lon, lat, spec, grid, fwhm_deg, support_deg):
    """Returns (V [C, ny, nx], W [ny, nx])."""
    spec = np.asarray(spec, dtype=np.float64)
    if spec.ndim == 1:
        spec = spec[:, None]
    w, _ = weights(grid, lon, lat, fwhm_deg, support_deg)
    W = w.sum(1)
    U = w @ spec  # [G, C]
    with np.errstate(invalid="ignore", divide="ignore"):
        V = np.where(W[:, None] > 0, U / W[:, None], np.nan)
    return V.T.reshape(spec.shape[1], grid.ny, grid.nx), W.reshape(grid.ny, grid.nx)


def kernel_weights(cell_lon, cell_lat, lon, lat, kernel, support_deg):
    """[G, N] weights of arbitrary cells and samples for the kernel shapes of
    the oracle (``oracle.Kernel``), with chord distances and the sample's
    bearing taken in the tangent plane of the cell (east / north unit
    vectors), not from spherical trigonometry as in the C oracle."""
    u = unit(cell_lon, cell_lat)[:, None, :]                 # [G, 1, 3]
    v = unit(lon, lat)[None, :, :]                           # [1, N, 3]
    diff = v - u
    chord = np.sqrt((diff ** 2).sum(-1))
    d = 2.0 * np.arcsin(np.minimum(chord / 2.0, 1.0))
    if kernel.type == 0:
        sig = kernel.fwhm * DEG / (2.0 * np.sqrt(2.0 * np.log(2.0)))
        w = np.exp(-d * d / (2.0 * sig * sig))
    elif kernel.type == 1:
        lon_c = np.asarray(cell_lon, dtype=np.float64)[:, None] * DEG
        lat_c = np.asarray(cell_lat, dtype=np.float64)[:, None] * DEG
        east = np.stack([-np.sin(lon_c), np.cos(lon_c), np.zeros_like(lon_c)], -1)
        north = np.stack([-np.sin(lat_c) * np.cos(lon_c), -np.sin(lat_c) * np.sin(lon_c),
                          np.cos(lat_c)], -1)
        xe = (diff * east).sum(-1)
        xn = (diff * north).sum(-1)
        beta = np.arctan2(xe, xn)
        t = beta - kernel.pa * DEG
        k = 2.0 * np.sqrt(2.0 * np.log(2.0))
        sa, sb = kernel.fwhm * DEG / k, kernel.fwhm_minor * DEG / k
        w = np.exp(-0.5 * d * d * (np.cos(t) ** 2 / sa ** 2 + np.sin(t) ** 2 / sb ** 2))
        w[d == 0.0] = 1.0
    else:
        x = d / (kernel.sinc * DEG)
        w = np.sinc(x) * np.exp(-(d / (kernel.taper * DEG)) ** 2)
    w[d > support_deg * DEG] = 0.0
    return w, d


def grid_points(lon, lat, spec, cell_lon, cell_lat, kernel, support_deg, masked=False):
    """Returns (V [G, C], W [G] or [G, C])."""
    spec = np.asarray(spec, dtype=np.float64)
    if spec.ndim == 1:
        spec = spec[:, None]
    w, _ = kernel_weights(cell_lon, cell_lat, lon, lat, kernel, support_deg)
    with np.errstate(invalid="ignore", divide="ignore"):
        if not masked:
            W = w.sum(1)
            V = np.where(W[:, None] != 0, (w @ spec) / W[:, None], np.nan)
        else:
            ok = np.isfinite(spec)
            W = w @ ok.astype(np.float64)
            V = np.where(W != 0, (w @ np.where(ok, spec, 0.0)) / W, np.nan)
    return V, W
