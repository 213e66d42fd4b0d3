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
