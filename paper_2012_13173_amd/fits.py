"""Minimal FITS writer for gridded cubes (the export of the result-processing
module, Section 3.1).

``write_cube`` writes the cube [C][ny][nx] as the primary HDU (BITPIX -32,
big-endian IEEE floats, NaN for cells without samples) and, optionally, the
weight map W [ny][nx] as an IMAGE extension, each with a world coordinate
system for the map's linear longitude/latitude grid.  That grid is exactly the
plate carree projection (CAR) with the reference point on the equator
(Calabretta & Greisen 2002, the WCS reference the paper gives in Section 2.1):
CRVAL = (lon0, 0), CDELT = (dlon, dlat) and the reference pixel placed so that
pixel (ix + 1, iy + 1) is the cell centre lon0 + (ix - (nx-1)/2) dlon,
lat0 + (iy - (ny-1)/2) dlat.  A projected map (``Projection``: CAR, SFL, SIN
or TAN with CRPIX, CDELT, CRVAL and optionally LONPOLE / LATPOLE, the target
that ``hcg_wcs_centres`` and ``hcg_plan_ex`` grid onto) is written with its
own cards.  The third axis is the channel index.

Layout follows the FITS standard 4.0: 80-character ASCII cards in 2880-byte
header blocks ending with END, data padded to a multiple of 2880 bytes.
"""
from __future__ import annotations

import numpy as np

BLOCK = 2880


def _card(key: str, value=None, comment: str = "") -> bytes:
    if value is None:
        text = key.ljust(80)
    else:
        if isinstance(value, bool):
            v = "T" if value else "F"
            v = v.rjust(20)
        elif isinstance(value, (int, np.integer)):
            v = str(int(value)).rjust(20)
        elif isinstance(value, (float, np.floating)):
            v = repr(float(value)).upper()
            if "E" not in v and "." not in v:
                v += ".0"
            v = v.rjust(20)
        else:
            s = str(value).replace("'", "''")
            v = ("'" + s.ljust(8) + "'").ljust(20)
        text = f"{key:<8}= {v}"
        if comment:
            text += " / " + comment
        text = text[:80].ljust(80)
    b = text.encode("ascii")
    assert len(b) == 80
    return b


def _header(cards) -> bytes:
    h = b"".join(cards) + _card("END")
    return h + b" " * ((-len(h)) % BLOCK)


def _data(a: np.ndarray) -> bytes:
    d = np.ascontiguousarray(a, dtype=">f4").tobytes()
    return d + b"\0" * ((-len(d)) % BLOCK)


def grid_wcs(grid, ctype=("RA", "DEC")):
    """WCS cards of a linear lon/lat grid (nx, ny, lon0, lat0, dlon, dlat) as
    CAR with the reference point on the equator."""
    crpix1 = (grid.nx + 1) / 2.0
    crpix2 = (grid.ny + 1) / 2.0 - grid.lat0 / grid.dlat
    return [
        _card("CTYPE1", ctype[0].ljust(4, "-") + "-CAR"),
        _card("CRPIX1", float(crpix1)), _card("CRVAL1", float(grid.lon0)),
        _card("CDELT1", float(grid.dlon)), _card("CUNIT1", "deg"),
        _card("CTYPE2", ctype[1].ljust(4, "-") + "-CAR"),
        _card("CRPIX2", float(crpix2)), _card("CRVAL2", 0.0),
        _card("CDELT2", float(grid.dlat)), _card("CUNIT2", "deg"),
    ]


class Projection:
    """A projected map: ``proj`` in CAR, SFL, SIN, TAN; FITS reference pixel
    ``crpix`` (1-based), ``cdelt`` and ``crval`` in degrees; ``lonpole`` None
    for its default."""

    def __init__(self, proj, nx, ny, crpix, cdelt, crval, lonpole=None, latpole=90.0):
        if proj.upper() not in ("CAR", "SFL", "SIN", "TAN"):
            raise ValueError(f"projection {proj} is not one of CAR, SFL, SIN, TAN")
        self.proj, self.nx, self.ny = proj.upper(), int(nx), int(ny)
        self.crpix = (float(crpix[0]), float(crpix[1]))
        self.cdelt = (float(cdelt[0]), float(cdelt[1]))
        self.crval = (float(crval[0]), float(crval[1]))
        self.lonpole = None if lonpole is None else float(lonpole)
        self.latpole = float(latpole)


def projection_wcs(pr: Projection, ctype=("RA", "DEC")):
    """WCS cards of a projected map."""
    cards = []
    for ax in (0, 1):
        k = str(ax + 1)
        cards += [_card("CTYPE" + k, ctype[ax].ljust(4, "-") + "-" + pr.proj),
                  _card("CRPIX" + k, pr.crpix[ax]), _card("CRVAL" + k, pr.crval[ax]),
                  _card("CDELT" + k, pr.cdelt[ax]), _card("CUNIT" + k, "deg")]
    if pr.lonpole is not None:
        cards.append(_card("LONPOLE", pr.lonpole))
    cards.append(_card("LATPOLE", pr.latpole))
    return cards


def write_cube(path: str, cube, grid, weights=None, bunit: str = "",
               fwhm_deg: float | None = None) -> None:
    """Writes the cube [C][ny][nx] (float32; NaN where W = 0) and optionally W
    [ny][nx] to ``path``.  ``grid`` is the linear grid or a ``Projection``.
    ``cube`` and ``weights`` may be numpy arrays or CPU torch tensors."""
    wcs_cards = projection_wcs if isinstance(grid, Projection) else grid_wcs
    cube = np.asarray(cube, dtype=np.float32)
    if cube.ndim != 3 or cube.shape[1:] != (grid.ny, grid.nx):
        raise ValueError(f"cube must be [C, {grid.ny}, {grid.nx}]")
    C = cube.shape[0]
    w = None
    if weights is not None:
        w = np.asarray(weights, dtype=np.float32)
        if w.shape != (grid.ny, grid.nx):
            raise ValueError(f"weights must be [{grid.ny}, {grid.nx}]")
    cards = [_card("SIMPLE", True, "conforms to FITS standard"), _card("BITPIX", -32),
             _card("NAXIS", 3), _card("NAXIS1", grid.nx), _card("NAXIS2", grid.ny),
             _card("NAXIS3", C), _card("EXTEND", weights is not None)]
    cards += wcs_cards(grid)
    cards += [_card("CTYPE3", "CHANNEL"), _card("CRPIX3", 1.0), _card("CRVAL3", 0.0),
              _card("CDELT3", 1.0)]
    if bunit:
        cards.append(_card("BUNIT", bunit))
    if fwhm_deg is not None:
        cards.append(_card("BMAJ", float(fwhm_deg), "gridding kernel FWHM (deg)"))
    with open(path, "wb") as f:
        f.write(_header(cards))
        f.write(_data(cube))
        if w is not None:
            ext = [_card("XTENSION", "IMAGE", "image extension"), _card("BITPIX", -32),
                   _card("NAXIS", 2), _card("NAXIS1", grid.nx), _card("NAXIS2", grid.ny),
                   _card("PCOUNT", 0), _card("GCOUNT", 1), _card("EXTNAME", "WEIGHTS")]
            ext += wcs_cards(grid)
            f.write(_header(ext))
            f.write(_data(w))
