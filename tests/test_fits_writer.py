"""The FITS writer (paper_2012_13173_amd/fits.py; result export of Section 3.1)
read back by a reader written here from the FITS standard 4.0: 80-byte cards
in 2880-byte blocks, big-endian IEEE floats, data padded to whole blocks.  The
world coordinates it writes are checked with the WCS oracle: its CAR cards
must put every pixel centre on the linear lon/lat grid of the gather."""
import numpy as np
import pytest

from oracle import wcs
from paper_2012_13173_amd import fits
from synth import GridDesc


def read_fits(path):
    """[(header dict, data array)] for every HDU."""
    raw = open(path, "rb").read()
    assert len(raw) % 2880 == 0
    hdus, off = [], 0
    while off < len(raw):
        hdr = {}
        while True:
            block = raw[off:off + 2880]
            off += 2880
            done = False
            for i in range(36):
                card = block[80 * i:80 * i + 80].decode("ascii")
                key = card[:8].strip()
                if key == "END":
                    done = True
                    break
                if card[8:10] == "= ":
                    v = card[10:].split(" / ")[0].strip()
                    if v.startswith("'"):
                        v = v[1:v.rindex("'")].rstrip()
                    elif v in ("T", "F"):
                        v = v == "T"
                    else:
                        v = float(v) if any(ch in v for ch in ".E") else int(v)
                    hdr[key] = v
            if done:
                break
        shape = tuple(hdr[f"NAXIS{k}"] for k in range(hdr["NAXIS"], 0, -1))
        n = int(np.prod(shape))
        assert hdr["BITPIX"] == -32
        data = np.frombuffer(raw[off:off + 4 * n], dtype=">f4").reshape(shape)
        off += 4 * n + (-(4 * n)) % 2880
        hdus.append((hdr, data))
    return hdus


@pytest.mark.parametrize("grid", [GridDesc(29, 17, 180.0, 30.0, 0.5 / 60, 0.5 / 60),
                                  GridDesc(40, 31, 0.2, -60.0, -0.01, 0.02)])
def test_cube_and_weights_round_trip(tmp_path, grid):
    rng = np.random.default_rng(5)
    cube = rng.standard_normal((6, grid.ny, grid.nx)).astype(np.float32)
    cube[2, 3, 4] = np.nan
    W = rng.uniform(0, 5, (grid.ny, grid.nx)).astype(np.float32)
    path = str(tmp_path / "cube.fits")
    fits.write_cube(path, cube, grid, W, bunit="K", fwhm_deg=3.0 / 60)
    (h0, d0), (h1, d1) = read_fits(path)
    assert h0["SIMPLE"] is True and h0["NAXIS"] == 3 and h0["EXTEND"] is True
    assert (h0["NAXIS1"], h0["NAXIS2"], h0["NAXIS3"]) == (grid.nx, grid.ny, 6)
    np.testing.assert_array_equal(d0, cube)  # NaN compares equal by position too
    assert h1["XTENSION"] == "IMAGE" and h1["EXTNAME"] == "WEIGHTS"
    np.testing.assert_array_equal(d1, W)
    # the WCS cards put pixel (ix + 1, iy + 1) on the gather's cell centres
    for h in (h0, h1):
        assert h["CTYPE1"] == "RA---CAR" and h["CTYPE2"] == "DEC--CAR"
        lon, lat = wcs.cell_centres("CAR", grid.nx, grid.ny, (h["CRPIX1"], h["CRPIX2"]),
                                    (h["CDELT1"], h["CDELT2"]), (h["CRVAL1"], h["CRVAL2"]))
        iy, ix = np.meshgrid(np.arange(grid.ny), np.arange(grid.nx), indexing="ij")
        elon = grid.lon0 + (ix - (grid.nx - 1) / 2) * grid.dlon
        elat = grid.lat0 + (iy - (grid.ny - 1) / 2) * grid.dlat
        np.testing.assert_allclose((lon - elon + 180) % 360 - 180, 0, atol=1e-9)
        np.testing.assert_allclose(lat, elat, atol=1e-9)


def test_shape_errors(tmp_path):
    g = GridDesc(4, 3, 10.0, 0.0, 0.1, 0.1)
    with pytest.raises(ValueError):
        fits.write_cube(str(tmp_path / "a.fits"), np.zeros((2, 4, 3), np.float32), g)
    with pytest.raises(ValueError):
        fits.write_cube(str(tmp_path / "b.fits"), np.zeros((2, 3, 4), np.float32), g,
                        np.zeros((4, 3), np.float32))


@pytest.mark.parametrize("proj,crval,lonpole", [("SIN", (120.0, 62.0), None),
                                                ("TAN", (10.0, -80.0), None),
                                                ("SFL", (359.9, -35.0), None),
                                                ("CAR", (200.0, 40.0), 0.0)])
def test_projected_map_cards(tmp_path, proj, crval, lonpole):
    pr = fits.Projection(proj, 21, 17, (11.0, 9.5), (-0.01, 0.01), crval, lonpole=lonpole)
    cube = np.zeros((2, 17, 21), np.float32)
    path = str(tmp_path / "p.fits")
    fits.write_cube(path, cube, pr, np.ones((17, 21), np.float32))
    for h, _ in read_fits(path):
        assert h["CTYPE1"] == "RA---" + proj and h["CTYPE2"] == "DEC--" + proj
        assert (h["CRPIX1"], h["CRPIX2"]) == pr.crpix and (h["CDELT1"], h["CDELT2"]) == pr.cdelt
        assert (h["CRVAL1"], h["CRVAL2"]) == pr.crval and h["LATPOLE"] == 90.0
        assert h.get("LONPOLE") == lonpole
        # the cards give back the map's pixel centres through the WCS oracle
        a = wcs.cell_centres(proj, 21, 17, (h["CRPIX1"], h["CRPIX2"]), (h["CDELT1"], h["CDELT2"]),
                             (h["CRVAL1"], h["CRVAL2"]), h.get("LONPOLE"), h["LATPOLE"])
        b = wcs.cell_centres(proj, 21, 17, pr.crpix, pr.cdelt, pr.crval, lonpole, 90.0)
        np.testing.assert_array_equal(a[0], b[0])
        np.testing.assert_array_equal(a[1], b[1])
    with pytest.raises(ValueError):
        fits.Projection("AIT", 4, 4, (1, 1), (1, 1), (0, 0))
