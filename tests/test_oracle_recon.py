"""Pins for the oracle's binning, canonicalisation, NN, Delaunay and linear
interpolation (Algorithm 1, Sections 3.3-3.4), each checked against
something other than the oracle itself: brute force, SciPy, closed forms and
invariants."""
import itertools
import os

import numpy as np
import pytest
from scipy.interpolate import LinearNDInterpolator
from scipy.spatial import ConvexHull, Delaunay, cKDTree

import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def _rand_points(rng, m, lo=-48000, hi=48000, z=None):
    u = rng.integers(lo, hi, m)
    v = rng.integers(lo, hi, m)
    zz = rng.integers(-4000, 4000, m) if z is None else z
    rgb = rng.integers(0, 65536, (m, 3))
    return u, v, zz, rgb


# ---------------------------------------------------------------- binning
def _brute_bins(region, x, y, tile_list):
    S = region.tile_size
    H = S // 2 + region.pad * region.cell
    bins = []
    for t in tile_list:
        cx = region.origin_x + (t % region.tiles_x) * S + S // 2
        cy = region.origin_y + (t // region.tiles_x) * S + S // 2
        sel = [i for i in range(len(x)) if cx - H <= x[i] < cx + H and cy - H <= y[i] < cy + H]
        bins.append(sel)
    return bins


@pytest.mark.parametrize("pad", [16, 0, 40])
def test_bin_matches_brute_force(oracle_lib, pad):
    rng = np.random.default_rng(pad)
    region = synth.Region(origin_x=-12345, origin_y=777, tiles_x=3, tiles_y=2, pad=pad)
    S = region.tile_size
    H = S // 2 + pad * region.cell
    n = 1500
    x = rng.integers(region.origin_x - 70000, region.origin_x + 3 * S + 70000, n)
    y = rng.integers(region.origin_y - 70000, region.origin_y + 2 * S + 70000, n)
    # points exactly on window edges (inclusive low edge, exclusive high edge)
    cx = region.origin_x + S + S // 2
    cy = region.origin_y + S // 2
    x[:4] = [cx - H, cx + H, cx - H - 1, cx + H - 1]
    y[:4] = cy
    tile_list = [4, 1, 0, 5]  # a subset, not in id order
    off, idx = oracle_lib.bin_points(region, x, y, tile_list)
    bins = _brute_bins(region, x, y, tile_list)
    assert off[0] == 0
    for k, sel in enumerate(bins):
        assert idx[off[k]:off[k + 1]].tolist() == sel


def test_bin_multiplicity(oracle_lib):
    region = synth.Region(tiles_x=5, tiles_y=5)
    rng = np.random.default_rng(0)
    S = region.tile_size
    n = 20000
    x = rng.integers(0, 5 * S, n)
    y = rng.integers(0, 5 * S, n)
    off, idx = oracle_lib.bin_points(region, x, y, np.arange(25))
    mult = np.bincount(idx, minlength=n)
    interior = (x >= S) & (x < 4 * S) & (y >= S) & (y < 4 * S)
    assert set(np.unique(mult[interior]).tolist()) <= {1, 2, 4}
    # 160 m halo on a 640 m tile: E[mult] = (320^2 + 2*4*160*320 + 4*4*160^2)/640^2 = 2.25
    assert abs(mult[interior].mean() - 2.25) < 0.03
    assert off[-1] == mult.sum()


# ---------------------------------------------------------------- canon
def test_canon_dedupe(oracle_lib):
    rng = np.random.default_rng(1)
    u, v, z, rgb = _rand_points(rng, 400, -20, 20)  # many duplicates
    pts = oracle_lib.make_points(u, v, z, rgb)
    out = oracle_lib.canon(pts)
    best = {}
    for i in range(len(u)):
        key = (int(v[i]), int(u[i]))
        val = (int(z[i]),) + tuple(int(c) for c in rgb[i])
        if key not in best or val > best[key]:
            best[key] = val
    assert len(out) == len(best)
    for p in out:
        assert best[(int(p["v"]), int(p["u"]))] == (int(p["z"]),) + tuple(int(c) for c in p["rgb"])
    keys = [(int(p["v"]), int(p["u"])) for p in out]
    assert keys == sorted(keys)


# ---------------------------------------------------------------- NN
def _texel_centres(region):
    R, C = region.R, region.cell
    H = region.tile_size // 2 + region.pad * C
    c = -H + C // 2 + C * np.arange(R)
    qx, qy = np.meshgrid(c, c)  # qx varies along columns j, qy along rows i
    return qx, qy


@pytest.mark.parametrize("res,pad,m", [(8, 0, 30), (64, 16, 200)])
def test_nn_brute_force_and_kdtree(oracle_lib, res, pad, m):
    rng = np.random.default_rng(res)
    region = synth.Region(res=res, pad=pad, tile_size=64000)
    H = region.tile_size // 2 + pad * region.cell
    u, v, z, rgb = _rand_points(rng, m, -H, H)
    # force exact ties: a mirrored pair around a texel centre
    qx, qy = _texel_centres(region)
    u[0], v[0] = qx[0, 1] - 300, qy[0, 1]
    u[1], v[1] = qx[0, 1] + 300, qy[0, 1]
    pts = oracle_lib.make_points(u, v, z, rgb)
    out = oracle_lib.recon_tile(region, pts)
    cp = out["points"]
    P = np.stack([cp["u"], cp["v"]], 1).astype(np.int64)
    Q = np.stack([qx.ravel(), qy.ravel()], 1).astype(np.int64)
    d2 = ((Q[:, None, :] - P[None, :, :]) ** 2).sum(-1)
    # brute force: lexicographic min of (d2, v, u)
    order = np.lexsort((P[:, 0], P[:, 1]))  # by v then u
    rank = np.empty(len(P), np.int64)
    rank[order] = np.arange(len(P))
    key = d2 * len(P) + rank[None, :]
    want = key.argmin(1)
    assert np.array_equal(out["nn_idx"].ravel(), want)
    # the tie resolved to the smaller u (same v)
    assert cp[out["nn_idx"][0, 1]]["u"] == u[0]
    dist, _ = cKDTree(P.astype(np.float64)).query(Q.astype(np.float64))
    np.testing.assert_allclose(np.sqrt(d2[np.arange(len(Q)), want]), dist, rtol=1e-12)
    np.testing.assert_array_equal(out["hm_nn"].ravel(), cp["z"][want] * 0.01)


# ---------------------------------------------------------------- Delaunay
def _orient(a, b, c):
    return (int(b[0]) - int(a[0])) * (int(c[1]) - int(a[1])) - (int(b[1]) - int(a[1])) * (int(c[0]) - int(a[0]))


def _incircle(a, b, c, d):
    rows = []
    for p in (a, b, c):
        dx, dy = int(p[0]) - int(d[0]), int(p[1]) - int(d[1])
        rows.append((dx, dy, dx * dx + dy * dy))
    (a0, a1, a2), (b0, b1, b2), (c0, c1, c2) = rows
    return a0 * (b1 * c2 - b2 * c1) - a1 * (b0 * c2 - b2 * c0) + a2 * (b0 * c1 - b1 * c0)


def _certificate(P, tri, strict=True):
    """CCW, empty circumcircles, area = hull area, Euler count."""
    for a, b, c in tri:
        assert _orient(P[a], P[b], P[c]) > 0
    idx = np.arange(len(P))
    for a, b, c in tri:
        for d in idx:
            if d in (a, b, c):
                continue
            s = _incircle(P[a], P[b], P[c], P[d])
            assert s <= 0 if not strict else s < 0
    hull = ConvexHull(P.astype(np.float64))
    hv = hull.vertices
    hull2 = sum(int(P[hv[k], 0]) * int(P[hv[(k + 1) % len(hv)], 1]) -
                int(P[hv[(k + 1) % len(hv)], 0]) * int(P[hv[k], 1]) for k in range(len(hv)))
    area2 = sum(_orient(P[a], P[b], P[c]) for a, b, c in tri)
    assert area2 == abs(hull2)
    return hv


def _canon_tris(tri):
    out = set()
    for t in tri:
        k = int(np.argmin(t))
        out.add(tuple(int(t[(k + i) % 3]) for i in range(3)))
    return out


@pytest.mark.parametrize("m,seed", [(5, 0), (9, 1), (12, 2)])
def test_delaunay_brute_force_small(oracle_lib, m, seed):
    rng = np.random.default_rng(seed)
    u, v, z, rgb = _rand_points(rng, m)
    pts = oracle_lib.canon(oracle_lib.make_points(u, v, z, rgb))
    P = np.stack([pts["u"], pts["v"]], 1)
    tri = oracle_lib.delaunay(pts, seed=3)
    # definition: every CCW triple with an empty circumcircle (general position)
    want = set()
    for a, b, c in itertools.combinations(range(len(P)), 3):
        if _orient(P[a], P[b], P[c]) < 0:
            b, c = c, b
        if _orient(P[a], P[b], P[c]) == 0:
            continue
        if all(_incircle(P[a], P[b], P[c], P[d]) < 0 for d in range(len(P)) if d not in (a, b, c)):
            want.add((a, b, c))
    assert _canon_tris(tri) == _canon_tris(np.array(sorted(want)))


@pytest.mark.parametrize("m,seed", [(60, 0), (400, 1), (1500, 2)])
def test_delaunay_certificate_and_scipy(oracle_lib, m, seed):
    rng = np.random.default_rng(seed)
    u, v, z, rgb = _rand_points(rng, m)
    pts = oracle_lib.canon(oracle_lib.make_points(u, v, z, rgb))
    P = np.stack([pts["u"], pts["v"]], 1).astype(np.int64)
    tri = oracle_lib.delaunay(pts, seed=seed + 10)
    if m <= 400:
        hv = _certificate(P, tri)
        assert len(tri) == 2 * len(P) - 2 - len(hv)
    sp = Delaunay(P.astype(np.float64)).simplices
    sp = np.array([t if _orient(P[t[0]], P[t[1]], P[t[2]]) > 0 else t[[0, 2, 1]] for t in sp])
    assert _canon_tris(tri) == _canon_tris(sp)
    # insertion order does not matter
    tri2 = oracle_lib.delaunay(pts, seed=seed + 999)
    assert _canon_tris(tri) == _canon_tris(tri2)


def test_delaunay_degenerate_lattice(oracle_lib):
    rng = np.random.default_rng(5)
    g = rng.choice(400, 150, replace=False)
    u = (g % 20 - 10) * 100
    v = (g // 20 - 10) * 100
    pts = oracle_lib.canon(oracle_lib.make_points(u, v, np.zeros(150, int), np.zeros((150, 3), int)))
    P = np.stack([pts["u"], pts["v"]], 1).astype(np.int64)
    tri = oracle_lib.delaunay(pts)
    _certificate(P, tri, strict=False)


def test_delaunay_collinear_and_tiny(oracle_lib):
    u = np.arange(10) * 100
    v = 2 * u
    pts = oracle_lib.canon(oracle_lib.make_points(u, v, np.zeros(10, int), np.zeros((10, 3), int)))
    assert len(oracle_lib.delaunay(pts)) == 0
    assert len(oracle_lib.delaunay(pts[:2])) == 0


# ---------------------------------------------------------------- interpolation
def test_planar_reproduction(oracle_lib):
    """A planar height field is reproduced exactly at every hull texel."""
    region = synth.Region()
    rng = np.random.default_rng(7)
    H = 48000
    g = rng.choice(960 * 960, 3000, replace=False)
    u = (g % 960) * 100 - H
    v = (g // 960) * 100 - H
    # the window's extreme lattice corners: the hull then covers every texel centre
    u = np.concatenate([u, [-H, H - 100, -H, H - 100]])
    v = np.concatenate([v, [-H, -H, H - 100, H - 100]])
    z = (3 * u - 2 * v) // 100 + 500
    pts = oracle_lib.make_points(u, v, z, np.zeros((len(u), 3), int))
    out = oracle_lib.recon_tile(region, pts)
    assert out["inside"].all()
    qx, qy = _texel_centres(region)
    plane = ((3 * qx - 2 * qy) / 100 + 500) * 0.01
    np.testing.assert_allclose(out["hm_lin"], plane, atol=1e-9)


def test_constant_field(oracle_lib):
    region = synth.Region()
    rng = np.random.default_rng(8)
    u, v, _, rgb = _rand_points(rng, 300)
    z = np.full(300, 1234)
    out = oracle_lib.recon_tile(region, oracle_lib.make_points(u, v, z, rgb))
    # barycentric weights sum to one up to FP64 rounding
    np.testing.assert_allclose(out["hm_lin"], 12.34, rtol=0, atol=1e-12)
    assert np.all(out["hm_nn"] == 12.34)
    assert abs(out["cz"] - 12.34) < 1e-12
    assert np.abs(out["x"][..., :2]).max() < 1e-14


def test_linear_matches_scipy(oracle_lib):
    region = synth.Region()
    rng = np.random.default_rng(9)
    u, v, z, rgb = _rand_points(rng, 500, -40000, 40000)
    out = oracle_lib.recon_tile(region, oracle_lib.make_points(u, v, z, rgb))
    cp = out["points"]
    P = np.stack([cp["u"], cp["v"]], 1).astype(np.float64)
    qx, qy = _texel_centres(region)
    f = LinearNDInterpolator(P, cp["z"] * 0.01)
    ref = f(qx.astype(np.float64), qy.astype(np.float64))
    inside = ~np.isnan(ref)
    assert np.array_equal(inside, out["inside"])
    np.testing.assert_allclose(out["hm_lin"][inside], ref[inside], atol=1e-9)
    np.testing.assert_array_equal(out["hm_lin"][~inside], out["hm_nn"][~inside])
    for c in range(3):
        fc = LinearNDInterpolator(P, cp["rgb"][:, c].astype(np.float64))
        rc = fc(qx.astype(np.float64), qy.astype(np.float64))
        np.testing.assert_allclose(out["x"][..., 2 + c][inside] * 65535, rc[inside], atol=1e-6)


def test_normalisation_closed_form_and_shift(oracle_lib):
    region = synth.Region()
    rng = np.random.default_rng(10)
    u, v, z, rgb = _rand_points(rng, 300)
    a = oracle_lib.recon_tile(region, oracle_lib.make_points(u, v, z, rgb))
    b = oracle_lib.recon_tile(region, oracle_lib.make_points(u, v, z + 77777, rgb))
    R = region.R
    assert a["cz"] == a["hm_lin"][R // 2, R // 2]
    np.testing.assert_allclose(a["x"][..., 0], (a["hm_lin"] - a["cz"]) / 480.0, rtol=0, atol=1e-15)
    np.testing.assert_allclose(a["x"][..., 1], (a["hm_nn"] - a["cz"]) / 480.0, rtol=0, atol=1e-15)
    assert abs(b["cz"] - a["cz"] - 777.77) < 1e-9
    np.testing.assert_allclose(b["x"], a["x"], atol=1e-12)


def test_empty_and_nn_only_tiles(oracle_lib):
    region = synth.Region()
    e = oracle_lib.recon_tile(region, oracle_lib.make_points([], [], [], np.zeros((0, 3))))
    assert e["status"] == oracle_lib.ORA_EMPTY and np.all(e["x"] == 0) and e["cz"] == 0
    two = oracle_lib.recon_tile(region, oracle_lib.make_points([0, 5000], [0, 100], [100, 200], np.ones((2, 3))))
    assert two["status"] == oracle_lib.ORA_NN_ONLY
    assert np.array_equal(two["hm_lin"], two["hm_nn"])
    col = oracle_lib.recon_tile(region, oracle_lib.make_points([0, 100, 200], [0, 100, 200], [1, 2, 3],
                                                               np.ones((3, 3))))
    assert col["status"] == oracle_lib.ORA_NN_ONLY


def _load_golden(name):
    rows = []
    with open(os.path.join(HERE, "golden", name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append(line.split())
    return rows


def test_golden_three_point_tile(oracle_lib):
    """Hand-derived values for a three-point tile (golden/three_point_tile.txt)."""
    rows = _load_golden("three_point_tile.txt")
    pts = [r[1:] for r in rows if r[0] == "point"]
    u = [int(p[0]) for p in pts]
    v = [int(p[1]) for p in pts]
    z = [int(p[2]) for p in pts]
    rgb = [[int(c) for c in p[3:6]] for p in pts]
    region = synth.Region()
    out = oracle_lib.recon_tile(region, oracle_lib.make_points(u, v, z, rgb))
    for r in rows:
        if r[0] == "cz":
            assert abs(out["cz"] - float(r[1])) < 1e-12
        elif r[0] == "texel":
            i, j = int(r[1]), int(r[2])
            assert abs(out["hm_lin"][i, j] - float(r[3])) < 1e-12
            assert abs(out["hm_nn"][i, j] - float(r[4])) < 1e-12
            assert bool(out["inside"][i, j]) == (r[5] == "inside")


def test_golden_three_point_texture(oracle_lib):
    """Texture of the three-point tile through the all-zero network, and the
    colour clamp, against hand-derived values (golden/three_point_texture.txt):
    pins oracle.texture (h = c_z + r y_h, colour clamp) and the network's
    residual on the crop."""
    rows = _load_golden("three_point_tile.txt")
    pts = [r[1:] for r in rows if r[0] == "point"]
    region = synth.Region()
    out = oracle_lib.recon_tile(region, oracle_lib.make_points(
        [int(p[0]) for p in pts], [int(p[1]) for p in pts], [int(p[2]) for p in pts],
        [[int(c) for c in p[3:6]] for p in pts]))
    w0 = np.zeros(oracle_lib.num_params())
    y = oracle_lib.unet_forward(w0, out["x"][None], region.res, region.pad)
    tex = oracle_lib.texture(y, np.array([out["cz"]]), region)[0]
    gold = _load_golden("three_point_texture.txt")
    n = 0
    for r in gold:
        if r[0] == "ctexel":
            i, j = int(r[1]), int(r[2])
            want = [float(v) for v in r[3:7]]
            np.testing.assert_allclose(tex[i, j], want, rtol=0, atol=1e-12)
            n += 1
        elif r[0] == "clamp":
            yv = np.array([float(v) for v in r[1:5]]).reshape(1, 1, 1, 4)
            got = oracle_lib.texture(yv, np.array([20.25]), region)[0, 0, 0]
            np.testing.assert_allclose(got, [float(v) for v in r[5:9]], rtol=0, atol=1e-12)
            n += 1
    assert n == 8


def test_recon_tiles_equals_per_tile_composition(oracle_lib):
    """The batch driver = binning, gather to tile-local coordinates and
    Algorithm 1 per listed tile, on a region with tiles_x != tiles_y, a
    non-zero origin and a tile list out of id order.  Tile centres come from
    the tiling's definition (tile (tx, ty) covers [origin + t S, origin +
    (t + 1) S) per axis, linear id ty * tiles_x + tx), enumerated row by row."""
    rng = np.random.default_rng(21)
    region = synth.Region(origin_x=-12345, origin_y=777, tiles_x=3, tiles_y=2)
    S = region.tile_size
    H = S // 2 + region.pad * region.cell
    n = 1500
    x = rng.integers(region.origin_x - 20000, region.origin_x + 3 * S + 20000, n)
    y = rng.integers(region.origin_y - 20000, region.origin_y + 2 * S + 20000, n)
    z = rng.integers(-3000, 3000, n)
    rgb = rng.integers(0, 65536, (n, 3))
    tile_list = np.array([5, 0, 3, 1], np.int32)
    xo, cz, st = oracle_lib.recon_tiles(region, x, y, z, rgb, tile_list)
    centres = []
    for ty in range(region.tiles_y):
        for tx in range(region.tiles_x):
            lo_x, lo_y = region.origin_x + tx * S, region.origin_y + ty * S
            centres.append((lo_x + S // 2, lo_y + S // 2))
    for k, t in enumerate(tile_list):
        cx, cy = centres[t]
        sel = [i for i in range(n) if cx - H <= x[i] < cx + H and cy - H <= y[i] < cy + H]
        ref = oracle_lib.recon_tile(region, oracle_lib.make_points(x[sel] - cx, y[sel] - cy, z[sel], rgb[sel]))
        np.testing.assert_allclose(xo[k], ref["x"], rtol=0, atol=1e-12)
        assert abs(cz[k] - ref["cz"]) <= 1e-12 and st[k] == ref["status"]


def test_recon_tiles_plane_in_region_coordinates(oracle_lib):
    """A plane in region coordinates, z = (3x - 2y)/100 + 500 raw, sampled on
    the 100 cm lattice (plus every window's corner lattice points, so each
    hull covers all texel centres), is reproduced by the batch driver at every
    texel of every listed tile at the texel centre's region coordinates:
    pins the tile centres and axes of the batch driver by a closed form."""
    rng = np.random.default_rng(22)
    region = synth.Region(origin_x=-12300, origin_y=700, tiles_x=3, tiles_y=2)
    S = region.tile_size
    H = S // 2 + region.pad * region.cell
    x0, y0 = region.origin_x - H, region.origin_y - H
    nx, ny = (3 * S + 2 * H) // 100, (2 * S + 2 * H) // 100
    g = rng.choice(nx * ny, 40000, replace=False)
    x = x0 + (g % nx) * 100
    y = y0 + (g // nx) * 100
    tile_list = np.array([4, 2, 0], np.int32)
    cx_all, cy_all = [], []
    for t in tile_list:
        cx = region.origin_x + (t % 3) * S + S // 2
        cy = region.origin_y + (t // 3) * S + S // 2
        lo_x, hi_x = cx - H, cx + H - 100  # lattice points: region origin offsets are multiples of 100
        lo_y, hi_y = cy - H, cy + H - 100
        cx_all += [lo_x, hi_x, lo_x, hi_x]
        cy_all += [lo_y, lo_y, hi_y, hi_y]
    x = np.concatenate([x, cx_all])
    y = np.concatenate([y, cy_all])
    assert np.all((x - x0) % 100 == 0) and np.all((y - y0) % 100 == 0)
    z = (3 * x - 2 * y) // 100 + 500
    assert np.all((3 * x - 2 * y) % 100 == 0)
    xo, cz, st = oracle_lib.recon_tiles(region, x, y, z, np.zeros((len(x), 3), int), tile_list)
    c = -H + region.cell // 2 + region.cell * np.arange(region.R)
    for k, t in enumerate(tile_list):
        cx = region.origin_x + (t % 3) * S + S // 2
        cy = region.origin_y + (t // 3) * S + S // 2
        qx, qy = np.meshgrid(cx + c, cy + c)
        plane = ((3 * qx - 2 * qy) / 100 + 500) * 0.01
        h = xo[k, ..., 0] * 480.0 + cz[k]
        np.testing.assert_allclose(h, plane, rtol=0, atol=1e-9)
        assert st[k] == 0


def test_cocircular_lattice_interpolation_valid(oracle_lib):
    """Lattice points with random heights (exactly cocircular squares, whose
    two diagonals give different heights; texels sit on the diagonals): the
    oracle's linear map comes from a valid Delaunay triangulation at every
    texel, and the test is not vacuous (many texels have two admissible
    values)."""
    from delaunay_check import check_linear_valid, lattice_points

    region = synth.Region()
    rng = np.random.default_rng(31)
    u, v, z = lattice_points(rng)
    out = oracle_lib.recon_tile(region, oracle_lib.make_points(u, v, z, np.zeros((len(u), 3), int)))
    cp = out["points"]
    qx, qy = _texel_centres(region)
    n, amb = check_linear_valid(np.stack([cp["u"], cp["v"]], 1), cp["z"] * 0.01, qx, qy, out["hm_lin"],
                                out["hm_nn"], 1e-9)
    assert amb > 100, amb
