"""GPU parity: binning CSR (bit-exact), nearest-neighbour maps (exact) and
Delaunay-linear maps (<= 1e-4 m) of ls_recon_tiles against the FP64 oracle
(Algorithm 1 and the Section 3.4 normalisation)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2509_20198_amd as ls
import synth
from gpu_helpers import R_M, arrays_to_dev, points_to_dev

pytestmark = pytest.mark.gpu

TOL_M = 1e-4


def _gpu_recon(region, ps_np, tile_list, want_csr=True, order=ls.ORDER_LIST):
    g = ls.Grid.of(region)
    xt, yt, zt, rt = arrays_to_dev(*ps_np)
    tl = torch.from_numpy(np.ascontiguousarray(tile_list, np.int32)).cuda()
    nt = len(tile_list)
    if want_csr:
        off = torch.empty(nt + 1, dtype=torch.int32, device="cuda")
        idx = torch.empty(max(4 * len(ps_np[0]), 1), dtype=torch.int32, device="cuda")
        xo, cz, st = ls.recon_tiles(g, xt, yt, zt, rt, tl, order=order, bin_off=off, bin_idx=idx)
    else:
        off = idx = None
        xo, cz, st = ls.recon_tiles(g, xt, yt, zt, rt, tl, order=order)
    torch.cuda.synchronize()
    out = dict(x=xo.cpu().numpy().astype(np.float64), cz=cz.cpu().numpy(), status=st.cpu().numpy())
    if want_csr:
        o = off.cpu().numpy()
        out["off"] = o
        out["idx"] = idx.cpu().numpy()[: o[-1]]
    return out


def _compare(region, ps_np, tile_list, gpu=None):
    x, y, z, rgb = ps_np
    xo, cz, st = oracle.recon_tiles(region, x, y, z, rgb, tile_list)
    gpu = gpu or _gpu_recon(region, ps_np, tile_list)
    off, idx = oracle.bin_points(region, x, y, tile_list)
    if "off" in gpu:
        assert np.array_equal(gpu["off"], off)
        assert np.array_equal(gpu["idx"], idx)
    r = (region.tile_size / 2 + region.pad * region.cell) * region.scale_xy  # padded half side, metres
    np.testing.assert_allclose(gpu["cz"], cz, rtol=0, atol=1e-9)
    # heights in metres: linear within 1e-4 m, nearest neighbour exact up to FP32 rounding of x
    err_lin = np.abs(gpu["x"][..., 0] - xo[..., 0]).max() * r
    err_nn = np.abs(gpu["x"][..., 1] - xo[..., 1]).max() * r
    assert err_lin <= TOL_M, err_lin
    assert err_nn <= 1e-6 * max(1.0, np.abs(xo[..., 1]).max() * r), err_nn
    # colours: NN exact (integer colour), linear within 1e-5 of [0, 1]
    assert np.array_equal(np.rint(gpu["x"][..., 5:8] * 65535), np.rint(xo[..., 5:8] * 65535))
    assert np.abs(gpu["x"][..., 2:5] - xo[..., 2:5]).max() <= 1e-5
    assert np.array_equal(gpu["status"] & 3, st)
    return gpu, (xo, cz, st)


def test_single_tile_400():
    w = synth.single_tile(seed=1, n=400)
    _compare(w.region, w.points.numpy(), w.tile_list)


@pytest.mark.parametrize("seed", [2, 3])
def test_batch_6x6_loguniform(seed):
    w = synth.batch_tiles(seed=seed, tiles_x=6, tiles_y=6)
    _compare(w.region, w.points.numpy(), w.tile_list)


def test_subset_tile_list_and_pad0():
    w = synth.batch_tiles(seed=4, tiles_x=5, tiles_y=4, pad=0)
    tl = np.array([7, 3, 19, 0, 12], np.int32)
    _compare(w.region, w.points.numpy(), tl)


@pytest.mark.parametrize("n", [9000, 16000])
def test_dense_tile_points_outside_lds(n):
    """Windows too dense for the canonical points to fit in LDS (they stay in
    global memory) and bucket grids near their maximum side."""
    w = synth.single_tile(seed=n, n=n)
    _compare(w.region, w.points.numpy(), w.tile_list)


def test_pareto_counts_small_tiles():
    counts = synth.counts_pareto(6, 64)
    w = synth.sparse_workload("pareto", 8, 8, counts, 6, order="id")
    _compare(w.region, w.points.numpy(), w.tile_list)


def test_edge_cases_empty_nn_only_duplicates():
    region = synth.Region(tiles_x=4, tiles_y=1)
    S = 64000
    # tile 0: empty window (no points near), tile 1: 1 point, tile 2: 2 points + collinear triple nearby
    # tile 3: duplicates (same xy, different z/colour)
    xs = [S + 32000, 2 * S + 100, 2 * S + 900, 2 * S + 1700, 3 * S + 5000, 3 * S + 5000, 3 * S + 5000,
          3 * S + 20000, 3 * S + 40000]
    ys = [32000, 10000, 10800, 11600, 30000, 30000, 30000, 50000, 12345]
    zs = [100, 200, 300, 400, 500, 700, 700, 800, 900]
    rgb = np.array([[1, 2, 3]] * 5 + [[9, 9, 9], [9, 9, 10], [4, 4, 4], [5, 5, 5]], np.uint16) * 257
    # move tile 1's point so tile 0's window (reaching 160 m into tile 1) stays empty
    xs[0] = S + 40000
    ps = (np.array(xs, np.int32), np.array(ys, np.int32), np.array(zs, np.int32), rgb)
    gpu, (xo, cz, st) = _compare(region, ps, np.arange(4, dtype=np.int32))
    assert st[0] == oracle.ORA_EMPTY and (gpu["status"][0] & ls.TILE_EMPTY)
    assert np.all(gpu["x"][0] == 0)


def test_bad_and_duplicate_tile_ids():
    w = synth.batch_tiles(seed=9, tiles_x=3, tiles_y=3)
    tl = np.array([4, 4, 99, 1], np.int32)
    gpu = _gpu_recon(w.region, w.points.numpy(), tl, want_csr=False)
    assert gpu["status"][1] & ls.TILE_BADID and gpu["status"][2] & ls.TILE_BADID
    assert not gpu["status"][0] & ls.TILE_BADID and not gpu["status"][3] & ls.TILE_BADID
    assert np.all(gpu["x"][1] == 0) and np.all(gpu["x"][2] == 0)
    xo, cz, st = oracle.recon_tiles(w.region, *w.points.numpy(), np.array([4, 1], np.int32))
    assert np.abs(gpu["x"][[0, 3]] - xo).max() * R_M <= TOL_M


def test_cap_too_small_flags_every_tile():
    w = synth.batch_tiles(seed=10, tiles_x=2, tiles_y=2)
    g = ls.Grid.of(w.region)
    xt, yt, zt, rt = points_to_dev(w.points)
    tl = torch.from_numpy(w.tile_list).cuda()
    off = torch.empty(5, dtype=torch.int32, device="cuda")
    idx = torch.empty(10, dtype=torch.int32, device="cuda")
    xo, cz, st = ls.recon_tiles(g, xt, yt, zt, rt, tl, bin_off=off, bin_idx=idx)
    torch.cuda.synchronize()
    o, _ = oracle.bin_points(w.region, *w.points.numpy()[:2], w.tile_list)
    assert int(off[-1].item()) == o[-1]
    assert np.all(st.cpu().numpy() & ls.TILE_CAP)


def test_planar_reproduction_lattice():
    """Cocircular lattice points: every triangulation reproduces a plane."""
    region = synth.Region()
    rng = np.random.default_rng(7)
    H = 48000
    gsel = rng.choice(960 * 960, 3000, replace=False)
    u = np.concatenate([(gsel % 960) * 100 - H, [-H, H - 100, -H, H - 100]])
    v = np.concatenate([(gsel // 960) * 100 - H, [-H, -H, H - 100, H - 100]])
    z = (3 * u - 2 * v) // 100 + 500
    ps = ((u + 32000).astype(np.int32), (v + 32000).astype(np.int32), z.astype(np.int32),
          np.zeros((len(u), 3), np.uint16))
    gpu = _gpu_recon(region, ps, np.zeros(1, np.int32), want_csr=False)
    c = -H + 500 + 1000 * np.arange(96)
    qx, qy = np.meshgrid(c, c)
    plane = ((3 * qx - 2 * qy) / 100 + 500) * 0.01
    h = gpu["x"][0, ..., 0] * R_M + gpu["cz"][0]
    assert np.abs(h - plane).max() <= TOL_M
    assert gpu["status"][0] == 0


def _window_points(u, v, rng):
    z = rng.integers(0, 5000, len(u)).astype(np.int32)
    rgb = rng.integers(0, 65536, (len(u), 3)).astype(np.uint16)
    return ((np.asarray(u) + 32000).astype(np.int32), (np.asarray(v) + 32000).astype(np.int32), z, rgb)


@pytest.mark.parametrize("n", [40, 900])
def test_points_on_window_boundary_lines(n):
    """Points on the four edges and corners of the window: hull edges lie on
    the window boundary, where the neighbour search region is a thin strip."""
    region = synth.Region()
    rng = np.random.default_rng(n)
    H = 48000
    side = rng.integers(0, 5, n)
    t, s = rng.integers(-H, H, n), rng.integers(-H, H, n)
    u = np.select([side == 0, side == 1], [-H, H - 1], t)
    v = np.select([side == 2, side == 3], [-H, H - 1], s)
    u = np.concatenate([u, [-H, H - 1, -H, H - 1]])
    v = np.concatenate([v, [-H, -H, H - 1, H - 1]])
    _compare(region, _window_points(u, v, rng), np.zeros(1, np.int32))


def test_near_collinear_band():
    """Points in a narrow band along a line: circumcircles of neighbouring
    triples are huge and the left-side caps thin."""
    region = synth.Region()
    rng = np.random.default_rng(3)
    H = 48000
    u = rng.integers(-H, H, 700)
    v = np.clip((u * 3) // 7 + rng.integers(0, 3, 700), -H, H - 1)
    extra_u, extra_v = rng.integers(-H, H, 30), rng.integers(-H, H, 30)
    _compare(region, _window_points(np.concatenate([u, extra_u]), np.concatenate([v, extra_v]), rng),
             np.zeros(1, np.int32))


@pytest.mark.parametrize("k", [16, 30, 48])
def test_high_degree_wheels(k):
    """Hubs ringed by k points on a circle: each hub has k Delaunay
    neighbours (more than a star successor list holds) and the ring points
    are nearly cocircular, so recorded and searched steps mix with the exact
    fallbacks of the predicates."""
    region = synth.Region()
    rng = np.random.default_rng(k)
    H = 48000
    hubs = rng.integers(-H + 8000, H - 8000, (5, 2))
    u, v = [], []
    for hx, hy in hubs:
        r = int(rng.integers(2000, 5000))
        t = 2 * np.pi * (np.arange(k) + rng.uniform(0, 1)) / k
        u += [hx] + list(np.rint(hx + r * np.cos(t)).astype(np.int64))
        v += [hy] + list(np.rint(hy + r * np.sin(t)).astype(np.int64))
    bu, bv = rng.integers(-H, H, 600), rng.integers(-H, H, 600)
    far = np.min(np.hypot(bu[:, None] - hubs[None, :, 0], bv[:, None] - hubs[None, :, 1]), axis=1) > 7500
    u = np.concatenate([u, bu[far], [-H, H - 1, -H, H - 1]])
    v = np.concatenate([v, bv[far], [-H, -H, H - 1, H - 1]])
    _compare(region, _window_points(u, v, rng), np.zeros(1, np.int32))


def test_deterministic_and_order_independent():
    w = synth.batch_tiles(seed=11, tiles_x=4, tiles_y=4)
    ps = w.points.numpy()
    a = _gpu_recon(w.region, ps, w.tile_list)
    b = _gpu_recon(w.region, ps, w.tile_list)
    perm = np.random.default_rng(0).permutation(len(ps[0]))
    c = _gpu_recon(w.region, tuple(p[perm] for p in ps), w.tile_list, want_csr=False)
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["idx"], b["idx"])
    assert np.array_equal(a["x"], c["x"])


def test_full_batch_1024_sampled():
    """The 1024-tile batch in the launch configuration the benchmark uses;
    the oracle checks a sample of tiles one by one."""
    w = synth.batch_tiles(seed=2)
    ps = w.points.numpy()
    gpu = _gpu_recon(w.region, ps, w.tile_list, want_csr=False)
    rng = np.random.default_rng(1)
    ks = np.concatenate([[0, 1, len(w.tile_list) - 1], rng.choice(len(w.tile_list), 9, replace=False)])
    xo, cz, st = oracle.recon_tiles(w.region, *ps, w.tile_list[ks])
    assert np.abs(gpu["x"][ks][..., 0] - xo[..., 0]).max() * R_M <= TOL_M
    assert np.abs(gpu["x"][ks][..., 1] - xo[..., 1]).max() * R_M <= 1e-5
    np.testing.assert_allclose(gpu["cz"][ks], cz, atol=1e-9)
    assert np.all(gpu["status"] == 0)


def test_viewpoint_priority_order():
    """Tiles listed by distance to a viewpoint (Pareto counts as in the
    streaming workload) processed in list order: identical bits to the
    longest-first order, CSR and maps equal to the oracle on every tile."""
    w = synth.stream_tiles(seed=12, tiles_x=12, tiles_y=10)
    ps = w.points.numpy()
    a = _gpu_recon(w.region, ps, w.tile_list, order=ls.ORDER_LIST)
    b = _gpu_recon(w.region, ps, w.tile_list, order=ls.ORDER_LONGEST_FIRST)
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["cz"], b["cz"])
    assert np.array_equal(a["status"], b["status"]) and np.array_equal(a["idx"], b["idx"])
    _compare(w.region, ps, w.tile_list, gpu=a)


def test_cocircular_lattice_with_relief():
    """Lattice points with random heights: many exactly cocircular squares
    whose two diagonals give different heights, texel centres on the
    diagonals.  The GPU's symbolic perturbation picks one triangulation; its
    linear map must come from a valid Delaunay triangulation at every texel
    (several are correct), and its nearest-neighbour map (unique) must equal
    the oracle's."""
    from delaunay_check import check_linear_valid, lattice_points

    region = synth.Region()
    rng = np.random.default_rng(31)
    u, v, z = lattice_points(rng)
    ps = ((u + 32000).astype(np.int32), (v + 32000).astype(np.int32), z.astype(np.int32),
          np.zeros((len(u), 3), np.uint16))
    gpu = _gpu_recon(region, ps, np.zeros(1, np.int32), want_csr=False)
    xo, cz, st = oracle.recon_tiles(region, *ps, np.zeros(1, np.int32))
    assert np.abs(gpu["x"][0, ..., 1] - xo[0, ..., 1]).max() * R_M <= 1e-5
    H = 48000
    c = -H + 500 + 1000 * np.arange(96)
    qx, qy = np.meshgrid(c, c)
    h_lin = gpu["x"][0, ..., 0] * R_M + gpu["cz"][0]
    h_nn = gpu["x"][0, ..., 1] * R_M + gpu["cz"][0]
    n, amb = check_linear_valid(np.stack([u, v], 1), z * 0.01, qx, qy, h_lin, h_nn, TOL_M)
    print(f"lattice: {amb} of {n} texels had two admissible values")
    assert amb > 100
