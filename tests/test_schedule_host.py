"""The library's host schedule (C++, sk_schedule) equals the oracle's
simulator bit for bit (CPU only).  The simulator is given the launch
parameters the library resolved (workgroups, split point, tile order,
problem order, dealing rule) and derives every segment itself."""
import random

import pytest
import torch

import paper_2407_00044_amd as sk
from oracle import schedule as sch
from paper_2407_00044_amd import synth

BK = {torch.float32: 32, torch.float16: 64, torch.bfloat16: 64, torch.float8_e4m3fn: 128}


def compare(shapes, dtype, tile, g, mode, dp_tiles=-1, group_m=0, min_iters=0):
    cfg = sk.Config(tile=tile, mode=mode, num_cu=g, dp_tiles=dp_tiles, group_m=group_m,
                    min_iters=min_iters)
    lib_segs = sk.schedule(shapes, dtype, cfg)
    lp = sk.launch_params(shapes, dtype, cfg)
    plan, sim = sch.simulate(shapes, tile[0], tile[1], BK[dtype], **lp)
    assert lib_segs == [s.as_tuple() for s in sim]
    sch.check(shapes, tile[0], tile[1], BK[dtype], plan.g, sim, order=lp["order"],
              dp_grid=lp["dp_grid"], deal=lp["deal"])
    # the report's decompositions: S as the oracle reads them
    if mode in ("sk", "hybrid", "dp") and lp["g"] == g:
        T = len(sch.tile_grid(shapes, tile[0], tile[1], BK[dtype]))
        want = {"sk": sch.MODE_SK, "hybrid": sch.MODE_HYBRID, "dp": sch.MODE_DP}[mode]
        assert lp["S"] == sch.split_for_mode(T, g, want, dp_tiles)


@pytest.mark.parametrize("mode", ["sk", "hybrid", "dp", "auto"])
def test_random_small_shapes(mode):
    r = random.Random(7)
    sizes = [1, 5, 31, 32, 33, 64, 127, 128, 129, 200, 255, 256, 257, 300]
    tiles = {torch.float32: [(128, 128)], torch.bfloat16: [(128, 128), (256, 128), (256, 256)],
             torch.float8_e4m3fn: [(64, 128), (128, 128)]}
    for _ in range(150):
        dt = r.choice(list(tiles))
        shape = (r.choice(sizes), r.choice(sizes), r.choice(sizes + [0, 1000]))
        g = r.choice([1, 2, 3, 7, 8, 16, 64, 120, 255, 256])
        dp = r.choice([-1, -1, 0, 3]) if mode != "dp" else -1
        gm = r.choice([0, -1, -1, 2, 5])
        compare([shape], dt, r.choice(tiles[dt]), g, mode, dp, gm, r.choice([0, 0, 1, 3, 40]))


def test_paper_configurations():
    compare([(512, 512, 512)], torch.float32, (128, 128), 256, "sk")
    compare([(3840, 4096, 4096)], torch.float16, (256, 128), 256, "hybrid")
    compare([(3840, 4096, 4096)], torch.bfloat16, (256, 256), 256, "hybrid")
    compare([(3840, 4096, 4096)], torch.float16, (256, 128), 256, "dp")
    compare([(480, 512, 512)], torch.float16, (256, 128), 120, "sk")
    compare([(1920, 2000, 2000)], torch.float16, (256, 128), 120, "hybrid")
    for M, N, K in [(8192, 11008, 4096), (8192, 4096, 11008), (11008, 4096, 8192)]:
        compare([(M, N, K)], torch.bfloat16, (256, 128), 256, "hybrid")


def test_sweep_shapes():
    for M, N, K in synth.sweep_shapes()[:24]:
        compare([(M, N, K)], torch.bfloat16, (256, 128), 256, "hybrid")
        compare([(M, N, K)], torch.bfloat16, (128, 128), 256, "hybrid", group_m=-1)
        compare([(M, N, K)], torch.bfloat16, (128, 128), 256, "auto", group_m=-1)


def test_auto_decisions_on_sweep_shapes_every_type():
    # the split / no-split decisions the sweeps measure: every shape, every
    # input type, on the default tile and the full grid
    for dt in BK:
        for M, N, K in synth.sweep_shapes():
            tile = sk.default_tile(M, N, K, dt)
            compare([(M, N, K)], dt, tile, 256, "auto", group_m=-1)


def test_grouped_sets():
    shapes = synth.grouped_shapes()
    for tile in [(128, 128), (64, 128), (256, 128)]:
        for mode in ["sk", "hybrid", "dp", "auto"]:
            compare(shapes, torch.float8_e4m3fn, tile, 256, mode)
    r = random.Random(3)
    for _ in range(40):
        shapes = [(r.choice([0, 16, 100, 300]), r.choice([0, 64, 129, 500]),
                   r.choice([0, 64, 1000])) for _ in range(r.randint(1, 7))]
        compare(shapes, torch.bfloat16, (128, 128), r.choice([4, 64, 256]),
                r.choice(["sk", "hybrid", "dp"]))
