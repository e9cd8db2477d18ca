"""The library's launch policy against hand-worked values (CPU only).

The schedule simulator in oracle/ takes a launch's resolved parameters as
inputs.  How the library resolves them is its own policy, measured on MI355X
rather than taken from the report, and is pinned here by values worked out by
hand from the rules the header states:

* grid floor (min_iters): g' = min(g, max(1, W_all // m)), automatic
  m = ceil(I_mean / c), c the largest integer >= 1 with f c^2 <= I_mean,
  f = max(4, BM*BN/8192) MAC iterations per partial tile for 16-bit and e4m3
  iterations, max(1, BM*BN/32768) for FP32 iterations;
* SK_MODE_AUTO: no split when b + ceil(b/4) + f >= ceil(T/g') * I_mean
  (FP32: b + f), b = ceil(W_all/g'), the left side taken 9/8 times when the
  data-parallel launch is one partial wave on an unshrunk grid; with nothing
  split on one problem the launch is the data-parallel grid;
* automatic tile order (group_m = -1): with Stream-K tiles, bands of the
  largest divisor of q/gcd(q, I) not above the tile rows; otherwise 8;
* grouped launches: problems by iterations per tile, largest first (the
  data-parallel grid keeps the caller's order).
"""
import random

import torch

import paper_2407_00044_amd as sk

F32, F16, BF16, E4 = torch.float32, torch.float16, torch.bfloat16, torch.float8_e4m3fn


def P(shapes, dtype, tile, g, mode, **kw):
    if isinstance(shapes, tuple):
        shapes = [shapes]
    return sk.plan(shapes, dtype, sk.Config(tile=tile, mode=mode, num_cu=g, **kw))


def t(p, *keys):
    return tuple(p[k] for k in keys)


def test_grid_floor_hand_values():
    # 607x187x3155 on 256x128x64: 3x2 = 6 tiles of 50 iterations, W_all =
    # 300; f = 4, c = 3 (4*9 <= 50 < 4*16), m = ceil(50/3) = 17, so the grid
    # shrinks from 256 to 300 // 17 = 17 workgroups: 300 = 17*17 + 11
    p = P((607, 187, 3155), BF16, (256, 128), 256, "hybrid", min_iters=0)
    assert t(p, "T", "g", "S", "W", "q", "rho") == (6, 17, 6, 300, 17, 11)
    # m = 1 keeps the grid: 300 iterations over 256 workgroups
    p = P((607, 187, 3155), BF16, (256, 128), 256, "hybrid", min_iters=1)
    assert t(p, "g", "q", "rho") == (256, 1, 44)
    # 256x256 tiles (f = 8) at 3840x4096x4096: c = 2 (8*4 <= 64 < 8*9),
    # m = 32, 15360 // 32 = 480 > 256: the grid stays
    p = P((3840, 4096, 4096), BF16, (256, 256), 256, "sk", min_iters=0)
    assert t(p, "T", "g", "W", "q") == (240, 256, 15360, 60)
    # explicit m; a floor above W_all leaves one workgroup; DP ignores it
    p = P((512, 512, 512), F32, (128, 128), 256, "sk", min_iters=40)
    assert t(p, "g", "q", "rho") == (6, 42, 4)           # 256 iterations // 40
    p = P((100, 100, 100), F32, (128, 128), 256, "sk", min_iters=9)
    assert t(p, "g", "q") == (1, 4)
    p = P((512, 512, 512), F32, (128, 128), 256, "dp", min_iters=40)
    assert p["g"] == 16
    # the floor feeds the hybrid rule: 20 tiles x 8 iterations are too short
    # to split (c = 1, m = 8) -> g' = 160 // 8 = 20 = T -> S = 0
    p = P((20 * 128, 128, 8 * 64), BF16, (128, 128), 256, "hybrid", min_iters=0)
    assert t(p, "T", "g", "S", "W") == (20, 20, 0, 0)
    # 20 tiles x 64 iterations: c = 4, m = 16 -> g' = 80; S = min(20, 100)
    p = P((20 * 128, 128, 64 * 64), BF16, (128, 128), 256, "hybrid", min_iters=0)
    assert t(p, "g", "S", "q", "rho") == (80, 20, 16, 0)
    # FP32 512^3 on 128x128x32: 16 tiles of 16 iterations; f = 1, c = 4,
    # m = 4, g' = 64: every tile in 4 pieces of 4 iterations
    p = P((512, 512, 512), F32, (128, 128), 256, "sk", min_iters=0)
    assert t(p, "g", "q", "rho") == (64, 4, 0)


def test_grid_floor_properties():
    rng = random.Random(77)
    sizes = [1, 7, 64, 65, 127, 129, 200, 257, 1000, 3000]
    for _ in range(300):
        shape = (rng.choice(sizes), rng.choice(sizes), rng.choice(sizes + [0]))
        dt, tile = rng.choice([(F32, (128, 128)), (BF16, (256, 128)), (BF16, (128, 128)),
                               (E4, (64, 128))])
        g = rng.choice([1, 2, 3, 7, 16, 64, 120, 256])
        m = rng.choice([0, 3, 50])
        p = P(shape, dt, tile, g, rng.choice(["sk", "hybrid"]), min_iters=m)
        assert 1 <= p["g"] <= g
        if m > 1 and p["g"] not in (g, 1):
            # an explicit floor leaves every workgroup at least m iterations
            assert p["T"] * p["max_iters"] // p["g"] >= m


def test_auto_tile_order_hand_values():
    # q = 120, I = 64: D = 120 / 8 = 15 <= 15 tile rows -> bands of 15
    assert P((3840, 4096, 4096), F16, (256, 128), 256, "hybrid")["group_m"] == 15
    # 256x256 tiles: q = 60, gcd(60, 64) = 4 -> D = 15
    assert P((3840, 4096, 4096), BF16, (256, 256), 256, "sk")["group_m"] == 15
    # no Stream-K tiles: bands of 8 rows
    assert P((3840, 4096, 4096), BF16, (256, 256), 256, "dp")["group_m"] == 8
    # q = 17, I = 50 (coprime): D = 17, largest divisor <= tm = 3 is 1
    assert P((607, 187, 3155), BF16, (256, 128), 256, "hybrid", min_iters=0)["group_m"] == 1
    # 4826x1341x13813 on 128x128x64: tm = 38, I = 216, q = 352:
    # D = 352 / gcd(352, 216) = 44; largest divisor of 44 <= 38 is 22
    p = P((4826, 1341, 13813), BF16, (128, 128), 256, "hybrid", min_iters=0)
    assert t(p, "q", "group_m") == (352, 22)


def test_auto_mode_cost_rule():
    # 9 tiles of 4 16-bit iterations on 4 workgroups: b + ceil(b/4) + 4 =
    # 9 + 3 + 4 = 16 >= 3 waves x 4 = 12 -> no split; hybrid keeps S = 5
    assert P((384, 384, 256), BF16, (128, 128), 4, "auto")["S"] == 0
    assert P((384, 384, 256), BF16, (128, 128), 4, "hybrid")["S"] == 5
    # FP32 iterations: no L2 term, f = 1: 9 + 1 = 10 < 12 -> S = 5
    assert P((384, 384, 128), F32, (128, 128), 4, "auto")["S"] == 5
    # FP32 3840x4096x4096 on 128x128: 960 tiles x 128 on 256: 480 + 1 <
    # 4 x 128 -> split, S = 960 mod 256 + 256 = 448
    p = P((3840, 4096, 4096), F32, (128, 128), 256, "auto")
    assert t(p, "T", "S") == (960, 448)
    # 480 tiles x 64 on 256 (256x128): 120 + 30 + 4 = 154 >= 128 -> DP grid
    p = P((3840, 4096, 4096), F16, (256, 128), 256, "auto")
    assert t(p, "S", "W", "g", "dp_grid") == (0, 0, 480, 1)
    # ... a grouped launch stays on the persistent grid
    p = P([(3840, 4096, 4096)] * 2, F16, (256, 128), 256, "auto")
    assert t(p, "S", "g", "dp_grid") == (0, 256, 0)
    # 2190x3876x2048 on 128x128: 558 tiles x 32: b = 70, 70 + 18 + 4 = 92 <
    # 96 -> two-tile rule, S = 558 mod 256 + 256 = 302
    assert t(P((2190, 3876, 2048), BF16, (128, 128), 256, "auto"), "T", "S") == (558, 302)
    # K = 1024 (16 iterations): b = 35, 35 + 9 + 4 = 48 >= 48 -> DP
    p = P((2190, 3876, 1024), BF16, (128, 128), 256, "auto")
    assert t(p, "T", "S", "dp_grid") == (558, 0, 1)
    # ... and on 256x256 (f = 8): 144 tiles, b = 9, 9 + 3 + 8 >= 16 -> DP
    assert P((2190, 3876, 1024), BF16, (256, 256), 256, "auto")["S"] == 0
    # one partial data-parallel wave on the full grid: e4m3 6160x303x2722 on
    # 128x128x128, 147 tiles x 22 (floor m = 11 leaves 294 > 256): b = 13,
    # (13 + 4 + 4) * 9/8 = 23.6 >= 22 -> DP (21 alone would split)
    p = P((6160, 303, 2722), E4, (128, 128), 256, "auto")
    assert t(p, "T", "g", "S", "dp_grid") == (147, 147, 0, 1)
    # the same shape in BF16 (43 iterations): b = 25, (25 + 7 + 4) * 9/8 =
    # 40.5 < 43 -> split
    assert t(P((6160, 303, 2722), BF16, (128, 128), 256, "auto"), "T", "g", "S") == (
        147, 256, 147)
    # T < g' but the floor shrank the grid (g' = 759 // 12 = 63): no 9/8;
    # b = 13, 13 + 4 + 4 = 21 < 23 -> split
    assert t(P((1286, 292, 1415), BF16, (128, 128), 256, "auto"), "T", "g", "S") == (
        33, 63, 33)
    # long K, few tiles: 6 tiles x 50 on g' = 17: 18 + 5 + 4 = 27 < 50
    assert t(P((607, 187, 3155), BF16, (256, 128), 256, "auto"), "g", "S") == (17, 6)


def test_grouped_problem_order_longest_first():
    # iterations per tile (BK = 64): 1, 4, 2, 4 -> problems 1, 3, 2, 0
    probs = [(128, 128, 64), (128, 256, 256), (256, 128, 128), (128, 128, 256)]
    cfg = sk.Config(tile=(128, 128), mode="hybrid", num_cu=4)
    assert sk.plan_order(probs, BF16, cfg) == [1, 3, 2, 0]
    assert sk.plan_order(probs, BF16, sk.Config(tile=(128, 128), mode="dp", num_cu=4)) == [
        0, 1, 2, 3]
    # global tiles follow that order: 2 + 1 + 2 + 1 tiles
    segs = sk.schedule(probs, BF16, sk.Config(tile=(128, 128), mode="hybrid", num_cu=4,
                                              dp_tiles=10))
    by_tile = {s[2]: s[1] for s in segs}
    assert [by_tile[i] for i in range(6)] == [1, 1, 3, 2, 2, 0]
