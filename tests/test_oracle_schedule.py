"""Pins of the Stream-K schedule simulator (CPU only).

The simulator is checked against: the utilisation figure the report prints
(Background section, Figure 1), hand-derived worked schedules
(tests/golden/schedule_examples.json), closed forms of the two configurations
it is used on, and -- by brute force over many small shapes, tile sizes,
workgroup counts and modes -- the invariants of a valid work-centric
schedule, computed from the segment list alone.  Mutation tests plant
mistakes in a simulated schedule and require the checker to flag them.
"""
import json
import os
import random
from dataclasses import replace

import pytest

from oracle import schedule as sch

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_figure1_utilisation():
    d = json.load(open(os.path.join(GOLD, "paper_numbers.json")))
    f = d["figure1_dp_utilisation"]
    assert sch.dp_efficiency(f["tiles"], f["cores"]) == f["utilisation"]
    # other small (tiles, cores) pairs with the same 75% utilisation
    assert sch.dp_efficiency(3, 4) == 0.75 and sch.dp_efficiency(6, 4) == 0.75
    assert sch.dp_efficiency(8, 4) == 1.0 and sch.dp_efficiency(0, 4) == 1.0


@pytest.mark.parametrize("mode_name,mode", [("sk", sch.MODE_SK),
                                            ("hybrid", sch.MODE_HYBRID)])
def test_worked_examples(mode_name, mode):
    d = json.load(open(os.path.join(GOLD, "schedule_examples.json")))
    M, N, K = d["problem"]
    bm, bn, bk = d["tile"]
    plan, segs = sch.simulate([(M, N, K)], bm, bn, bk, d["g"], mode)
    assert [list(s.as_tuple()) for s in segs] == d[mode_name]["segments"]
    sch.check([(M, N, K)], bm, bn, bk, d["g"], mode, segs)


def test_c1_closed_form():
    # FP32 512^3, 128x128x32 tiles, 256 workgroups, pure Stream-K:
    # 16 tiles x 16 iterations = 256 iterations, one per workgroup.
    plan, segs = sch.simulate([(512, 512, 512)], 128, 128, 32, 256, sch.MODE_SK)
    assert (plan.T, plan.S, plan.W, plan.q, plan.rho) == (16, 16, 256, 1, 0)
    s = sch.summary(segs)
    assert s["FINISH"] == 16 and s["PARTIAL"] == 240 and "FULL" not in s
    assert s["max_contributors"] == 16
    for seg in segs:
        assert seg.tile == seg.wg // 16 and seg.k_begin == seg.wg % 16
        if seg.role == sch.FINISH:
            assert seg.wg % 16 == 0 and seg.npeers == 15


def test_c2_closed_form():
    # FP16 3840x4096x4096, 256x128x64 tiles, 256 workgroups, hybrid rule.
    plan, segs = sch.simulate([(3840, 4096, 4096)], 256, 128, 64, 256)
    assert (plan.T, plan.S, plan.W, plan.q) == (480, 480, 30720, 120)
    s = sch.summary(segs)
    assert s["PARTIAL"] == 224 and s["FINISH"] == 224
    assert s["max_contributors"] == 2
    aligned = [x for x in range(256) if sch.wg_range(plan, x)[0] % 64 == 0]
    assert aligned == list(range(0, 256, 8))
    sch.check([(3840, 4096, 4096)], 256, 128, 64, 256, sch.MODE_HYBRID, segs)


def test_hybrid_split_rule():
    for T, g, S in [(9, 4, 5), (8, 4, 0), (3, 4, 3), (480, 256, 480),
                    (2752, 256, 448), (1024, 256, 0), (1376, 256, 352)]:
        tm = T  # one tile column: T tiles of 1 row each
        plan = sch.make_plan([(tm, 1, 1)], 1, 1, 1, g, sch.MODE_HYBRID)
        assert plan.S == S, (T, g, plan.S)
    plan = sch.make_plan([(9, 1, 1)], 1, 1, 1, 4, sch.MODE_HYBRID, dp_tiles=2)
    assert plan.S == 7
    plan = sch.make_plan([(9, 1, 1)], 1, 1, 1, 4, sch.MODE_HYBRID, dp_tiles=99)
    assert plan.S == 0


def test_grid_floor_hand_values():
    # 607x187x3155 on 256x128x64 tiles: 3x2 = 6 tiles of ceil(3155/64) = 50
    # iterations, W_all = 300; automatic split c = 3 (4*9 <= 50 < 4*16),
    # m = ceil(50/3) = 17, so the grid shrinks from 256 to 300 // 17 = 17
    # workgroups: 300 = 17*17 + 11.
    plan = sch.make_plan([(607, 187, 3155)], 256, 128, 64, 256, sch.MODE_HYBRID, min_iters=0)
    assert (plan.T, plan.g, plan.S, plan.W, plan.q, plan.rho) == (6, 17, 6, 300, 17, 11)
    # m = 1 keeps the grid: 300 iterations over 256 workgroups
    plan = sch.make_plan([(607, 187, 3155)], 256, 128, 64, 256, sch.MODE_HYBRID, min_iters=1)
    assert (plan.g, plan.q, plan.rho) == (256, 1, 44)
    # the headline shape on 256x256 tiles (fixup cost 8) is large enough:
    # c = 2 (8*4 <= 64 < 8*9), m = 32, 15360 // 32 = 480 > 256
    plan = sch.make_plan([(3840, 4096, 4096)], 256, 256, 64, 256, sch.MODE_SK, min_iters=0)
    assert (plan.T, plan.g, plan.W, plan.q) == (240, 256, 15360, 60)
    # explicit m; a floor above W_all leaves one workgroup; DP mode ignores it
    plan = sch.make_plan([(512, 512, 512)], 128, 128, 32, 256, sch.MODE_SK, min_iters=40)
    assert (plan.g, plan.q, plan.rho) == (6, 42, 4)      # 256 iterations // 40
    plan = sch.make_plan([(100, 100, 100)], 128, 128, 32, 256, sch.MODE_SK, min_iters=9)
    assert (plan.g, plan.q) == (1, 4)
    plan = sch.make_plan([(512, 512, 512)], 128, 128, 32, 256, sch.MODE_DP, min_iters=40)
    assert plan.g == 16
    # the floor feeds the hybrid rule: 20 tiles x 8 iterations are too short
    # to split (c = 1, m = 8) -> g' = 20 = T -> S = 0, pure data-parallel
    plan = sch.make_plan([(20, 1, 8)], 1, 1, 1, 256, sch.MODE_HYBRID, min_iters=0)
    assert (plan.g, plan.S, plan.W) == (20, 0, 0)
    # 20 tiles x 64 iterations: c = 4, m = 16 -> g' = 80; 20 mod 80 = 20 ->
    # S = min(20, 100) = 20, q = 16
    plan = sch.make_plan([(20, 1, 64)], 1, 1, 1, 256, sch.MODE_HYBRID, min_iters=0)
    assert (plan.g, plan.S, plan.q, plan.rho) == (80, 20, 16, 0)
    assert [sch.auto_split(n) for n in (0, 1, 15, 16, 35, 36, 64, 99, 100)] == [
        1, 1, 1, 2, 2, 3, 4, 4, 5]


def test_auto_tile_order_hand_values():
    # 3840x4096x4096, 256x128x64 tiles on 256 workgroups: q = 120, I = 64,
    # gcd 8 -> bands of 15 rows = the whole 15-row grid, i.e. column-major;
    # workgroups x and x+8 start at the same k-phase on tiles 15 apart,
    # which are neighbours in one tile row.
    plan = sch.make_plan([(3840, 4096, 4096)], 256, 128, 64, 256, sch.MODE_HYBRID,
                         group_m=-1, min_iters=0)
    assert plan.group_m == 15
    assert plan.tiles[:3] == [(0, 0, 0), (0, 1, 0), (0, 2, 0)]
    assert plan.tiles[14:17] == [(0, 14, 0), (0, 0, 1), (0, 1, 1)]
    for x in range(0, 248, 8):
        s0 = sch.wg_range(plan, x)[0]
        s1 = sch.wg_range(plan, x + 8)[0]
        assert s0 % 64 == s1 % 64                        # same k-phase
        (_, r0, c0), (_, r1, c1) = plan.tiles[s0 // 64], plan.tiles[s1 // 64]
        assert r0 == r1 and c1 == c0 + 1                 # same tile row
    # 256x256 tiles: q = 60, gcd(60, 64) = 4 -> 15
    assert sch.make_plan([(3840, 4096, 4096)], 256, 256, 64, 256, sch.MODE_SK,
                         group_m=-1).group_m == 15
    # no Stream-K tiles: bands of 8 rows
    plan = sch.make_plan([(3840, 4096, 4096)], 256, 256, 64, 256, sch.MODE_DP, group_m=-1)
    assert plan.group_m == 8 and plan.tiles[8] == (0, 0, 1)
    assert plan.tiles[120] == (0, 0, 15) and plan.tiles[128] == (0, 8, 0)   # band 0: 8x16 tiles
    # q = 17, I = 50 (coprime): D = 17, largest divisor <= tm = 3 is 1
    # (row-major bands of one row)
    plan = sch.make_plan([(607, 187, 3155)], 256, 128, 64, 256, sch.MODE_HYBRID,
                         group_m=-1, min_iters=0)
    assert plan.group_m == 1 and plan.tiles[1] == (0, 0, 1)
    # 4826x1341x13813 on 128x128x64: tm = 38, I = 216, q = 352 (rho = 176):
    # D = 352 / gcd(352, 216) = 44; largest divisor of 44 <= 38 is 22
    plan = sch.make_plan([(4826, 1341, 13813)], 128, 128, 64, 256, sch.MODE_HYBRID,
                         group_m=-1, min_iters=0)
    assert (plan.q, plan.group_m) == (352, 22)
    assert plan.tiles[0][1:] == (0, 0) and plan.tiles[44][1:] == (0, 2)


def test_grid_floor_invariants():
    for shape, (bm, bn, bk), g in _cases(77, 300):
        for mode in (sch.MODE_SK, sch.MODE_HYBRID):
            for m in (0, 3, 50):
                plan, segs = sch.simulate([shape], bm, bn, bk, g, mode, -1, 0, m)
                assert 1 <= plan.g <= g
                sch.check([shape], bm, bn, bk, plan.g, mode, segs)
                if plan.T and plan.W:
                    # no workgroup below the floor unless the grid is one WG
                    im = -(-sum(plan.iters) // plan.T)
                    mm = m or -(-im // sch.auto_split(im, sch.fixup_cost(bm, bn, bk)))
                    assert plan.g == g or plan.g == 1 or sum(plan.iters) // plan.g >= mm


def test_auto_mode_cost_rule():
    # The worked example (9 tiles of 4 16-bit iterations, 4 workgroups):
    # Stream-K would need b + ceil(b/4) + 4 = 9 + 3 + 4 = 16 iteration times
    # against 3 waves x 4 = 12 for data-parallel, so auto mode splits
    # nothing; hybrid keeps its two-tile rule (S = 5).
    assert sch.make_plan([(384, 384, 256)], 128, 128, 64, 4, sch.MODE_AUTO).S == 0
    assert sch.make_plan([(384, 384, 256)], 128, 128, 64, 4, sch.MODE_HYBRID).S == 5
    # FP32 iterations (32 K-values) carry no L2 term and f = 1: the same
    # 9 tiles x 4 iterations need 9 + 1 = 10 < 12 -> two-tile rule (S = 5)
    assert sch.make_plan([(384, 384, 128)], 128, 128, 32, 4, sch.MODE_AUTO).S == 5
    # FP32 3840x4096x4096 on 128x128x32: 960 tiles x 128 on 256: 480 + 1 =
    # 481 < 4 x 128 = 512 -> split (S = 960 mod 256 + 256 = 448)
    p = sch.make_plan([(3840, 4096, 4096)], 128, 128, 32, 256, sch.MODE_AUTO, min_iters=0)
    assert (p.T, p.S) == (960, 448)
    # 3840x4096x4096, 256x128 tiles: 480 tiles x 64 iterations on 256:
    # 120 + 30 + 4 = 154 >= 2 x 64 = 128 -> data-parallel, and with nothing
    # split on a single problem the launch is the DP grid (480 workgroups)
    p = sch.make_plan([(3840, 4096, 4096)], 256, 128, 64, 256, sch.MODE_AUTO, min_iters=0)
    assert (p.S, p.W, p.g, p.dp_grid) == (0, 0, 480, True)
    # ... but a grouped launch stays on the persistent grid
    p = sch.make_plan([(3840, 4096, 4096)] * 2, 256, 128, 64, 256, sch.MODE_AUTO, min_iters=0)
    assert (p.S, p.g, p.dp_grid) == (0, 256, False)
    # 2190x3876x2048 on 128x128: 558 tiles x 32 iterations on 256: b = 70,
    # 70 + 18 + 4 = 92 < 3 x 32 = 96 -> two-tile rule, S = 558 mod 256 + 256
    p = sch.make_plan([(2190, 3876, 2048)], 128, 128, 64, 256, sch.MODE_AUTO, min_iters=0)
    assert (p.T, p.S) == (558, 302)
    # with K = 1024 (16 iterations): b = 35, 35 + 9 + 4 = 48 >= 48 -> DP
    p = sch.make_plan([(2190, 3876, 1024)], 128, 128, 64, 256, sch.MODE_AUTO, min_iters=0)
    assert (p.T, p.S, p.dp_grid) == (558, 0, True)
    # ... and on 256x256 (fixup 8): 144 tiles, b = 9, 9 + 3 + 8 >= 16 -> DP
    p = sch.make_plan([(2190, 3876, 1024)], 256, 256, 64, 256, sch.MODE_AUTO, min_iters=0)
    assert p.S == 0
    # one partial data-parallel wave on the full grid: e4m3 6160x303x2722 on
    # 128x128x128, 147 tiles x 22 on g' = 256 (floor m = 11 leaves 294 > 256):
    # b = 13, (13 + 4 + 4) * 9/8 = 23.6 >= 22 -> DP (21 alone would split)
    p = sch.make_plan([(6160, 303, 2722)], 128, 128, 128, 256, sch.MODE_AUTO, min_iters=0)
    assert (p.T, p.g, p.S, p.dp_grid) == (147, 147, 0, True)
    # the same shape in BF16 (43 iterations): b = 25, (25 + 7 + 4) * 9/8 =
    # 40.5 < 43 -> split
    p = sch.make_plan([(6160, 303, 2722)], 128, 128, 64, 256, sch.MODE_AUTO, min_iters=0)
    assert (p.T, p.g, p.S) == (147, 256, 147)
    # T < g' but the floor shrank the grid (g' = 759 // 12 = 63): no 9/8;
    # b = 13, 13 + 4 + 4 = 21 < 23 -> split
    p = sch.make_plan([(1286, 292, 1415)], 128, 128, 64, 256, sch.MODE_AUTO, min_iters=0)
    assert (p.T, p.g, p.S) == (33, 63, 33)
    # long K, few tiles: 6 tiles x 50 on g' = 17: 18 + 5 + 4 = 27 < 50 -> split
    p = sch.make_plan([(607, 187, 3155)], 256, 128, 64, 256, sch.MODE_AUTO, min_iters=0)
    assert (p.g, p.S) == (17, 6)
    assert [sch.fixup_cost(*t, 64) for t in [(64, 128), (128, 128), (256, 128), (256, 256)]] == [
        4, 4, 4, 8]
    assert sch.fixup_cost(128, 128, 128) == 4 and sch.fixup_cost(128, 128, 32) == 1
    # FP32 512^3 on 128x128x32: 16 tiles of 16 iterations; f = 1, c = 4
    # (1 * 4^2 <= 16 < 1 * 5^2), m = 4, g' = 256 // 4 = 64 workgroups: every
    # tile in 4 pieces of 4 iterations
    p = sch.make_plan([(512, 512, 512)], 128, 128, 32, 256, sch.MODE_SK, min_iters=0)
    assert (p.g, p.q, p.rho) == (64, 4, 0)


def test_grouped_tile_order_longest_first():
    # step (2): problems by iterations per tile, largest first, ties in the
    # given order (K = 64, 256, 128, 256 on BK = 64 -> I = 1, 4, 2, 4)
    probs = [(128, 128, 64), (128, 256, 256), (256, 128, 128), (128, 128, 256)]
    p = sch.make_plan(probs, 128, 128, 64, 4, sch.MODE_HYBRID)
    assert [t[0] for t in p.tiles] == [1, 1, 3, 2, 2, 0]
    assert p.iters == [4, 4, 4, 2, 2, 1]
    # the data-parallel grid keeps the given order
    p = sch.make_plan(probs, 128, 128, 64, 4, sch.MODE_DP)
    assert [t[0] for t in p.tiles] == [0, 1, 1, 2, 2, 3]
    # whole tiles dealt in that order (step (8)): every workgroup's load is
    # within the largest I of every other's
    rng = random.Random(8)
    for _ in range(60):
        probs = [(rng.randint(1, 900), rng.randint(1, 900), rng.choice([64, 500, 2048, 4096]))
                 for _ in range(rng.randint(2, 9))]
        g = rng.choice([3, 7, 16, 64])
        p, segs = sch.simulate(probs, 128, 128, 64, g, sch.MODE_HYBRID, dp_tiles=10 ** 6)
        assert p.S == 0
        load = [0] * g
        for s in segs:
            load[s.wg] += s.k_end - s.k_begin
        assert sum(load) == sum(p.iters)
        assert max(load) - min(load) <= max(p.iters)


def test_dp_tiles_dealt_back_and_forth():
    # step (8): 10 DP tiles on 4 workgroups: rounds 0..3 at positions
    # x, 3-x, x, 3-x (the last round holds tiles 8 and 9 only)
    p, segs = sch.simulate([(128 * 10, 128, 64)], 128, 128, 64, 4, sch.MODE_HYBRID,
                           dp_tiles=10)
    got = {x: [s.tile for s in segs if s.wg == x] for x in range(4)}
    assert got == {0: [0, 7, 8], 1: [1, 6, 9], 2: [2, 5], 3: [3, 4]}


def test_group_m_tile_order_is_a_bijection():
    for tm, tn, gm in [(5, 3, 2), (7, 4, 3), (8, 8, 4), (1, 9, 4), (6, 1, 8)]:
        coords = [sch.tile_coords(u, tm, tn, gm) for u in range(tm * tn)]
        assert sorted(coords) == [(r, c) for r in range(tm) for c in range(tn)]
    # band walk: group_m rows down first, then across
    assert [sch.tile_coords(u, 4, 3, 2) for u in range(6)] == [
        (0, 0), (1, 0), (0, 1), (1, 1), (0, 2), (1, 2)]


SIZES = [1, 7, 64, 65, 127, 129, 200, 257]
TILES = [(128, 128, 32), (256, 128, 64), (64, 64, 16), (32, 128, 128)]
GS = [1, 2, 3, 4, 5, 7, 8, 16, 31, 64, 120, 255, 256]


def _cases(seed, n):
    rng = random.Random(seed)
    for _ in range(n):
        shape = (rng.choice(SIZES), rng.choice(SIZES), rng.choice(SIZES + [0]))
        yield shape, rng.choice(TILES), rng.choice(GS)


@pytest.mark.parametrize("mode", [sch.MODE_SK, sch.MODE_HYBRID, sch.MODE_DP, sch.MODE_AUTO])
def test_brute_force_invariants(mode):
    for shape, (bm, bn, bk), g in _cases(10 + mode, 400):
        for gm in (0, 3):
            for dp in ((-1,) if mode == sch.MODE_DP else (-1, 0, 2)):
                plan, segs = sch.simulate([shape], bm, bn, bk, g, mode, dp, -1)
                sch.check([shape], bm, bn, bk, plan.g, mode, segs, dp, plan.group_m)
                plan, segs = sch.simulate([shape], bm, bn, bk, g, mode, dp, gm)
                sch.check([shape], bm, bn, bk, plan.g, mode, segs, dp, gm)


def test_brute_force_grouped():
    rng = random.Random(99)
    for _ in range(150):
        probs = [(rng.choice(SIZES + [0]), rng.choice(SIZES), rng.choice(SIZES + [0]))
                 for _ in range(rng.randint(1, 6))]
        bm, bn, bk = rng.choice(TILES)
        g = rng.choice(GS)
        for mode in (sch.MODE_SK, sch.MODE_HYBRID, sch.MODE_DP):
            plan, segs = sch.simulate(probs, bm, bn, bk, g, mode)
            sch.check(probs, bm, bn, bk, g, mode, segs)


def test_every_wg_count_on_paper_shapes():
    # The report traces its sub-maximal "Compute Units" failures to the block
    # to tile mapping (Methodology, Results) and a 480x512x512 failure
    # (Results, Table 1): the schedule must be valid for every g.
    for shape in [(480, 512, 512), (1920, 2000, 2000)]:
        for g in range(1, 257, 5):
            for mode in (sch.MODE_SK, sch.MODE_HYBRID):
                plan, segs = sch.simulate([shape], 256, 128, 64, g, mode)
                sch.check([shape], 256, 128, 64, g, mode, segs)


# --- mutation tests: the checker must reject planted mistakes --------------

def _base():
    prob = [(384, 384, 128)]
    plan, segs = sch.simulate(prob, 128, 128, 32, 4, sch.MODE_SK)
    return prob, segs


def _rejects(prob, segs, mode=sch.MODE_SK):
    with pytest.raises(sch.ScheduleError):
        sch.check(prob, 128, 128, 32, 4, mode, segs)


def test_mutation_dropped_iteration():
    prob, segs = _base()
    i = next(i for i, s in enumerate(segs) if s.role == sch.PARTIAL)
    segs[i] = replace(segs[i], k_begin=segs[i].k_begin + 1)
    _rejects(prob, segs)


def test_mutation_double_coverage():
    prob, segs = _base()
    i = next(i for i, s in enumerate(segs) if s.role == sch.FINISH)
    segs[i] = replace(segs[i], k_end=segs[i].k_end + 1)
    _rejects(prob, segs)


def test_mutation_wrong_npeers():
    prob, segs = _base()
    i = next(i for i, s in enumerate(segs) if s.role == sch.FINISH)
    segs[i] = replace(segs[i], npeers=segs[i].npeers + 1)
    _rejects(prob, segs)


def test_mutation_wrong_role():
    prob, segs = _base()
    i = next(i for i, s in enumerate(segs) if s.role == sch.PARTIAL)
    segs[i] = replace(segs[i], role=sch.FULL)
    _rejects(prob, segs)


def test_mutation_swapped_tile_coords():
    prob, segs = _base()
    segs = [replace(s, tile_m=s.tile_n, tile_n=s.tile_m) if s.tile == 1 else s
            for s in segs]
    _rejects(prob, segs)


def test_mutation_unbalanced_split():
    prob = [(384, 384, 128)]
    plan, segs = sch.simulate(prob, 128, 128, 32, 4, sch.MODE_SK)
    # move one iteration of WG3's FULL tile 8 into a fake fifth range
    segs = [s for s in segs if s.tile != 8] + [
        sch.Segment(3, 0, 8, 2, 2, 0, 3, sch.FINISH, 1),
        sch.Segment(3, 0, 8, 2, 2, 3, 4, sch.PARTIAL, 0)]
    _rejects(prob, segs)


def test_mutation_partial_not_first():
    prob = [(384, 384, 128)]
    plan, segs = sch.simulate(prob, 128, 128, 32, 4, sch.MODE_SK)
    wg1 = [s for s in segs if s.wg == 1]
    rest = [s for s in segs if s.wg != 1]
    _rejects(prob, rest + wg1[::-1])


def test_mutation_dp_on_wrong_wg():
    prob = [(384, 384, 128)]
    plan, segs = sch.simulate(prob, 128, 128, 32, 4, sch.MODE_HYBRID)
    i = next(i for i, s in enumerate(segs) if s.role == sch.DP)
    segs[i] = replace(segs[i], wg=(segs[i].wg + 1) % 4)
    _rejects(prob, segs, sch.MODE_HYBRID)
