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
    for deal in (sch.CYCLIC, sch.SERPENTINE):    # one round of whole tiles: same
        plan, segs = sch.simulate_mode([(M, N, K)], bm, bn, bk, d["g"], mode, deal=deal)
        assert [list(s.as_tuple()) for s in segs] == d[mode_name]["segments"]
        sch.check([(M, N, K)], bm, bn, bk, d["g"], segs, deal=deal)


def test_c1_closed_form():
    # FP32 512^3, 128x128x32 tiles, 256 workgroups, pure Stream-K:
    # 16 tiles x 16 iterations = 256 iterations, one per workgroup.
    plan, segs = sch.simulate_mode([(512, 512, 512)], 128, 128, 32, 256, sch.MODE_SK)
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
    plan, segs = sch.simulate_mode([(3840, 4096, 4096)], 256, 128, 64, 256, sch.MODE_HYBRID)
    assert (plan.T, plan.S, plan.W, plan.q) == (480, 480, 30720, 120)
    s = sch.summary(segs)
    assert s["PARTIAL"] == 224 and s["FINISH"] == 224
    assert s["max_contributors"] == 2
    aligned = [x for x in range(256) if sch.wg_range(plan, x)[0] % 64 == 0]
    assert aligned == list(range(0, 256, 8))
    sch.check([(3840, 4096, 4096)], 256, 128, 64, 256, segs)


def test_hybrid_split_rule():
    for T, g, S in [(9, 4, 5), (8, 4, 0), (3, 4, 3), (480, 256, 480),
                    (2752, 256, 448), (1024, 256, 0), (1376, 256, 352)]:
        assert sch.two_tile_split(T, g) == S, (T, g)
        # through the simulator: T tiles of one row each
        plan = sch.simulate_mode([(T, 1, 1)], 1, 1, 1, g, sch.MODE_HYBRID)[0]
        assert plan.S == S
    assert sch.split_for_mode(9, 4, sch.MODE_HYBRID, dp_tiles=2) == 7
    assert sch.split_for_mode(9, 4, sch.MODE_HYBRID, dp_tiles=99) == 0
    assert sch.split_for_mode(9, 4, sch.MODE_SK) == 9
    assert sch.split_for_mode(9, 4, sch.MODE_DP) == 0


def test_same_phase_workgroups_share_a_tile_row_in_column_order():
    # 3840x4096x4096, 256x128x64 tiles on 256 workgroups: q = 120, I = 64.
    # Workgroups x and x+8 start 960 iterations = 15 tiles apart at the same
    # k-phase; in bands of 15 tile rows (= column-major on the 15-row grid)
    # those tiles are neighbours in one tile row.
    plan = sch.make_plan([(3840, 4096, 4096)], 256, 128, 64, 256, 480, group_m=15)
    assert plan.tiles[:3] == [(0, 0, 0), (0, 1, 0), (0, 2, 0)]
    assert plan.tiles[14:17] == [(0, 14, 0), (0, 0, 1), (0, 1, 1)]
    for x in range(0, 248, 8):
        s0 = sch.wg_range(plan, x)[0]
        s1 = sch.wg_range(plan, x + 8)[0]
        assert s0 % 64 == s1 % 64                        # same k-phase
        (_, r0, c0), (_, r1, c1) = plan.tiles[s0 // 64], plan.tiles[s1 // 64]
        assert r0 == r1 and c1 == c0 + 1                 # same tile row
    # bands of 8 rows: band 0 is 8 x 16 tiles of the 15 x 16 grid
    plan = sch.make_plan([(3840, 4096, 4096)], 256, 256, 64, 256, 0, group_m=8)
    assert plan.tiles[8] == (0, 0, 1)
    assert plan.tiles[120] == (0, 0, 15) and plan.tiles[128] == (0, 8, 0)


def test_whole_tiles_longest_first_balance():
    # step (8) with the problems concatenated by iterations per tile,
    # largest first: whole tiles dealt in rounds of g leave every
    # workgroup's load within the largest I of every other's (each round
    # hands out g consecutive tiles of a non-increasing list)
    rng = random.Random(8)
    for _ in range(60):
        probs = [(rng.randint(1, 900), rng.randint(1, 900), rng.choice([64, 500, 2048, 4096]))
                 for _ in range(rng.randint(2, 9))]
        order = sorted(range(len(probs)), key=lambda p: -max(1, -(-probs[p][2] // 64)))
        g = rng.choice([3, 7, 16, 64])
        for deal in (sch.CYCLIC, sch.SERPENTINE):
            p, segs = sch.simulate(probs, 128, 128, 64, g, 0, order=order, deal=deal)
            sch.check(probs, 128, 128, 64, g, segs, order=order, deal=deal)
            load = [0] * g
            for s in segs:
                load[s.wg] += s.k_end - s.k_begin
            assert sum(load) == sum(p.iters)
            assert max(load) - min(load) <= max(p.iters)


def test_whole_tiles_dealing_rules():
    # step (8): 10 whole tiles on 4 workgroups
    p, segs = sch.simulate([(128 * 10, 128, 64)], 128, 128, 64, 4, 0, deal=sch.SERPENTINE)
    got = {x: [s.tile for s in segs if s.wg == x] for x in range(4)}
    assert got == {0: [0, 7, 8], 1: [1, 6, 9], 2: [2, 5], 3: [3, 4]}
    p, segs = sch.simulate([(128 * 10, 128, 64)], 128, 128, 64, 4, 0, deal=sch.CYCLIC)
    got = {x: [s.tile for s in segs if s.wg == x] for x in range(4)}
    assert got == {0: [0, 4, 8], 1: [1, 5, 9], 2: [2, 6], 3: [3, 7]}


def test_problem_order_is_an_input():
    probs = [(128, 128, 64), (128, 256, 256), (256, 128, 128)]
    p = sch.make_plan(probs, 128, 128, 64, 4, 0, order=[1, 2, 0])
    assert [t[0] for t in p.tiles] == [1, 1, 2, 2, 0]
    assert p.iters == [4, 4, 2, 2, 1]
    with pytest.raises(ValueError):
        sch.make_plan(probs, 128, 128, 64, 4, 0, order=[0, 0, 1])


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


@pytest.mark.parametrize("mode", [sch.MODE_SK, sch.MODE_HYBRID, sch.MODE_DP])
def test_brute_force_invariants(mode):
    for shape, (bm, bn, bk), g in _cases(10 + mode, 400):
        for gm in (0, 3):
            for dp in ((-1,) if mode == sch.MODE_DP else (-1, 0, 2)):
                for deal in (sch.CYCLIC, sch.SERPENTINE):
                    plan, segs = sch.simulate_mode([shape], bm, bn, bk, g, mode, dp, gm,
                                                   deal=deal)
                    sch.check([shape], bm, bn, bk, plan.g, segs, dp_grid=mode == sch.MODE_DP,
                              deal=deal)


def test_brute_force_any_split_point():
    # every S in [0, T] (not only the three decompositions) gives a valid
    # schedule
    rng = random.Random(5)
    for shape, (bm, bn, bk), g in _cases(31, 300):
        T = len(sch.tile_grid([shape], bm, bn, bk))
        S = rng.randint(0, T)
        deal = rng.choice([sch.CYCLIC, sch.SERPENTINE])
        plan, segs = sch.simulate([shape], bm, bn, bk, g, S, rng.choice([0, 1, 2, 5]),
                                  deal=deal)
        sch.check([shape], bm, bn, bk, g, segs, deal=deal)


def test_brute_force_grouped():
    rng = random.Random(99)
    for _ in range(150):
        probs = [(rng.choice(SIZES + [0]), rng.choice(SIZES), rng.choice(SIZES + [0]))
                 for _ in range(rng.randint(1, 6))]
        bm, bn, bk = rng.choice(TILES)
        g = rng.choice(GS)
        order = list(range(len(probs)))
        rng.shuffle(order)
        for mode in (sch.MODE_SK, sch.MODE_HYBRID, sch.MODE_DP):
            plan, segs = sch.simulate_mode(probs, bm, bn, bk, g, mode, order=order)
            sch.check(probs, bm, bn, bk, plan.g, segs, order=order,
                      dp_grid=mode == sch.MODE_DP)


def test_every_wg_count_on_paper_shapes():
    # The report traces its sub-maximal "Compute Units" failures to the block
    # to tile mapping (Methodology, Results) and a 480x512x512 failure
    # (Results, Table 1): the schedule must be valid for every g.
    for shape in [(480, 512, 512), (1920, 2000, 2000)]:
        for g in range(1, 257, 5):
            for mode in (sch.MODE_SK, sch.MODE_HYBRID):
                plan, segs = sch.simulate_mode([shape], 256, 128, 64, g, mode)
                sch.check([shape], 256, 128, 64, g, segs)


# --- mutation tests: the checker must reject planted mistakes --------------

def _base():
    prob = [(384, 384, 128)]
    plan, segs = sch.simulate_mode(prob, 128, 128, 32, 4, sch.MODE_SK)
    return prob, segs


def _rejects(prob, segs, deal=sch.CYCLIC):
    with pytest.raises(sch.ScheduleError):
        sch.check(prob, 128, 128, 32, 4, segs, deal=deal)


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
    plan, segs = sch.simulate_mode(prob, 128, 128, 32, 4, sch.MODE_SK)
    # move one iteration of WG3's FULL tile 8 into a fake fifth range
    segs = [s for s in segs if s.tile != 8] + [
        sch.Segment(3, 0, 8, 2, 2, 0, 3, sch.FINISH, 1),
        sch.Segment(3, 0, 8, 2, 2, 3, 4, sch.PARTIAL, 0)]
    _rejects(prob, segs)


def test_mutation_partial_not_first():
    prob = [(384, 384, 128)]
    plan, segs = sch.simulate_mode(prob, 128, 128, 32, 4, sch.MODE_SK)
    wg1 = [s for s in segs if s.wg == 1]
    rest = [s for s in segs if s.wg != 1]
    _rejects(prob, rest + wg1[::-1])


def test_mutation_dp_on_wrong_wg():
    prob = [(384, 384, 128)]
    plan, segs = sch.simulate_mode(prob, 128, 128, 32, 4, sch.MODE_HYBRID)
    i = next(i for i, s in enumerate(segs) if s.role == sch.DP)
    segs[i] = replace(segs[i], wg=(segs[i].wg + 1) % 4)
    _rejects(prob, segs)


def test_mutation_wrong_dealing_rule():
    # 10 whole tiles on 4 workgroups dealt back and forth, checked as cyclic
    prob = [(128 * 10, 128, 64)]
    plan, segs = sch.simulate(prob, 128, 128, 64, 4, 0, deal=sch.SERPENTINE)
    with pytest.raises(sch.ScheduleError):
        sch.check(prob, 128, 128, 64, 4, segs, deal=sch.CYCLIC)


def test_mutation_wrong_problem_order():
    probs = [(128, 128, 64), (128, 256, 256)]
    plan, segs = sch.simulate(probs, 128, 128, 64, 2, 3, order=[1, 0])
    sch.check(probs, 128, 128, 64, 2, segs, order=[1, 0])
    with pytest.raises(sch.ScheduleError):
        sch.check(probs, 128, 128, 64, 2, segs, order=[0, 1])
