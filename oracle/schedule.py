"""Stream-K schedule simulator and invariant checker -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
use this module.  It shares no code with the C++/HIP schedule of the GPU
library; it is a second, plain-Python derivation of the same reading.

What the report fixes (Background section): a tile-per-core decomposition
leaves cores idle whenever the tile count is not a multiple of the core count
(its Figure 1 example runs at 75% utilisation), and Stream-K instead divides
the multiply-accumulate work into even-sized units spread over all cores.
The report gives no equations or pseudocode, so the schedule below is the
reading used throughout this project (each numbered step is named where it is
applied):

  (1) Per problem p: tm = ceil(M/BM), tn = ceil(N/BN), T_p = tm*tn output
      tiles, I_p = max(1, ceil(K/BK)) MAC-loop iterations per tile.  (A K = 0
      problem keeps one empty iteration per tile so that its tiles still reach
      the epilogue C = beta*Cin.)
  (2) Tiles are numbered problem-major, the problems taken by I_p, largest
      first, ties in the given order (a reading for grouped launches, which
      the report does not treat: whole tiles then alternate evenly between
      the persistent workgroups, longest first; DP mode keeps the given
      order); inside a problem tile u maps to
      (tm, tn) row-major, or, with group_m > 0, band-wise: bands of group_m
      tile rows, walked down the rows first, then across the columns.
      group_m = -1 (automatic; a locality reading, not in the report) is
      resolved after step (5): with Stream-K tiles, D = q / gcd(q, I) for the
      first problem that has tiles (I iterations, tm tile rows) and group_m
      is the largest divisor of D not above tm (workgroups whose ranges start
      at the same k-phase of their tiles then sit in one tile row); otherwise
      group_m = 8.
  (2b) Grid floor (not in the report; a reading that keeps split tiles from
      having dozens of contributors when the problem is small): with
      min_iters = m > 1 a Stream-K or hybrid launch uses
      g' = min(g, max(1, W_all // m)) workgroups, W_all = sum of I over all T
      tiles, so that no workgroup gets much less than m iterations.  m = 0
      selects m = ceil(I_mean / c) with I_mean = ceil(W_all / T) and c the
      largest integer >= 1 with f c^2 <= I_mean: if one partial tile costs
      about f MAC iterations (store, wait, load and add; measured:
      f = max(4, BM*BN/8192) for 16-bit and e4m3 iterations, f = max(1,
      BM*BN/32768) for FP32 iterations of 32 K-values, which take ~4.5x as
      long), a tile of I iterations split into c pieces
      takes about I/c + f(c - 1) iteration times, least near c = sqrt(I/f);
      with c = 1 tiles are not split at all.  m = 1 keeps g.  Steps (3)-(5)
      use g'.
  (3) Split point S over the T = sum T_p tiles: tiles [0,S) are Stream-K
      tiles, [S,T) data-parallel tiles.  SK mode: S = T.  DP mode: S = 0 with
      one workgroup per tile.  Hybrid ("two-tile SK + DP"): S = 0 when
      T mod g == 0, else min(T, T mod g + g).  Auto mode (not in the report):
      the hybrid rule, and S = 0 also when Stream-K cannot beat the
      data-parallel waves under the cost model of step (2b) with a quarter
      added for the L2 reuse that workgroups at different k-phases lose
      (nothing for FP32 iterations, which move too few bytes per clock for
      that loss to show): with b = ceil(W_all / g), when
      b + ceil(b / 4) + f >= ceil(T / g) * ceil(W_all / T) (FP32: b + f).
      When the DP launch would be one partial wave (T < g') and the floor
      left g' = g, the Stream-K side is taken 9/8 times (measured: T busy
      workgroups outrun g busy ones, and predicted gains under ~12% were
      losses there).  An explicit
      dp_tiles >= 0 sets S = T - min(dp_tiles, T).  Auto mode with S = 0 on a
      single problem launches the DP grid (one workgroup per tile) instead of
      dealing whole tiles to the persistent workgroups (step (8)).
  (4) Iteration space of the SK tiles: J_0 = 0, J_{t+1} = J_t + I_t, W = J_S.
  (5) Even split over g persistent workgroups: q = W // g, rho = W % g;
      workgroup x owns [s_x, e_x) with s_x = x*q + min(x, rho) and
      e_x = s_x + q + (1 if x < rho else 0).
  (6) Workgroup x walks its range tile by tile, emitting one segment per tile
      touched: FULL (all of the tile's iterations), FINISH (starts at the
      tile's iteration 0 but stops early) or PARTIAL (starts past iteration 0).
  (7) The FINISH owner of a split tile waits for the PARTIAL contributions of
      workgroups x+1 .. y, where y owns the tile's last iteration;
      npeers = y - x.
  (8) The DP tiles are dealt in rounds of g after all SK segments: in round
      r workgroup x takes tile S + r*g + x when r is even and
      S + r*g + (g-1-x) when r is odd (a reading: with step (2)'s
      longest-first order this evens out the workgroups' loads), while the
      tile exists.
"""
from bisect import bisect_right
from collections import defaultdict
from math import gcd
from dataclasses import dataclass

FULL, FINISH, PARTIAL, DP = 0, 1, 2, 3
ROLE_NAMES = {FULL: "FULL", FINISH: "FINISH", PARTIAL: "PARTIAL", DP: "DP"}
MODE_HYBRID, MODE_SK, MODE_DP, MODE_AUTO = 0, 1, 2, 3


@dataclass(frozen=True)
class Segment:
    wg: int
    problem: int
    tile: int
    tile_m: int
    tile_n: int
    k_begin: int
    k_end: int
    role: int
    npeers: int

    def as_tuple(self):
        return (self.wg, self.problem, self.tile, self.tile_m, self.tile_n,
                self.k_begin, self.k_end, self.role, self.npeers)


def cdiv(a, b):
    return -(-a // b)


def tile_coords(u, tm, tn, group_m):
    """Step (2): local tile index u -> (tile row, tile column)."""
    if group_m <= 0:
        return u // tn, u % tn
    band = u // (group_m * tn)
    h = min(group_m, tm - band * group_m)
    v = u % (group_m * tn)
    return band * group_m + v % h, v // h


@dataclass
class Plan:
    """Schedule parameters of steps (1)-(5)."""
    tiles: list          # global tile t -> (problem, tile_m, tile_n)
    iters: list          # global tile t -> I_t
    T: int
    S: int
    W: int
    g: int
    q: int
    rho: int
    J: list              # prefix sums over the SK tiles, len S+1
    dp_grid: bool        # DP mode: one workgroup per tile
    group_m: int = 0     # tile order used


def fixup_cost(block_m, block_n, block_k):
    """Step (2b): MAC iterations one partial tile costs (measured): FP32
    iterations (32 K-values) are ~4.5x longer than 16-bit / e4m3 ones."""
    if block_k == 32:
        return max(1, block_m * block_n // 32768)
    return max(4, block_m * block_n // 8192)


def auto_split(I_mean, f=4):
    """Largest c >= 1 with f c^2 <= I_mean, by plain search."""
    c = 1
    while f * (c + 1) * (c + 1) <= I_mean:
        c += 1
    return c


def grid_floor(g, iters, min_iters, f=4):
    """Step (2b): workgroups actually launched for Stream-K/hybrid."""
    T = len(iters)
    W_all = sum(iters)
    if T == 0 or W_all == 0:
        return g
    m = min_iters
    if m == 0:
        I_mean = cdiv(W_all, T)
        m = cdiv(I_mean, auto_split(I_mean, f))
    if m <= 1:
        return g
    return min(g, max(1, W_all // m))


def make_plan(problems, block_m, block_n, block_k, g, mode=MODE_HYBRID,
              dp_tiles=-1, group_m=0, min_iters=1):
    """Steps (1)-(5) for a list of (M, N, K) problems."""
    local, iters, first = [], [], None
    order = list(range(len(problems)))
    if mode != MODE_DP:                              # stable: ties keep their order
        order.sort(key=lambda p: -max(1, cdiv(problems[p][2], block_k)))
    for p in order:
        M, N, K = problems[p]
        tm = cdiv(M, block_m) if M > 0 else 0
        tn = cdiv(N, block_n) if N > 0 else 0
        I = max(1, cdiv(K, block_k))
        if tm * tn > 0 and first is None:
            first = (I, tm)
        for u in range(tm * tn):
            local.append((p, u, tm, tn))
            iters.append(I)
    T = len(local)
    f = fixup_cost(block_m, block_n, block_k)
    g_full = g
    if mode != MODE_DP:
        g = grid_floor(g, iters, min_iters, f)
    if mode == MODE_DP:
        S = 0
        g = T
    elif mode == MODE_SK:
        S = T
    else:
        S = 0 if (g == 0 or T % g == 0) else min(T, T % g + g)
        W_all = sum(iters)
        b = cdiv(W_all, g) if g > 0 else 0
        l2 = 0 if block_k == 32 else cdiv(b, 4)
        if mode == MODE_AUTO and S > 0:
            sk_cost = b + l2 + f
            if T < g and g == g_full:         # one partial data-parallel wave
                sk_cost = sk_cost * 9 / 8
            if sk_cost >= cdiv(T, g) * cdiv(W_all, T):
                S = 0
    if mode != MODE_DP and dp_tiles >= 0:
        S = T - min(dp_tiles, T)
    dp_grid = mode == MODE_DP or (mode == MODE_AUTO and S == 0 and len(problems) == 1)
    if dp_grid:
        g = T
    J = [0]
    for t in range(S):
        J.append(J[-1] + iters[t])
    W = J[-1]
    q, rho = (W // g, W % g) if g > 0 else (0, 0)
    if group_m < 0:
        if S > 0 and q > 0:
            D = q // gcd(q, first[0])
            group_m = max(G for G in range(1, min(D, first[1]) + 1) if D % G == 0)
        else:
            group_m = 8
    tiles = []
    for p, u, tm, tn in local:
        r, c = tile_coords(u, tm, tn, group_m)
        tiles.append((p, r, c))
    return Plan(tiles, iters, T, S, W, g, q, rho, J, dp_grid, group_m)


def wg_range(plan, x):
    """Step (5): iteration range [s_x, e_x) of workgroup x."""
    s = x * plan.q + min(x, plan.rho)
    return s, s + plan.q + (1 if x < plan.rho else 0)


def owner(plan, it):
    """The workgroup whose step-(5) range contains global iteration it."""
    # Scan the (at most g) workgroup ranges; plain and obviously right.
    for x in range(plan.g):
        s, e = wg_range(plan, x)
        if s <= it < e:
            return x
    raise ValueError(f"iteration {it} has no owner")


def simulate(problems, block_m, block_n, block_k, g, mode=MODE_HYBRID,
             dp_tiles=-1, group_m=0, min_iters=1):
    """Segments of every workgroup, in workgroup order and, inside a
    workgroup, in processing order (steps (6)-(8))."""
    plan = make_plan(problems, block_m, block_n, block_k, g, mode, dp_tiles,
                     group_m, min_iters)
    segs = []
    if plan.dp_grid:
        for t, (p, r, c) in enumerate(plan.tiles):
            segs.append(Segment(t, p, t, r, c, 0, plan.iters[t], DP, 0))
        return plan, segs
    for x in range(plan.g):
        s, e = wg_range(plan, x)
        it = s
        while it < e:
            t = bisect_right(plan.J, it) - 1          # J_t <= it < J_{t+1}
            p, r, c = plan.tiles[t]
            I = plan.iters[t]
            kb = it - plan.J[t]
            ke = min(e, plan.J[t + 1]) - plan.J[t]
            if kb == 0 and ke == I:
                role, npeers = FULL, 0
            elif kb == 0:
                role = FINISH
                npeers = owner(plan, plan.J[t + 1] - 1) - x
            else:
                role, npeers = PARTIAL, 0
            segs.append(Segment(x, p, t, r, c, kb, ke, role, npeers))
            it = plan.J[t] + ke
        rnd = 0
        while True:
            pos = x if rnd % 2 == 0 else plan.g - 1 - x
            t = plan.S + rnd * plan.g + pos
            if t >= plan.T:
                break
            p, r, c = plan.tiles[t]
            segs.append(Segment(x, p, t, r, c, 0, plan.iters[t], DP, 0))
            rnd += 1
    return plan, segs


# ---------------------------------------------------------------------------
# Invariants.  These are properties any correct work-centric schedule of this
# reading must have; they are computed from the segment list alone, without
# reusing the generator above.
# ---------------------------------------------------------------------------

class ScheduleError(AssertionError):
    pass


def _fail(msg):
    raise ScheduleError(msg)


def check(problems, block_m, block_n, block_k, g, mode, segs, dp_tiles=-1,
          group_m=0):
    """Raise ScheduleError unless ``segs`` satisfies invariants I1-I8.

    I1 every (SK tile, k-iteration) and every DP tile is covered exactly once
    I2 every workgroup's SK iteration count is q or q+1 and they sum to W
    I3 a workgroup has at most one PARTIAL (its first SK segment) and at most
       one FINISH (its last SK segment); SK segments precede DP segments
    I4 a FINISH waits only on higher workgroups, whose contribution to the
       tile is their first segment, and the contributions tile [0, I_t)
       contiguously in increasing workgroup order (no wait cycles)
    I5 a split tile has exactly one FINISH, with npeers = contributors - 1
    I6 slots used <= g (one per PARTIAL workgroup), flags used <= S
    I7 #FULL + #FINISH == S
    I8 single-problem hybrid with S >= g: split tiles have 2 contributors;
       DP mode: no SK segments
    plus: roles agree with (k_begin, k_end); tile coordinates are a bijection
    onto each problem's tile grid; a workgroup's SK ranges are contiguous in
    the global iteration order.
    """
    # Independent recomputation of the tile grid (no call into make_plan):
    # step (2)'s order, as one pass per distinct I from the largest down.
    grid = {}
    tile_list = []
    per_tile_iters = [max(1, cdiv(K, block_k)) for _, _, K in problems]
    passes = [None] if mode == MODE_DP else sorted(set(per_tile_iters), reverse=True)
    for want in passes:
        for p, (M, N, K) in enumerate(problems):
            I = per_tile_iters[p]
            if want is not None and I != want:
                continue
            tm = cdiv(M, block_m) if M > 0 else 0
            tn = cdiv(N, block_n) if N > 0 else 0
            for _ in range(tm * tn):
                tile_list.append((p, I, tm, tn))
    T = len(tile_list)
    seen_coords = defaultdict(set)

    sk = [s for s in segs if s.role != DP]
    dp = [s for s in segs if s.role == DP]
    if mode == MODE_DP:
        if sk:
            _fail("I8: DP mode produced SK segments")
        S = 0
    else:
        sk_tiles = {s.tile for s in sk}
        S = (max(sk_tiles) + 1) if sk_tiles else 0
        if mode == MODE_SK and dp_tiles < 0 and S != T:
            _fail(f"SK mode must make every tile an SK tile (S={S}, T={T})")

    for s in segs:
        if not (0 <= s.tile < T):
            _fail(f"segment on nonexistent tile {s.tile}")
        p, I, tm, tn = tile_list[s.tile]
        if s.problem != p:
            _fail(f"tile {s.tile} belongs to problem {p}, not {s.problem}")
        if not (0 <= s.tile_m < tm and 0 <= s.tile_n < tn):
            _fail(f"tile coords out of range: {s}")
        if not (0 <= s.k_begin < s.k_end <= I):
            _fail(f"bad k range: {s}")
        want = (DP if s.role == DP else FULL if (s.k_begin == 0 and s.k_end == I)
                else FINISH if s.k_begin == 0 else PARTIAL)
        if s.role != want:
            _fail(f"role mismatch: {s}")
        grid.setdefault(s.tile, (s.problem, s.tile_m, s.tile_n))
        if grid[s.tile] != (s.problem, s.tile_m, s.tile_n):
            _fail(f"tile {s.tile} has two coordinates")

    for t, (p, r, c) in grid.items():
        if (r, c) in seen_coords[p]:
            _fail(f"two tiles of problem {p} share coordinates {(r, c)}")
        seen_coords[p].add((r, c))

    # I1: coverage.
    cover = defaultdict(int)
    for s in sk:
        if s.tile >= S:
            _fail("SK segment beyond the split point")
        for k in range(s.k_begin, s.k_end):
            cover[(s.tile, k)] += 1
    for t in range(S):
        I = tile_list[t][1]
        for k in range(I):
            if cover[(t, k)] != 1:
                _fail(f"I1: SK (tile {t}, k {k}) covered {cover[(t, k)]} times")
    dp_count = defaultdict(int)
    for s in dp:
        if s.tile < S:
            _fail("DP segment on an SK tile")
        dp_count[s.tile] += 1
    for t in range(S, T):
        if dp_count[t] != 1:
            _fail(f"I1: DP tile {t} covered {dp_count[t]} times")
    if len(grid) != T:
        _fail("not every tile appears")

    # Per-workgroup order and contiguity.
    by_wg = defaultdict(list)
    for s in segs:
        by_wg[s.wg].append(s)
    W = sum(tile_list[t][1] for t in range(S))
    if mode == MODE_DP:
        for s in dp:
            if s.wg != s.tile:
                _fail("DP mode: workgroup t must process tile t")
    else:
        if any(not (0 <= x < g) for x in by_wg):
            _fail("workgroup id out of range")
        # global iteration index of (tile, k): prefix over SK tiles
        pref = [0]
        for t in range(S):
            pref.append(pref[-1] + tile_list[t][1])
        q = W // g if g else 0
        total = 0
        prev_end = 0
        for x in range(g):
            lst = by_wg.get(x, [])
            sk_x = [s for s in lst if s.role != DP]
            dp_x = [s for s in lst if s.role == DP]
            if lst[:len(sk_x)] != sk_x:
                _fail(f"I3: workgroup {x} has DP work before SK work")
            n = sum(s.k_end - s.k_begin for s in sk_x)
            if n not in (q, q + 1):
                _fail(f"I2: workgroup {x} has {n} iterations, q={q}")
            total += n
            for i, s in enumerate(sk_x):
                start = pref[s.tile] + s.k_begin
                if start != prev_end:
                    _fail(f"workgroup {x} range not contiguous at {s}")
                prev_end = pref[s.tile] + s.k_end
                if s.role == PARTIAL and i != 0:
                    _fail(f"I3: PARTIAL not first in workgroup {x}")
                if s.role == FINISH and i != len(sk_x) - 1:
                    _fail(f"I3: FINISH not last in workgroup {x}")
            if [s.tile for s in dp_x] != sorted(s.tile for s in dp_x):
                _fail(f"DP tiles of workgroup {x} out of order")
            for s in dp_x:
                rnd, pos = divmod(s.tile - S, g)
                if pos != (x if rnd % 2 == 0 else g - 1 - x):
                    _fail(f"DP tile {s.tile} on workgroup {x}")
        if total != W:
            _fail("I2: iteration counts do not sum to W")

    # I4/I5: fixup structure.
    contributors = defaultdict(list)
    for s in sk:
        contributors[s.tile].append(s)
    n_full = n_finish = 0
    partial_wgs = []
    for t, lst in contributors.items():
        I = tile_list[t][1]
        fin = [s for s in lst if s.role == FINISH]
        full = [s for s in lst if s.role == FULL]
        part = [s for s in lst if s.role == PARTIAL]
        if full:
            if len(lst) != 1:
                _fail(f"tile {t} has a FULL segment and other contributors")
            n_full += 1
            continue
        if len(fin) != 1:
            _fail(f"I5: split tile {t} has {len(fin)} FINISH segments")
        f = fin[0]
        n_finish += 1
        if f.npeers != len(part):
            _fail(f"I5: tile {t}: npeers {f.npeers} != {len(part)}")
        peers = sorted(part, key=lambda s: s.wg)
        if [s.wg for s in peers] != list(range(f.wg + 1, f.wg + 1 + f.npeers)):
            _fail(f"I4: tile {t}: peers are not workgroups x+1..x+npeers")
        k = f.k_end
        for s in peers:
            if s.k_begin != k:
                _fail(f"I4: tile {t}: contributions not contiguous")
            k = s.k_end
            first = [z for z in by_wg[s.wg] if z.role != DP][0]
            if first != s:
                _fail(f"I4: tile {t}: peer {s.wg}'s contribution is not its "
                      "first segment")
        if k != I:
            _fail(f"I4: tile {t}: contributions stop at {k} of {I}")
        partial_wgs.extend(s.wg for s in peers)
        if (mode in (MODE_HYBRID, MODE_AUTO) and dp_tiles < 0 and len(problems) == 1
                and S >= g and f.npeers != 1):
            _fail(f"I8: hybrid split tile {t} has {f.npeers + 1} contributors")

    # I6 / I7.
    if len(set(partial_wgs)) != len(partial_wgs) or len(partial_wgs) > max(g, 0):
        _fail("I6: a workgroup holds more than one partial slot")
    if n_finish > S:
        _fail("I6: more flags than SK tiles")
    if n_full + n_finish != S:
        _fail(f"I7: #FULL + #FINISH = {n_full + n_finish} != S = {S}")
    return True


def dp_efficiency(T, g):
    """Fraction of core-slots doing work when T equal tiles run one per core
    in waves of g: T / (ceil(T/g) * g).  The report's Figure 1 example
    (Background section) has 9 tiles on 4 cores and reads 75%."""
    if T == 0:
        return 1.0
    return T / (cdiv(T, g) * g)


def summary(segs):
    """Counts of each role and the largest contributor count of a tile."""
    counts = defaultdict(int)
    max_contrib = 1
    for s in segs:
        counts[ROLE_NAMES[s.role]] += 1
        if s.role == FINISH:
            max_contrib = max(max_contrib, s.npeers + 1)
    counts["max_contributors"] = max_contrib
    return dict(counts)
