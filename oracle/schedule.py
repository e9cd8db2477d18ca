"""Stream-K schedule simulator and invariant checker -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
use this module.  It shares no code with the C++/HIP schedule of the GPU
library; it is a second, plain-Python derivation of the same reading.

What the report fixes (Background section): a tile-per-core decomposition
leaves cores idle whenever the tile count is not a multiple of the core count
(its Figure 1 example runs at 75% utilisation), and Stream-K instead divides
the multiply-accumulate work into even-sized units spread over all cores.
The report gives no equations or pseudocode, so the schedule below is the
reading used throughout this project.

The simulator is a function of the launch it describes.  Its inputs are the
problems, the tile shape, and the launch parameters a caller has resolved:
the workgroup count g, the split point S, the tile order (group_m), the
order in which the problems are concatenated and the rule that deals whole
tiles.  How a library chooses those parameters (grid sizes, cost models,
orderings tuned on one machine) is policy, not part of the method, and is
not computed here.  Each numbered step is named where it is applied:

  (1) Per problem p: tm = ceil(M/BM), tn = ceil(N/BN), T_p = tm*tn output
      tiles, I_p = max(1, ceil(K/BK)) MAC-loop iterations per tile.  (A K = 0
      problem keeps one empty iteration per tile so that its tiles still reach
      the epilogue C = beta*Cin.)
  (2) Tiles are numbered problem-major, the problems concatenated in a given
      order (default: the order of the list); inside a problem tile u maps
      to (tm, tn) row-major, or, with group_m > 0, band-wise: bands of
      group_m tile rows, walked down the rows first, then across the columns.
  (3) Split point S: tiles [0,S) are Stream-K tiles, [S,T) whole tiles.
      The readings of the report's hybrid: all Stream-K (S = T), the
      data-parallel baseline (S = 0, one workgroup per tile) and the
      "two-tile" data-parallel + Stream-K rule S = 0 when T mod g == 0, else
      min(T, T mod g + g) (split_for_mode); any S in [0, T] is simulated.
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
  (8) The whole tiles [S, T) are dealt in rounds of g after all SK segments:
      in round r, workgroup x takes tile S + r*g + x ("cyclic") or, under the
      "serpentine" rule, S + r*g + (g-1-x) in odd rounds, while the tile
      exists.  In the data-parallel baseline workgroup t runs tile t alone.
"""
from bisect import bisect_right
from collections import defaultdict
from dataclasses import dataclass

FULL, FINISH, PARTIAL, DP = 0, 1, 2, 3
ROLE_NAMES = {FULL: "FULL", FINISH: "FINISH", PARTIAL: "PARTIAL", DP: "DP"}
MODE_HYBRID, MODE_SK, MODE_DP = 0, 1, 2
CYCLIC, SERPENTINE = "cyclic", "serpentine"


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


def two_tile_split(T, g):
    """Step (3): the data-parallel + Stream-K "two-tile" rule."""
    if g <= 0 or T % g == 0:
        return 0
    return min(T, T % g + g)


def split_for_mode(T, g, mode, dp_tiles=-1):
    """Step (3) for the report's three decompositions; dp_tiles >= 0 keeps
    that many whole tiles at the end (S = T - dp_tiles)."""
    if mode == MODE_DP:
        return 0
    S = T if mode == MODE_SK else two_tile_split(T, g)
    if dp_tiles >= 0:
        S = T - min(dp_tiles, T)
    return S


def tile_grid(problems, block_m, block_n, block_k, order=None):
    """Steps (1)-(2) without coordinates: (problem, u, tm, tn, I) per global
    tile, problems concatenated in `order`."""
    order = list(range(len(problems))) if order is None else list(order)
    if sorted(order) != list(range(len(problems))):
        raise ValueError("order must be a permutation of the problems")
    out = []
    for p in order:
        M, N, K = problems[p]
        tm = cdiv(M, block_m) if M > 0 else 0
        tn = cdiv(N, block_n) if N > 0 else 0
        I = max(1, cdiv(K, block_k))
        for u in range(tm * tn):
            out.append((p, u, tm, tn, I))
    return out


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
    dp_grid: bool        # data-parallel baseline: one workgroup per tile
    group_m: int = 0     # tile order used


def make_plan(problems, block_m, block_n, block_k, g, S, group_m=0, order=None,
              dp_grid=False):
    """Steps (1)-(5) for a list of (M, N, K) problems and resolved launch
    parameters: g workgroups, S Stream-K tiles, tile order group_m >= 0,
    problem order.  dp_grid: the baseline grid (S must be 0; g = T)."""
    grid = tile_grid(problems, block_m, block_n, block_k, order)
    T = len(grid)
    if not 0 <= S <= T:
        raise ValueError(f"S = {S} outside [0, {T}]")
    if group_m < 0:
        raise ValueError("group_m must be resolved (>= 0)")
    if dp_grid:
        if S != 0:
            raise ValueError("the data-parallel grid splits no tile")
        g = T
    elif g <= 0:
        raise ValueError("g must be positive")
    iters = [I for *_, I in grid]
    tiles = [(p,) + tile_coords(u, tm, tn, group_m) for p, u, tm, tn, _ in grid]
    J = [0]
    for t in range(S):
        J.append(J[-1] + iters[t])
    W = J[-1]
    q, rho = (W // g, W % g) if g > 0 else (0, 0)
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


def dealt_position(rnd, x, g, deal):
    """Step (8): offset inside round `rnd` of the tile workgroup x takes."""
    if deal == CYCLIC:
        return x
    if deal == SERPENTINE:
        return x if rnd % 2 == 0 else g - 1 - x
    raise ValueError(f"unknown dealing rule {deal!r}")


def simulate(problems, block_m, block_n, block_k, g, S, group_m=0, order=None,
             dp_grid=False, deal=CYCLIC):
    """Segments of every workgroup, in workgroup order and, inside a
    workgroup, in processing order (steps (6)-(8))."""
    plan = make_plan(problems, block_m, block_n, block_k, g, S, group_m, order, dp_grid)
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
            t = plan.S + rnd * plan.g + dealt_position(rnd, x, plan.g, deal)
            if t >= plan.T:
                break
            p, r, c = plan.tiles[t]
            segs.append(Segment(x, p, t, r, c, 0, plan.iters[t], DP, 0))
            rnd += 1
    return plan, segs


def simulate_mode(problems, block_m, block_n, block_k, g, mode, dp_tiles=-1, group_m=0,
                  order=None, deal=CYCLIC):
    """simulate() with S from one of the report's decompositions (step (3))."""
    T = len(tile_grid(problems, block_m, block_n, block_k, order))
    S = split_for_mode(T, g, mode, dp_tiles)
    return simulate(problems, block_m, block_n, block_k, g, S, group_m, order,
                    mode == MODE_DP, deal)


# ---------------------------------------------------------------------------
# Invariants.  These are properties any correct work-centric schedule of this
# reading must have; they are computed from the segment list alone, without
# reusing the generator above.
# ---------------------------------------------------------------------------

class ScheduleError(AssertionError):
    pass


def _fail(msg):
    raise ScheduleError(msg)


def check(problems, block_m, block_n, block_k, g, segs, order=None, dp_grid=False,
          deal=CYCLIC):
    """Raise ScheduleError unless ``segs`` satisfies invariants I1-I8.

    I1 every (SK tile, k-iteration) and every whole tile is covered exactly
       once
    I2 every workgroup's SK iteration count is q or q+1 and they sum to W
    I3 a workgroup has at most one PARTIAL (its first SK segment) and at most
       one FINISH (its last SK segment); SK segments precede whole tiles
    I4 a FINISH waits only on higher workgroups, whose contribution to the
       tile is their first segment, and the contributions tile [0, I_t)
       contiguously in increasing workgroup order (no wait cycles)
    I5 a split tile has exactly one FINISH, with npeers = contributors - 1
    I6 slots used <= g (one per PARTIAL workgroup), flags used <= S
    I7 #FULL + #FINISH == S
    I8 one problem with S >= g: every workgroup owns at least one tile's
       iterations, so a split tile has exactly 2 contributors; the
       data-parallel grid has no SK segments
    plus: roles agree with (k_begin, k_end); tile coordinates are a bijection
    onto each problem's tile grid; a workgroup's SK ranges are contiguous in
    the global iteration order; whole tiles follow the dealing rule.
    """
    # Independent recomputation of the tile grid (no call into make_plan).
    order = list(range(len(problems))) if order is None else list(order)
    tile_list = []
    for p in order:
        M, N, K = problems[p]
        tm = cdiv(M, block_m) if M > 0 else 0
        tn = cdiv(N, block_n) if N > 0 else 0
        I = max(1, cdiv(K, block_k))
        tile_list.extend([(p, I, tm, tn)] * (tm * tn))
    T = len(tile_list)
    grid = {}
    seen_coords = defaultdict(set)

    sk = [s for s in segs if s.role != DP]
    dp = [s for s in segs if s.role == DP]
    if dp_grid:
        if sk:
            _fail("I8: the data-parallel grid produced SK segments")
        S = 0
    else:
        sk_tiles = {s.tile for s in sk}
        S = (max(sk_tiles) + 1) if sk_tiles else 0

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
            _fail("whole-tile segment on an SK tile")
        dp_count[s.tile] += 1
    for t in range(S, T):
        if dp_count[t] != 1:
            _fail(f"I1: whole tile {t} covered {dp_count[t]} times")
    if len(grid) != T:
        _fail("not every tile appears")

    # Per-workgroup order and contiguity.
    by_wg = defaultdict(list)
    for s in segs:
        by_wg[s.wg].append(s)
    W = sum(tile_list[t][1] for t in range(S))
    if dp_grid:
        for s in dp:
            if s.wg != s.tile:
                _fail("data-parallel grid: workgroup t must process tile t")
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
                _fail(f"I3: workgroup {x} has whole tiles before SK work")
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
                _fail(f"whole tiles of workgroup {x} out of order")
            for s in dp_x:
                rnd, pos = divmod(s.tile - S, g)
                want = x if (deal == CYCLIC or rnd % 2 == 0) else g - 1 - x
                if pos != want:
                    _fail(f"whole tile {s.tile} on workgroup {x} ({deal} dealing)")
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
        if len(problems) == 1 and S >= g and f.npeers != 1:
            _fail(f"I8: split tile {t} has {f.npeers + 1} contributors with S >= g")

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
