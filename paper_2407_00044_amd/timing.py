"""GPU timing of library calls by HIP graph replay.

Each callable's `reps` calls are captured in one graph (torch.cuda.CUDAGraph,
a HIP graph on ROCm), so host-side call overhead, which exceeds the kernel
time of small problems, is not counted.  The graphs are replayed in turn for
several rounds, so clock or thermal drift hits every callable alike, and the
median per-call time of each is kept.

Anything a callable allocates must exist before capture: pass the library a
Workspace that was sized beforehand (Workspace.get outside the capture).
"""
import torch


def graph(fn, reps):
    """A graph holding `reps` calls of fn (fn runs once eagerly first)."""
    fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(reps):
            fn()
    g.replay()
    torch.cuda.synchronize()
    return g


def time_all(fns, reps, rounds=None):
    """Milliseconds per call of each fn (median over `rounds` rounds, default
    2 * len(fns) + 1).  Round r replays the graphs starting at a rotating
    offset, and every other round in reverse order, so each fn runs in every
    position and after each of its neighbours: under a power limit the clock
    a kernel gets depends on what ran just before it."""
    graphs = [graph(fn, reps) for fn in fns]
    n = len(graphs)
    rounds = rounds or 2 * n + 1
    times = [[] for _ in fns]
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    for r in range(rounds):
        order = [(r // 2 + k) % n for k in range(n)]
        if r % 2:
            order.reverse()
        for i in order:
            s.record()
            graphs[i].replay()
            e.record()
            torch.cuda.synchronize()
            times[i].append(s.elapsed_time(e) / reps)
    del graphs
    return [sorted(t)[len(t) // 2] for t in times]
