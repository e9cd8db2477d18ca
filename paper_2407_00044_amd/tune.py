"""Autotuner: picks the tile shape and the data-parallel / Stream-K split.

Candidates are every built tile for the input type crossed with a small set
of schedules: the cost-model (auto) rule, the two-tile hybrid rule, all
tiles Stream-K, a one-tile Stream-K remainder (dp_tiles = T - T mod g), and
the plain data-parallel grid, each with the automatic tile order; the
hybrid rule is also tried in plain row-major tile order.  The candidates run
on the caller's buffers and are timed together by graph replay (each
candidate's launches captured in one HIP graph, the graphs replayed in turn,
median kept; see timing.time_all), so host call overhead does not decide
between them on small shapes.  The fastest is cached in a JSON file keyed by
device, CU count, input/output types, layouts and shape, so a shape is
measured once per machine.
"""
import json
import os
import threading

import torch

from . import api
from .timing import time_all

_lock = threading.Lock()


def cache_path():
    return os.environ.get("SK_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "streamk_tune.json"))


def _load_cache():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(c):
    """Writes the cache; an unwritable location only costs re-tuning."""
    p = cache_path()
    tmp = p + f".tmp{os.getpid()}"
    try:
        os.makedirs(os.path.dirname(p), exist_ok=True)
        with open(tmp, "w") as f:
            json.dump(c, f, indent=1, sort_keys=True)
        os.replace(tmp, p)
    except OSError:
        pass


def _device_key():
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{getattr(props, 'gcnArchName', props.name)}/{props.multi_processor_count}cu"


def candidates(shapes, dtype, num_cu=0, tiles=None):
    """Candidate configs for problems `shapes` [(M, N, K), ...]."""
    tiles = tiles or [(bm, bn) for bm, bn, _ in api.supported_tiles(dtype)]
    out = []
    for t in tiles:
        base = api.Config(tile=t, num_cu=num_cu)
        p = api.plan(shapes, dtype, api.Config(tile=t, mode="hybrid", num_cu=num_cu))
        T, g = p["T"], p["g"]
        if T == 0:
            continue
        out.append(base)                                       # cost-model rule
        out.append(api.Config(tile=t, mode="hybrid", num_cu=num_cu))   # two-tile rule
        out.append(api.Config(tile=t, mode="hybrid", num_cu=num_cu, group_m=0))
        out.append(api.Config(tile=t, mode="sk", num_cu=num_cu))
        one = T - T % g if T % g else T                        # one-tile SK remainder
        if one not in (0, T):
            out.append(api.Config(tile=t, mode="hybrid", num_cu=num_cu, dp_tiles=one))
        out.append(api.Config(tile=t, mode="dp", num_cu=num_cu))
    return out


def _key(kind, shapes, A, B, out_dtype, num_cu):
    la, _ = api.operand_layout(A)
    lb, _ = api.operand_layout(B)
    shp = ";".join(f"{m}x{n}x{k}" for m, n, k in shapes)
    return f"{_device_key()}|{kind}|{A.dtype}|{out_dtype}|{la}{lb}|g{num_cu}|{shp}"


_FIELDS = ("mode", "num_cu", "dp_tiles", "group_m", "min_iters")


def config_to_dict(c):
    return {"tile": list(c.tile), **{f: getattr(c, f) for f in _FIELDS}}


def config_from_dict(d):
    return api.Config(tile=tuple(d["tile"]), **{f: d[f] for f in _FIELDS if f in d})


def tune_gemm(A, B, out_dtype=torch.float32, num_cu=0, reps=10, use_cache=True,
              report=None):
    """Best Config for out = A @ B on these operands (timed on them)."""
    M, K = A.shape
    N = B.shape[1]
    key = _key("gemm", [(M, N, K)], A, B, out_dtype, num_cu)
    if use_cache:
        hit = _load_cache().get(key)
        if hit:
            return config_from_dict(hit["config"])
    out = torch.empty((M, N), dtype=out_dtype, device=A.device)
    cands = candidates([(M, N, K)], A.dtype, num_cu)
    ws = api.Workspace(A.device)
    need = max(api.plan([(M, N, K)], A.dtype, c)["workspace_bytes"] for c in cands)
    ws.get(need, torch.cuda.current_stream().cuda_stream)     # before any capture
    fns = [(lambda c: (lambda: api.gemm(A, B, out=out, config=c, workspace=ws)))(c)
           for c in cands]
    results = sorted(zip(time_all(fns, reps, rounds=3), cands), key=lambda r: r[0])
    best_ms, best = results[0]
    if report is not None:
        report.extend(results)
    if use_cache:
        with _lock:
            c = _load_cache()
            c[key] = {"config": config_to_dict(best), "ms": best_ms}
            _store_cache(c)
    return best


def tune_grouped(problems, scales=None, num_cu=0, reps=10, use_cache=True, report=None):
    """Best Config for a grouped launch over `problems` (see GroupedGemm)."""
    shapes = [(p[0].shape[0], p[1].shape[1], p[0].shape[1]) for p in problems]
    A0, B0, O0 = problems[0][:3]
    key = _key("grouped", shapes, A0, B0, O0.dtype, num_cu)
    if use_cache:
        hit = _load_cache().get(key)
        if hit:
            return config_from_dict(hit["config"])
    cands = candidates(shapes, A0.dtype, num_cu)
    groups = [api.GroupedGemm(problems, config=c, scales=scales) for c in cands]
    results = sorted(zip(time_all([gg.run for gg in groups], reps, rounds=3), cands),
                     key=lambda r: r[0])
    del groups
    best_ms, best = results[0]
    if report is not None:
        report.extend(results)
    if use_cache:
        with _lock:
            c = _load_cache()
            c[key] = {"config": config_to_dict(best), "ms": best_ms}
            _store_cache(c)
    return best
