"""Calibration of the launch-time predictor (the library's cost model).

The report lists a predictive model of Stream-K's block-to-time behaviour as
future work (Results, the Block2Time paragraph; Future Work).  The library's
model predicts the time of a launch from its schedule: each workgroup's time
is the sum over its segments of

    t_tile + iterations * t_it(n) [* (1 + l2) for Stream-K iterations]
    + t_store       (a PARTIAL segment stores and publishes its partial tile)
    + npeers * t_peer   (a FINISH segment adds each peer's partial tile,
                         after waiting until that peer has published it),

plus t_cin for an epilogue that reads C_in (beta != 0), plus t_launch for
the launch; the launch takes as long as its slowest workgroup.  t_it(n) is the time of one MAC iteration when n workgroups run
at once (interpolated between a light load of 64 and a full load of 256
workgroups: the per-CU feed from L2 slows as more CUs share it), and l2 is
the share of an iteration lost when the workgroups of an XCD walk K at
different phases (Stream-K) instead of in step (data-parallel waves).

This script measures, per input type and tile (A row-major, B column-major,
FP32 C, beta = 0; graph-replayed launches), the launches the constants are
solved from:

  A  data-parallel grid, 256 tiles (one full wave), I = 8, 32, 64
     -> t_it(256) (slope), t_launch + t_tile (intercept)
  B  data-parallel grid, 64 tiles (one light wave), I = 8, 32, 64 -> t_it(64)
  C  data-parallel grid, 512 tiles (two full waves), I = 32 -> t_tile
  D  all Stream-K on 256 workgroups, 128 tiles of I = 64: every tile in two
     pieces (one peer)
  E  all Stream-K on 256 workgroups, 64 tiles of I = 64: four pieces (three
     peers)                                  -> t_store, t_peer (D and E)
  F  all Stream-K on 256 workgroups, 240 tiles of I = 64 (q = 60: every
     workgroup at its own k-phase)           -> l2
  G  as A with I = 32 and beta = 0.5 (the epilogue reads C_in) -> t_cin

The model is linear in its constants for these launches, so they are fitted
together by non-negative least squares on the relative error, and the script
prints them with the C++ table row the library compiles in.

    python -m paper_2407_00044_amd.calibrate [--reps 20] [--out FILE]
"""
import argparse
import json
import sys

import torch

from . import api, synth
from .timing import time_all

KE = {torch.float32: 32, torch.bfloat16: 64, torch.float16: 64, torch.float8_e4m3fn: 128}
NAMES = {torch.float32: "f32", torch.bfloat16: "bf16", torch.float16: "f16",
         torch.float8_e4m3fn: "e4m3"}
# (type, tile) pairs calibrated; f16 shares bf16's constants (same kernels and rate)
SET = [(torch.float32, (128, 128)),
       (torch.bfloat16, (256, 256)), (torch.bfloat16, (256, 128)), (torch.bfloat16, (128, 128)),
       (torch.float8_e4m3fn, (256, 256)), (torch.float8_e4m3fn, (256, 128)),
       (torch.float8_e4m3fn, (128, 128)), (torch.float8_e4m3fn, (64, 128))]


def _operands(M, N, K, dtype, dev):
    name = NAMES[dtype]
    if name == "e4m3":
        a, _ = synth.fp8_scaled(synth.normal((M, K), 91))
        b, _ = synth.fp8_scaled(synth.normal((K, N), 92))
    else:
        a = synth.round_to(synth.normal((M, K), 91), name)
        b = synth.round_to(synth.normal((K, N), 92), name)
    A, _, _ = synth.place(a, col_major=False, device=dev)
    B, _, _ = synth.place(b, col_major=True, device=dev)
    return A, B


def measure(dtype, tile, reps, dev, ws):
    """Times (us) of the calibration launches of one type and tile."""
    BM, BN = tile
    ke = KE[dtype]
    runs = {}
    # (name, tiles down, tiles across, I, mode)
    plan = [("A8", 16, 16, 8, "dp"), ("A32", 16, 16, 32, "dp"), ("A64", 16, 16, 64, "dp"),
            ("B8", 8, 8, 8, "dp"), ("B32", 8, 8, 32, "dp"), ("B64", 8, 8, 64, "dp"),
            ("C32", 32, 16, 32, "dp"),
            ("D64", 8, 16, 64, "sk"), ("E64", 8, 8, 64, "sk"), ("F64", 15, 16, 64, "sk"),
            ("G32", 16, 16, 32, "dp")]
    legs, fns = [], []
    for name, tm, tn, I, mode in plan:
        M, N, K = tm * BM, tn * BN, I * ke
        A, B = _operands(M, N, K, dtype, dev)
        out = torch.empty((M, N), device=dev)
        cfg = api.Config(tile=tile, mode=mode, num_cu=256, min_iters=1)
        info = api.plan([(M, N, K)], dtype, cfg)
        beta = 0.5 if name.startswith("G") else 0.0
        legs.append((name, M, N, K, info))
        fns.append((lambda A, B, out, cfg, beta: (
            lambda: api.gemm(A, B, out if beta else None, beta=beta, out=out, config=cfg,
                             workspace=ws)))(A, B, out, cfg, beta))
    # every launch of the set timed together: the rounds interleave them, so
    # clock drift under the power limit hits all alike
    times = time_all(fns, reps)
    for (name, M, N, K, info), t in zip(legs, times):
        runs[name] = {"us": t * 1e3, "M": M, "N": N, "K": K, "T": info["T"], "S": info["S"],
                      "g": info["g"], "q": info["q"]}
    return runs


# Critical-path composition of each calibration launch in the model's terms:
# coefficients of (t_launch, t_tile, t_it(256), t_it(64), t_store, t_peer,
# l2 * t_it(256), t_cin).  D and E: one segment per workgroup, the finisher
# waits for its peers' stores; F: a PARTIAL then a FINISH segment per
# workgroup; C: two waves.
ROWS = {"A8": [1, 1, 8, 0, 0, 0, 0, 0], "A32": [1, 1, 32, 0, 0, 0, 0, 0],
        "A64": [1, 1, 64, 0, 0, 0, 0, 0], "B8": [1, 1, 0, 8, 0, 0, 0, 0],
        "B32": [1, 1, 0, 32, 0, 0, 0, 0], "B64": [1, 1, 0, 64, 0, 0, 0, 0],
        "C32": [1, 2, 64, 0, 0, 0, 0, 0], "D64": [1, 1, 32, 0, 1, 1, 0, 0],
        "E64": [1, 1, 16, 0, 1, 3, 0, 0], "F64": [1, 2, 60, 0, 1, 1, 60, 0],
        "G32": [1, 1, 32, 0, 0, 0, 0, 1]}


def solve(r):
    """Constants of the model from one (type, tile)'s launches: non-negative
    least squares on the relative error of every launch."""
    import numpy as np
    from scipy.optimize import nnls
    names = list(ROWS)
    A = np.array([ROWS[n] for n in names], dtype=float)
    y = np.array([r[n]["us"] for n in names])
    x, _ = nnls(A / y[:, None], np.ones(len(y)))
    tl, tt, tf, tli, ts, tp, xl, tc = (float(v) for v in x)
    pred = A @ x
    return {"t_launch": tl, "t_tile": tt, "t_it_full": tf, "t_it_light": tli, "t_store": ts,
            "t_peer": tp, "l2": xl / tf if tf > 0 else 0.0, "t_cin": tc,
            "max_rel_err": float(np.max(np.abs(pred - y) / y))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--out", default="")
    a = ap.parse_args()
    dev = torch.device("cuda", 0)
    ws = api.Workspace(dev)
    ws.get(96 << 20, torch.cuda.current_stream().cuda_stream)
    res = []
    for dtype, tile in SET:
        r = measure(dtype, tile, a.reps, dev, ws)
        c = solve(r)
        res.append({"dtype": NAMES[dtype], "tile": list(tile), "runs": r, "constants": c})
        print(f"# {NAMES[dtype]} {tile[0]}x{tile[1]}: " +
              " ".join(f"{k}={v:.4f}" for k, v in c.items()), file=sys.stderr, flush=True)
    rows = []
    for e in res:
        c = e["constants"]
        dt = {"f32": 0, "bf16": 2, "e4m3": 3}[e["dtype"]]
        rows.append(f"    {{{dt}, {e['tile'][0]}, {e['tile'][1]}, {c['t_launch']:.3f}f, "
                    f"{c['t_tile']:.3f}f, {c['t_it_full']:.4f}f, {c['t_it_light']:.4f}f, "
                    f"{c['t_store']:.3f}f, {c['t_peer']:.3f}f, {c['l2']:.4f}f, "
                    f"{c['t_cin']:.3f}f}},")
    text = json.dumps(res)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text + "\n")
    print(text)
    print("\n".join(rows), file=sys.stderr)


if __name__ == "__main__":
    main()
