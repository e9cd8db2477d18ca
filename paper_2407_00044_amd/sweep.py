"""Shape sweep (BF16 by default): Stream-K vs equal-tile data-parallel tiling.

64 shapes with M, N log-uniform in [128, 8192] and K log-uniform in
[128, 16384] (seeded); A row-major, B column-major with leading dimensions
rounded up to 16 bytes, N(0,1) entries, FP32 C_in uniform in [-1, 1],
alpha = 1, beta = 0.5.  Times are GPU times: `reps` launches are captured in
one HIP graph and replayed, so host-side call overhead (which exceeds the
kernel time of the smallest shapes) is not counted.  For each shape both
schedules use the same tile: the library's Stream-K policy ('auto': the
two-tile hybrid rule, splitting tiles only where its cost model predicts a
gain), the plain two-tile hybrid rule, and the data-parallel grid;
the report lists TFLOP/s = 2*M*N*K / t per shape, the min and geometric mean
of each schedule, the predicted quantization loss of one-tile-per-workgroup
tiling 1 - T / (ceil(T/g) * g) and the measured ratio t_DP / t_SK.

    python -m paper_2407_00044_amd.sweep [--n 64] [--reps 10] [--tune] [--all-tiles]
                                         [--dtype bf16|f16|f32|e4m3]

--dtype runs the same shapes with another input type (leading dimensions
rounded to 16 bytes of that type; e4m3 with unit scales); the per-shape
roofline then takes that type's dense MFMA peak.
--all-tiles also times every 256/128-row tile of the menu for the type under both schedules
and auto mode in row-major tile order (per-shape "tiles" entries), the data
behind the default-tile and tile-order rules.
--tune also runs the autotuner on each shape and reports the tuned best, and
how often the default (auto mode on the default tile) is within 3% of it.
"""
import argparse
import json
import math
import sys
import time

import torch

from . import api, synth, tune
from .timing import time_all as _time_all


def gmean(xs):
    return math.exp(sum(math.log(x) for x in xs) / len(xs))


ALL_TILES = [(256, 256), (256, 128), (128, 128)]


DTYPES = {"bf16": torch.bfloat16, "f16": torch.float16, "f32": torch.float32,
          "e4m3": torch.float8_e4m3fn}
ELEM = {torch.bfloat16: 2, torch.float16: 2, torch.float32: 4, torch.float8_e4m3fn: 1}
PEAK = {torch.bfloat16: 2516.6, torch.float16: 2516.6, torch.float32: 157.3,
        torch.float8_e4m3fn: 5033.2}


def run(n=64, reps=10, use_tuner=False, seed=3, out=sys.stdout, all_tiles=False,
        dtype=torch.bfloat16):
    dev = torch.device("cuda", torch.cuda.current_device())
    cus, _ = api.device_query(api.Config(tile=(128, 128)), dtype)
    rows = []
    ws = api.Workspace(dev)
    ws.get(96 << 20, torch.cuda.current_stream().cuda_stream)   # before any capture
    for idx, (M, N, K) in enumerate(synth.sweep_shapes(seed, n)):
        gen = torch.Generator(device=dev)
        gen.manual_seed(300 + idx)
        lda = synth.ld_aligned(K, ELEM[dtype])
        ldb = synth.ld_aligned(K, ELEM[dtype])
        A = torch.randn((M, lda), generator=gen, device=dev).to(dtype)[:, :K]
        B = torch.randn((N, ldb), generator=gen, device=dev).to(dtype)[:, :K].t()
        C = (torch.rand((M, N), generator=gen, device=dev) * 2 - 1)
        outC = torch.empty_like(C)
        tile = api.default_tile(M, N, K, dtype)
        cfg_sk = api.Config(tile=tile, mode="auto")
        cfg_hy = api.Config(tile=tile, mode="hybrid")
        cfg_dp = api.Config(tile=tile, mode="dp")

        def go(cfg):
            return lambda: api.gemm(A, B, C, beta=0.5, out=outC, config=cfg, workspace=ws)
        t_sk, t_hy, t_dp = _time_all([go(cfg_sk), go(cfg_hy), go(cfg_dp)], reps)
        p = api.plan([(M, N, K)], dtype, cfg_sk)
        # the launch-time model's predictions (Block2Time-style) beside the
        # measured times of the two launches the auto mode chooses between
        ph = api.plan([(M, N, K)], dtype, cfg_hy, beta=0.5)
        T = p["T"]
        q_eff = T / (math.ceil(T / cus) * cus)
        flops = 2.0 * M * N * K
        # per-shape roofline: the input type's dense MFMA peak or HBM
        # bandwidth (8 TB/s) for A, B, C_in and C_out (FP32), whichever bounds it
        e = ELEM[dtype]
        roof = min(PEAK[dtype], flops / (e * M * K + e * K * N + 8 * M * N) * 8.0)
        row = {"M": M, "N": N, "K": K, "tile": list(tile), "T": T, "S": p["S"],
               "roofline_tflops": roof,
               "sk_tflops": flops / t_sk / 1e9, "hybrid_tflops": flops / t_hy / 1e9,
               "dp_tflops": flops / t_dp / 1e9,
               "dp_quant_eff": q_eff, "t_dp_over_t_sk": t_dp / t_sk,
               "hybrid_us": t_hy * 1e3, "dp_us": t_dp * 1e3, "hybrid_S": ph["S"],
               "pred_hybrid_us": ph["predicted_us"], "pred_dp_us": ph["predicted_dp_us"]}
        if all_tiles:
            row["tiles"] = {}
            for t in [x[:2] for x in api.supported_tiles(dtype) if x[:2] in ALL_TILES]:
                key = f"{t[0]}x{t[1]}"
                ts, tr, td = _time_all([go(api.Config(tile=t, mode="auto")),
                                        go(api.Config(tile=t, mode="auto", group_m=0)),
                                        go(api.Config(tile=t, mode="dp"))], reps)
                pt = api.plan([(M, N, K)], dtype, api.Config(tile=t, mode="auto"))
                row["tiles"][key] = {"sk": flops / ts / 1e9, "sk_rowmajor": flops / tr / 1e9,
                                     "dp": flops / td / 1e9, "T": pt["T"], "S": pt["S"],
                                     "g": pt["g"], "group_m": pt["group_m"]}
        if use_tuner:
            best = tune.tune_gemm(A, B, torch.float32, reps=max(3, reps // 2))
            t_best = _time_all([go(best)], reps)[0]
            row["tuned"] = {"config": tune.config_to_dict(best), "tflops": flops / t_best / 1e9}
        rows.append(row)
        print(f"# {idx:2d} {M}x{N}x{K} tile {tile} T={T}: SK {row['sk_tflops']:.1f} "
              f"DP {row['dp_tflops']:.1f} TFLOP/s  (DP quant eff {q_eff:.3f})",
              file=sys.stderr, flush=True)
        del A, B, C, outC
    sk = [r["sk_tflops"] for r in rows]
    hy = [r["hybrid_tflops"] for r in rows]
    dp = [r["dp_tflops"] for r in rows]
    summary = {"shapes": len(rows), "sk_min": min(sk), "sk_geomean": gmean(sk),
               "dp_min": min(dp), "dp_geomean": gmean(dp),
               "hybrid_min": min(hy), "hybrid_geomean": gmean(hy),
               "sk_beats_dp_geomean": gmean(sk) > gmean(dp), "sk_beats_dp_min": min(sk) > min(dp),
               # the slowest shape often runs the identical DP launch in both legs
               "sk_min_over_dp_min": min(sk) / min(dp),
               "mean_predicted_quant_loss": sum(1 - r["dp_quant_eff"] for r in rows) / len(rows),
               "sk_geomean_frac_of_roofline": gmean([r["sk_tflops"] / r["roofline_tflops"]
                                                     for r in rows]),
               "dp_geomean_frac_of_roofline": gmean([r["dp_tflops"] / r["roofline_tflops"]
                                                     for r in rows]),
               "geomean_t_dp_over_t_sk": gmean([r["t_dp_over_t_sk"] for r in rows])}
    # the model against measurement: error of each predicted time, and how
    # often the auto mode's choice (split or not) was the faster launch
    errs = sorted([abs(r["pred_hybrid_us"] / r["hybrid_us"] - 1) for r in rows if r["hybrid_S"] > 0]
                  + [abs(r["pred_dp_us"] / r["dp_us"] - 1) for r in rows])
    cand = [r for r in rows if r["hybrid_S"] > 0]
    right = sum(1 for r in cand if (r["S"] > 0) == (r["hybrid_us"] < r["dp_us"]))
    near = sum(1 for r in cand if (r["S"] > 0) == (r["hybrid_us"] < r["dp_us"])
               or abs(r["hybrid_us"] / r["dp_us"] - 1) <= 0.02)
    summary.update({"model_median_abs_err": errs[len(errs) // 2] if errs else 0.0,
                    "model_p90_abs_err": errs[int(0.9 * (len(errs) - 1))] if errs else 0.0,
                    "model_shapes_with_split_candidate": len(cand),
                    "model_choice_was_faster": right,
                    "model_choice_faster_or_within_2pct": near})
    if use_tuner:
        tb = [r["tuned"]["tflops"] for r in rows]
        # the default policy (auto mode, default tile) against the tuned best
        ratio = [r["sk_tflops"] / r["tuned"]["tflops"] for r in rows]
        summary.update({"tuned_min": min(tb), "tuned_geomean": gmean(tb),
                        "default_within_3pct_of_tuned": sum(x >= 0.97 for x in ratio),
                        "geomean_default_over_tuned": gmean(ratio)})
    json.dump({"summary": summary, "rows": rows}, out)
    out.write("\n")
    return summary


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--tune", action="store_true")
    ap.add_argument("--all-tiles", action="store_true")
    ap.add_argument("--dtype", choices=sorted(DTYPES), default="bf16")
    a = ap.parse_args()
    t0 = time.time()
    run(a.n, a.reps, a.tune, all_tiles=a.all_tiles, dtype=DTYPES[a.dtype])
    print(f"# sweep done in {time.time() - t0:.1f} s", file=sys.stderr)


if __name__ == "__main__":
    main()
