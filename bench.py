"""Benchmark: Stream-K vs data-parallel tiling on one MI355X.

Workload (one step = one GEMM through the whole Stream-K path): FP16 inputs
with FP32 accumulation and FP32 output, M=3840, N=4096, K=4096, A row-major,
B column-major, entries uniform in [-1, 1] (seeded), alpha=1, beta=0,
256x128 tiles, hybrid data-parallel + Stream-K schedule over one persistent
workgroup per CU.  The same shape is also timed with the equal-tile
data-parallel grid, and in BF16 with 256x256 tiles.

Prints one JSON line.  TFLOP/s = 2*M*N*K / time.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"f16": 2516.6, "bf16": 2516.6, "e4m3": 5033.2, "f32": 157.3}
HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--only", default="", help="run only this leg (sk|dp|bf16)")
    return ap.parse_args()


def make_operands(M, N, K, dtype, seed, device):
    import torch
    from paper_2407_00044_amd import synth
    a = synth.round_to(synth.uniform((M, K), seed), dtype)
    b = synth.round_to(synth.uniform((K, N), seed + 1), dtype)
    A, sa, lda = synth.place(a, col_major=False, device=device)
    B, sb, ldb = synth.place(b, col_major=True, device=device)
    torch.cuda.synchronize()
    return A, B, (sa, lda, sb, ldb)


def time_gemm(A, B, cfg, steps, warmup):
    """Average per-launch time (ms) over `steps` back-to-back launches,
    measured with HIP events recorded on the stream the kernels run on."""
    import torch
    import paper_2407_00044_amd as sk
    out = torch.empty((A.shape[0], B.shape[1]), dtype=torch.float32, device=A.device)
    for _ in range(warmup):
        sk.gemm(A, B, out=out, config=cfg)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        sk.gemm(A, B, out=out, config=cfg)
    end.record(stream)
    torch.cuda.synchronize()
    assert sk.check_device_error() == 0
    return start.elapsed_time(end) / steps, out


def cpu_baseline(host, M, N, K, rows=24):
    """The FP64 oracle on a bounded row sample of the same product."""
    import numpy as np
    from oracle import gemm as og
    from paper_2407_00044_amd import synth
    sa, lda, sb, ldb = host
    a = og.decode_f16(synth.codes(sa.cpu()))
    b = og.decode_f16(synth.codes(sb.cpu()))
    sel = np.arange(rows, dtype=np.int64) * (M // rows)
    og.gemm(M, N, K, a, lda, False, b, ldb, True, rows=sel[:2])   # warm
    t0 = time.perf_counter()
    og.gemm(M, N, K, a, lda, False, b, ldb, True, rows=sel)
    dt = time.perf_counter() - t0
    flops = 2.0 * rows * N * K
    return {"value": round(flops / dt / 1e12, 6), "unit": "TFLOP/s", "cores": og.num_threads(),
            "kind": "oracle",
            "sample": f"{rows} of {M} output rows ({rows}x{N}x{K} MACs), FP64 triple loop, "
                      f"{dt:.2f} s wall"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(every run of this build uses a single MI355X)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2407_00044_amd as sk

    dev = torch.device("cuda", 0)
    M, N, K = 3840, 4096, 4096
    flops = 2.0 * M * N * K
    cus, _ = sk.device_query(sk.Config(tile=(256, 128)), torch.float16)
    A, B, host = make_operands(M, N, K, "f16", 2, dev)

    cfg_sk = sk.Config(tile=(256, 128), mode="hybrid", num_cu=0)
    cfg_dp = sk.Config(tile=(256, 128), mode="dp")
    result = {}
    legs = [("sk", A, B, cfg_sk), ("dp", A, B, cfg_dp)]
    for name, a, b, cfg in legs:
        if args.only and args.only != name:
            continue
        ms, _ = time_gemm(a, b, cfg, args.steps, args.warmup)
        result[name] = ms
        print(f"# {name}: {ms * 1e3:.1f} us  {flops / ms / 1e9:.1f} TFLOP/s", file=sys.stderr,
              flush=True)
    bf = {}
    if not args.only or args.only == "bf16":
        Ab, Bb, _ = make_operands(M, N, K, "bf16", 4, dev)
        for name, cfg in [("sk_256x256", sk.Config(tile=(256, 256), mode="hybrid")),
                          ("dp_256x256", sk.Config(tile=(256, 256), mode="dp")),
                          ("sk_256x128", sk.Config(tile=(256, 128), mode="hybrid"))]:
            ms, _ = time_gemm(Ab, Bb, cfg, args.steps, args.warmup)
            bf[name] = {"ms": round(ms, 5), "tflops": round(flops / ms / 1e9, 1),
                        "frac_peak": round(flops / ms / 1e9 / PEAK_TFLOPS["bf16"], 4)}
            print(f"# bf16 {name}: {ms * 1e3:.1f} us  {flops / ms / 1e9:.1f} TFLOP/s",
                  file=sys.stderr, flush=True)
    if args.only and args.only != "sk":
        print(json.dumps({"partial": True, "bf16": bf, **result}))
        return

    ms = result["sk"]
    tflops = flops / ms / 1e9
    line = {
        "metric": "TFLOP/s & % MFMA peak: Stream-K vs data-parallel tiling, same GPU, per dtype",
        "value": round(tflops, 2),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16",
        "data": "synthetic",
        "config": {"workload": "fp16 GEMM 3840x4096x4096, A row-major, B column-major, "
                               "U[-1,1], FP32 accumulate and output, alpha=1 beta=0",
                   "M": M, "N": N, "K": K, "tile": [256, 128, 64], "schedule": "hybrid",
                   "persistent_workgroups": cus, "parallelism": "single GPU"},
        "pct_mfma_peak": round(100 * tflops / PEAK_TFLOPS["f16"], 2),
        "roofline": {"bound": "mfma", "achieved": round(tflops, 2),
                     "peak": PEAK_TFLOPS["f16"], "unit": "TFLOP/s",
                     "frac": round(tflops / PEAK_TFLOPS["f16"], 4), "traffic": None},
    }
    if "dp" in result:
        dtf = flops / result["dp"] / 1e9
        line["dp_baseline"] = {"ms": round(result["dp"], 5), "tflops": round(dtf, 2),
                               "pct_mfma_peak": round(100 * dtf / PEAK_TFLOPS["f16"], 2),
                               "sk_speedup": round(result["dp"] / ms, 4)}
    if bf:
        line["bf16_same_shape"] = bf
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(host, M, N, K)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
