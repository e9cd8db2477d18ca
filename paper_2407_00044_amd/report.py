"""Timings of the other workloads of record, beside the FP16 3840x4096x4096
headline of bench.py: FP32 512^3 split over 256 workgroups, the 64-shape
BF16 sweep (min and geometric mean per schedule), the BF16 linear
layer's forward, dX and dW products, the 48-problem FP8 grouped GEMM
(tile and schedule from the autotuner), and the headline shape in each input
type with its MFMA peak.
Each Stream-K launch is timed against its data-parallel comparator with
graph replays (warm-up, rotated order, median; see timing.time_all).

Inputs are drawn on the GPU with torch's seeded generator in the recipes'
distributions (timing only; the parity tests use synth.py's FP64 draws).

    python -m paper_2407_00044_amd.report [--extra]

--extra adds the report's two experiments on MI355X: the padding ablation of
Table 1 and Stream-K throughput against the "Compute Units" count, and the
data-parallel + Stream-K split variants (two-tile rule, one-tile remainder,
all Stream-K, auto, data-parallel).
"""
import json
import sys

import torch

from . import api, synth, tune
from .timing import time_all as _time_all


def _normal(shape, seed, dev):
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    return torch.randn(shape, generator=g, device=dev)


def _uniform(shape, seed, dev):
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    return torch.rand(shape, generator=g, device=dev) * 2 - 1


def _tf(flops, ms):
    return round(flops / ms / 1e9, 2)


def c1(dev, reps=20):
    """FP32 512^3, A and B row-major, 128x128x32 tiles, all Stream-K over 256
    workgroups (16 tiles, 16 contributors each) vs the 16-workgroup grid."""
    A = _uniform((512, 512), 1, dev)
    B = _uniform((512, 512), 2, dev)
    out = torch.empty((512, 512), device=dev)
    ws = api.Workspace(dev)
    ws.get(64 << 20, torch.cuda.current_stream().cuda_stream)
    cfgs = {"sk_g256": api.Config(tile=(128, 128), mode="sk", num_cu=256, min_iters=1),
            "auto": api.Config(tile=(128, 128), mode="auto"),
            "dp": api.Config(tile=(128, 128), mode="dp")}
    fns = [(lambda c: (lambda: api.gemm(A, B, out=out, config=c, workspace=ws)))(c)
           for c in cfgs.values()]
    ts = _time_all(fns, reps)
    fl = 2.0 * 512 ** 3
    return {"workload": "fp32 512x512x512, A and B row-major, 128x128x32 tiles",
            **{k: {"us": round(t * 1e3, 2), "tflops": _tf(fl, t)} for k, t in zip(cfgs, ts)}}


def c4(dev, reps=5):
    """BF16 linear layer Y = X W^T, X [8192, 4096], W [11008, 4096], dY
    [8192, 11008]: forward (A row, B col), dX = dY W (A row, B row) and
    dW = dY^T X (A col, B row), each Stream-K (auto) vs data-parallel at the
    default tile on the operands as laid out, and the two backward products
    on K-contiguous copies as the linear layer makes them (copies timed)."""
    X = _normal((8192, 4096), 4, dev).to(torch.bfloat16)
    W = _normal((11008, 4096), 5, dev).to(torch.bfloat16)
    dY = _normal((8192, 11008), 40, dev).to(torch.bfloat16)
    ws = api.Workspace(dev)
    ws.get(96 << 20, torch.cuda.current_stream().cuda_stream)
    res = {"workload": "bf16 linear layer X[8192,4096] W[11008,4096], FP32 products"}
    for name, A, B in [("forward", X, W.t()), ("dX", dY, W), ("dW", dY.t(), X)]:
        M, K = A.shape
        N = B.shape[1]
        tile = api.default_tile(M, N, K, torch.bfloat16)
        out = torch.empty((M, N), device=dev)
        cfgs = [api.Config(tile=tile, mode="auto"), api.Config(tile=tile, mode="dp")]
        t_sk, t_dp = _time_all([(lambda c: (lambda: api.gemm(A, B, out=out, config=c,
                                                                workspace=ws)))(c)
                                for c in cfgs], reps)
        fl = 2.0 * M * N * K
        p = api.plan([(M, N, K)], torch.bfloat16, cfgs[0])
        res[name] = {"M": M, "N": N, "K": K, "tile": list(tile), "stream_k_tiles": p["S"],
                     "tiles": p["T"], "sk_tflops": _tf(fl, t_sk), "dp_tflops": _tf(fl, t_dp)}
        if name != "forward":
            # the backward as StreamKLinearFn runs it at this size: K-contiguous
            # copies (sk_transpose) of the M- or N-major operands, then the
            # same auto GEMM; the copies' time is included
            def packed(c=cfgs[0]):
                api.gemm(api.k_contiguous(A, "a"), api.k_contiguous(B, "b"), out=out, config=c,
                         workspace=ws)
            (t_pk,) = _time_all([packed], reps)
            res[name]["packed_tflops"] = _tf(fl, t_pk)
            res[name]["packed_by_linear"] = api.pack_pays(M, N, K, torch.bfloat16)
        del out
    return res


def c5(dev, reps=5, tile=None):
    """48 FP8-e4m3 problems (synth.grouped_shapes), per-tensor amax scales,
    FP32 outputs: one grouped Stream-K launch vs one grouped data-parallel
    launch vs 48 separate data-parallel launches, equal tiles.  The grouped
    launch's tile and schedule come from the autotuner (tune.tune_grouped)
    unless `tile` is given (then auto mode on that tile)."""
    shapes = synth.grouped_shapes()
    probs, scales = [], []
    for i, (M, N, K) in enumerate(shapes):
        a = _normal((M, K), 500 + i, dev)
        b = _normal((N, K), 1500 + i, dev)
        sa = float(a.abs().max()) / 448.0
        sb = float(b.abs().max()) / 448.0
        A = (a / sa).to(torch.float8_e4m3fn)
        B = (b / sb).to(torch.float8_e4m3fn).t()          # K x N, column-major
        probs.append((A, B, torch.empty((M, N), device=dev)))
        scales.append((sa, sb))
    if tile is None:
        cfg = tune.tune_grouped(probs, scales=scales, reps=3)
        tuned = tune.config_to_dict(cfg)
    else:
        cfg, tuned = api.Config(tile=tile, mode="auto"), None
    cfg_dp = api.Config(tile=cfg.tile, mode="dp")
    g_sk = api.GroupedGemm(probs, config=cfg, scales=scales)
    g_dp = api.GroupedGemm(probs, config=cfg_dp, scales=scales)
    ws = api.Workspace(dev)
    ws.get(64 << 20, torch.cuda.current_stream().cuda_stream)

    def separate():
        for (A, B, out), (sa, sb) in zip(probs, scales):
            api.gemm(A, B, out=out, scale_a=sa, scale_b=sb, config=cfg_dp, workspace=ws)
    t_sk, t_gdp, t_sep = _time_all([g_sk.run, g_dp.run, separate], reps)
    fl = sum(2.0 * M * N * K for M, N, K in shapes)
    # roofline time: each problem at the FP8 MFMA peak or at HBM bandwidth
    # for its operands and FP32 output, whichever is slower
    t_roof = sum(max(2.0 * M * N * K / 5033.2e12, (M * K + K * N + 4 * M * N) / 8.0e12)
                 for M, N, K in shapes) * 1e3
    info = g_sk.info()
    # the persistent launch splits tiles only when the schedule gives it
    # Stream-K tiles; with S = 0 its gain over the grouped data-parallel
    # grid is whole-tile dealing alone
    leg = "grouped_stream_k" if info["S"] > 0 else "grouped_persistent_whole_tiles"
    return {"workload": "48 fp8-e4m3 problems, M log-uniform [16,4096], N in {1024,2048,4096}, "
                        "K in {2048,4096,8192}", "tile": list(cfg.tile), "config": tuned,
            "gflop": round(fl / 1e9, 1), "tiles": info["T"], "stream_k_tiles": info["S"],
            "persistent_leg": leg,
            f"{leg}_tflops": _tf(fl, t_sk), "grouped_dp_tflops": _tf(fl, t_gdp),
            "separate_dp_tflops": _tf(fl, t_sep), "roofline_us": round(t_roof * 1e3, 1),
            f"{leg}_frac_of_roofline": round(t_roof / t_sk, 4)}


def c3(dev, reps=10):
    """The 64-shape BF16 sweep (sweep.run): min and geometric-mean TFLOP/s of
    the auto policy, the two-tile hybrid and the data-parallel grid, the
    worst shape of each, and one compact row per shape."""
    import io
    from . import sweep
    buf = io.StringIO()
    sweep.run(n=64, reps=reps, out=buf)
    d = json.loads(buf.getvalue())
    sm, rows = d["summary"], d["rows"]

    def worst(key):
        r = min(rows, key=lambda r: r[key])
        return {"shape": f"{r['M']}x{r['N']}x{r['K']}", "tflops": round(r[key], 2),
                "dp_tflops": round(r["dp_tflops"], 2)}
    ratio = [r["sk_tflops"] / r["dp_tflops"] for r in rows]
    hyr = [r["hybrid_tflops"] / r["dp_tflops"] for r in rows]
    i_auto = min(range(len(rows)), key=lambda i: ratio[i])
    i_hy = min(range(len(rows)), key=lambda i: hyr[i])
    return {"workload": "64 bf16 shapes, M,N log-uniform [128,8192], K log-uniform [128,16384] "
                        "(seed 3), A row-major, B column-major, N(0,1), beta=0.5 with C_in "
                        "U[-1,1], FP32 C, default tile per shape, graph-timed",
            "auto_min": round(sm["sk_min"], 2), "auto_geomean": round(sm["sk_geomean"], 2),
            "hybrid_min": round(sm["hybrid_min"], 2),
            "hybrid_geomean": round(sm["hybrid_geomean"], 2),
            "dp_min": round(sm["dp_min"], 2), "dp_geomean": round(sm["dp_geomean"], 2),
            "geomean_t_dp_over_t_auto": round(sm["geomean_t_dp_over_t_sk"], 4),
            "worst_auto": worst("sk_tflops"), "worst_hybrid": worst("hybrid_tflops"),
            "worst_dp": worst("dp_tflops"),
            "worst_auto_over_dp": {"shape": "{M}x{N}x{K}".format(**rows[i_auto]),
                                   "ratio": round(ratio[i_auto], 4),
                                   "stream_k_tiles": rows[i_auto]["S"]},
            "worst_hybrid_over_dp": {"shape": "{M}x{N}x{K}".format(**rows[i_hy]),
                                     "ratio": round(hyr[i_hy], 4)},
            "shapes_split_by_auto": sum(1 for r in rows if r["S"] > 0),
            "auto_geomean_frac_of_roofline": round(sm["sk_geomean_frac_of_roofline"], 4),
            "model": {"median_abs_err": round(sm["model_median_abs_err"], 4),
                      "p90_abs_err": round(sm["model_p90_abs_err"], 4),
                      "shapes_with_split_candidate": sm["model_shapes_with_split_candidate"],
                      "choice_was_faster": sm["model_choice_was_faster"],
                      "choice_faster_or_within_2pct": sm["model_choice_faster_or_within_2pct"]},
            "rows": [[r["M"], r["N"], r["K"], f"{r['tile'][0]}x{r['tile'][1]}", r["S"],
                      round(r["sk_tflops"], 1), round(r["hybrid_tflops"], 1),
                      round(r["dp_tflops"], 1), round(r["hybrid_us"], 2),
                      round(r["pred_hybrid_us"], 2), round(r["dp_us"], 2),
                      round(r["pred_dp_us"], 2)] for r in rows],
            "row_fields": ["M", "N", "K", "tile", "auto_stream_k_tiles", "auto", "hybrid",
                           "dp", "hybrid_us", "predicted_hybrid_us", "dp_us",
                           "predicted_dp_us"]}


PEAK = {torch.float32: 157.3, torch.float16: 2516.6, torch.bfloat16: 2516.6,
        torch.float8_e4m3fn: 5033.2}      # dense MFMA TFLOP/s at 2.4 GHz


def per_dtype(dev, reps=5, shape=(3840, 4096, 4096)):
    """The headline shape in every input type (A row-major, B column-major,
    FP32 output), default tile: Stream-K (two-tile hybrid), the auto policy
    and the data-parallel grid, with each type's dense MFMA peak."""
    M, N, K = shape
    ws = api.Workspace(dev)
    ws.get(96 << 20, torch.cuda.current_stream().cuda_stream)
    out = torch.empty((M, N), device=dev)
    fl = 2.0 * M * N * K
    res = {"workload": f"{M}x{N}x{K}, A row-major, B column-major, FP32 output"}
    for dt in (torch.float32, torch.float16, torch.bfloat16, torch.float8_e4m3fn):
        a = _uniform((M, K), 7, dev)
        b = _uniform((N, K), 8, dev)
        A = a.to(dt)
        B = b.to(dt).t()
        tile = api.default_tile(M, N, K, dt)
        cfgs = {"stream_k": api.Config(tile=tile, mode="hybrid"),
                "auto": api.Config(tile=tile, mode="auto"),
                "dp": api.Config(tile=tile, mode="dp")}
        ts = _time_all([(lambda c: (lambda: api.gemm(A, B, out=out, config=c, workspace=ws)))(c)
                        for c in cfgs.values()], reps)
        row = {"tile": list(tile)}
        for n, t in zip(cfgs, ts):
            row[n] = {"tflops": _tf(fl, t), "pct_peak": round(100 * fl / t / 1e9 / PEAK[dt], 2)}
        res[str(dt).split(".")[-1]] = row
        del A, B
    return res


def mxfp8(dev, reps=5, shape=(3840, 4096, 4096), tile=(256, 128)):
    """MXFP8 (e4m3 elements with an E8M0 scale per 32 K-values, applied by
    the matrix cores) at the headline shape, beside MXFP8 with e5m2
    elements and plain e4m3 with per-tensor scales on the same tile:
    Stream-K (two-tile hybrid), the auto policy and the data-parallel grid;
    % of the dense FP8 MFMA peak."""
    M, N, K = shape
    ws = api.Workspace(dev)
    ws.get(96 << 20, torch.cuda.current_stream().cuda_stream)
    qa, sa = synth.mx_quantize(synth.normal((M, K), 61))
    qb, sb = synth.mx_quantize(synth.normal((N, K), 62))
    A, B = qa.to(dev), qb.to(dev).t()
    SA, SB = torch.from_numpy(sa).to(dev), torch.from_numpy(sb).to(dev)
    qa5, sa5 = synth.mx_quantize(synth.normal((M, K), 61), elem="e5m2")
    qb5, sb5 = synth.mx_quantize(synth.normal((N, K), 62), elem="e5m2")
    A5, B5 = qa5.to(dev), qb5.to(dev).t()
    SA5, SB5 = torch.from_numpy(sa5).to(dev), torch.from_numpy(sb5).to(dev)
    out = torch.empty((M, N), device=dev)
    fl = 2.0 * M * N * K
    cfgs = {"stream_k": api.Config(tile=tile, mode="hybrid"),
            "auto": api.Config(tile=tile, mode="auto"),
            "dp": api.Config(tile=tile, mode="dp")}
    fns = [(lambda c: (lambda: api.gemm_mx(A, B, SA, SB, out=out, config=c, workspace=ws)))(c)
           for c in cfgs.values()]
    fns += [(lambda c: (lambda: api.gemm(A, B, out=out, config=c, workspace=ws)))(c)
            for c in cfgs.values()]
    fns += [(lambda c: (lambda: api.gemm_mx(A5, B5, SA5, SB5, out=out, config=c,
                                            workspace=ws)))(c) for c in cfgs.values()]
    ts = _time_all(fns, reps)
    res = {"workload": f"{M}x{N}x{K}, A row-major, B column-major, FP32 output, tile "
                       f"{tile[0]}x{tile[1]}", "mxfp8": {}, "mxfp8_e5m2": {},
           "e4m3_per_tensor": {}}
    for i, n in enumerate(cfgs):
        for key, t in (("mxfp8", ts[i]), ("e4m3_per_tensor", ts[i + 3]),
                       ("mxfp8_e5m2", ts[i + 6])):
            res[key][n] = {"tflops": _tf(fl, t), "pct_peak": round(100 * fl / t / 1e9 / 5033.2, 2)}
    return res


def mxfp4(dev, reps=5, shape=(3840, 4096, 4096), tile=(256, 128)):
    """MXFP4 (E2M1 elements two per byte, an E8M0 scale per 32 K-values,
    applied by the matrix cores) at the headline shape on the same tile as
    the MXFP8 leg: Stream-K (two-tile hybrid), the auto policy and the
    data-parallel grid; % of the dense FP4 MFMA peak (10.1 PFLOP/s)."""
    M, N, K = shape
    ws = api.Workspace(dev)
    ws.get(96 << 20, torch.cuda.current_stream().cuda_stream)
    pa, sa = synth.mx4_quantize(synth.normal((M, K), 63))
    pb, sb = synth.mx4_quantize(synth.normal((N, K), 64))
    A, B = torch.from_numpy(pa).to(dev), torch.from_numpy(pb).to(dev).t()
    SA, SB = torch.from_numpy(sa).to(dev), torch.from_numpy(sb).to(dev)
    out = torch.empty((M, N), device=dev)
    fl = 2.0 * M * N * K
    cfgs = {"stream_k": api.Config(tile=tile, mode="hybrid"),
            "auto": api.Config(tile=tile, mode="auto"),
            "dp": api.Config(tile=tile, mode="dp")}
    fns = [(lambda c: (lambda: api.gemm_mx4(A, B, SA, SB, out=out, config=c, workspace=ws)))(c)
           for c in cfgs.values()]
    ts = _time_all(fns, reps)
    res = {"workload": f"{M}x{N}x{K}, A row-major, B column-major, FP32 output, tile "
                       f"{tile[0]}x{tile[1]}"}
    for n, t in zip(cfgs, ts):
        res[n] = {"tflops": _tf(fl, t), "pct_peak": round(100 * fl / t / 1e9 / 10066.3, 2)}
    return res


def mxfp6(dev, reps=5, shape=(3840, 4096, 4096), tile=(256, 128)):
    """MXFP6 (E2M3 and E3M2 elements, 24 bytes per 32, an E8M0 scale per
    32 K-values, applied by the matrix cores) at the headline shape on the
    MX tile: Stream-K (two-tile hybrid), the auto policy and the
    data-parallel grid; % of the dense FP6 MFMA peak (10.1 PFLOP/s)."""
    M, N, K = shape
    ws = api.Workspace(dev)
    ws.get(96 << 20, torch.cuda.current_stream().cuda_stream)
    out = torch.empty((M, N), device=dev)
    fl = 2.0 * M * N * K
    res = {"workload": f"{M}x{N}x{K}, A row-major, B column-major, FP32 output, tile "
                       f"{tile[0]}x{tile[1]}"}
    for fmt in ("e2m3", "e3m2"):
        pa, sa = synth.mx6_quantize(synth.normal((M, K), 65), fmt)
        pb, sb = synth.mx6_quantize(synth.normal((N, K), 66), fmt)
        A, B = torch.from_numpy(pa).to(dev), torch.from_numpy(pb).to(dev).t()
        SA, SB = torch.from_numpy(sa).to(dev), torch.from_numpy(sb).to(dev)
        cfgs = {"stream_k": api.Config(tile=tile, mode="hybrid"),
                "auto": api.Config(tile=tile, mode="auto"),
                "dp": api.Config(tile=tile, mode="dp")}
        fns = [(lambda c: (lambda: api.gemm_mx6(A, B, SA, SB, fmt=fmt, out=out, config=c,
                                                workspace=ws)))(c) for c in cfgs.values()]
        ts = _time_all(fns, reps)
        res[fmt] = {n: {"tflops": _tf(fl, t), "pct_peak": round(100 * fl / t / 1e9 / 10066.3, 2)}
                    for n, t in zip(cfgs, ts)}
        del A, B
    return res


def epilogue(dev, reps=5, shape=(3840, 4096, 4096), tile=(256, 256)):
    """Cost of the fused epilogue (bias per column, then ReLU / GELU / SiLU)
    on BF16 at the headline shape, auto policy: the plain GEMM, each fused
    variant, and the plain GEMM followed by torch's own bias and GELU passes
    over C (the unfused alternative: one more read and write of C)."""
    M, N, K = shape
    ws = api.Workspace(dev)
    ws.get(96 << 20, torch.cuda.current_stream().cuda_stream)
    A = _uniform((M, K), 2, dev).bfloat16()
    B = _uniform((N, K), 3, dev).bfloat16().t()
    bias = _uniform((1, N), 4, dev)[0].float().contiguous()
    out = torch.empty((M, N), device=dev)
    fl = 2.0 * M * N * K
    cfg = api.Config(tile=tile, mode="auto")

    def fused(act, b=bias):
        return lambda: api.gemm(A, B, out=out, bias=b, activation=act, config=cfg, workspace=ws)

    def unfused():
        api.gemm(A, B, out=out, config=cfg, workspace=ws)
        torch.nn.functional.gelu(out.add_(bias), approximate="none")

    legs = {"plain": fused("none", None), "bias": fused("none"), "bias_relu": fused("relu"),
            "bias_gelu": fused("gelu"), "bias_silu": fused("silu"),
            "plain_then_torch_bias_gelu": unfused}
    ts = _time_all(list(legs.values()), reps)
    res = {"workload": f"BF16 {M}x{N}x{K}, A row-major, B column-major, FP32 output, "
                       f"tile {tile[0]}x{tile[1]}, auto"}
    for n, t in zip(legs, ts):
        res[n] = {"ms": round(t, 4), "tflops": _tf(fl, t)}
    return res


def packing(dev, reps=5):
    """Operand packing: GEMMs with M- or N-major operands (A M-major and/or
    B N-major) as laid out (transposing LDS reads) and on K-contiguous
    copies made by sk_transpose (copies included), BF16 and e4m3, auto mode
    on the default tile, beside what the packing rule (pack_pays) decides."""
    ws = api.Workspace(dev)
    ws.get(96 << 20, torch.cuda.current_stream().cuda_stream)
    shapes = [(1024, 1024, 1024), (2048, 2048, 2048), (1024, 4096, 4096), (4096, 1024, 4096),
              (4096, 4096, 1024), (2048, 4096, 8192), (4096, 4096, 4096), (8192, 8192, 2048)]
    res = {"workload": "A row or col, B row or col (not both K-contiguous), auto, default tile"}
    for dt in (torch.bfloat16, torch.float8_e4m3fn):
        name = "bf16" if dt == torch.bfloat16 else "e4m3"
        rows = []
        for M, N, K in shapes:
            a = _uniform((M, K), 11, dev)
            b = _uniform((K, N), 12, dev)
            cfg = api.Config(tile=api.default_tile(M, N, K, dt), mode="auto")
            out = torch.empty((M, N), device=dev)
            for la, lb in (("row", "row"), ("col", "row"), ("col", "col")):
                A = (a if la == "row" else a.t().contiguous().t()).to(dt)
                B = (b.t().contiguous().t() if lb == "col" else b).to(dt)
                t0, t1 = _time_all([
                    lambda: api.gemm(A, B, out=out, config=cfg, workspace=ws),
                    lambda: api.gemm(A, B, out=out, config=cfg, workspace=ws, pack=True)], reps)
                rows.append({"shape": f"{M}x{N}x{K}", "layout": la[0] + lb[0],
                             "tile": list(cfg.tile), "as_laid_us": round(t0 * 1e3, 1),
                             "packed_us": round(t1 * 1e3, 1), "speedup": round(t0 / t1, 3),
                             "rule_packs": api.pack_pays(M, N, K, dt)})
                del A, B
            del out
            torch.cuda.empty_cache()
        res[name] = rows
    return res


def padding(dev, reps=10, tile=(256, 128)):
    """The report's padding experiment (Methodology, Results, Table 1) on
    FP16: each shape run unpadded (edges through out-of-range loads and
    dropped stores) and on copies zero-padded to tile multiples in M, N and
    K (every tile full); TFLOP/s counts the unpadded 2MNK in both."""
    out = {"tile": list(tile), "schedule": "hybrid"}
    ws = api.Workspace(dev)
    ws.get(96 << 20, torch.cuda.current_stream().cuda_stream)
    bk = 64
    for M, N, K in [(3840, 4096, 4096), (1920, 2000, 2000), (480, 512, 512)]:
        Mp = -(-M // tile[0]) * tile[0]
        Np = -(-N // tile[1]) * tile[1]
        Kp = -(-K // bk) * bk
        A = _uniform((M, K), 2, dev).half()
        Bt = _uniform((N, K), 3, dev).half()
        Ap = torch.zeros((Mp, Kp), device=dev, dtype=torch.half)
        Ap[:M, :K] = A
        Bp = torch.zeros((Np, Kp), device=dev, dtype=torch.half)
        Bp[:N, :K] = Bt
        o = torch.empty((M, N), device=dev)
        op = torch.empty((Mp, Np), device=dev)
        cfg = api.Config(tile=tile, mode="hybrid")
        t_u, t_p = _time_all([lambda: api.gemm(A, Bt.t(), out=o, config=cfg, workspace=ws),
                              lambda: api.gemm(Ap, Bp.t(), out=op, config=cfg, workspace=ws)],
                             reps)
        fl = 2.0 * M * N * K
        out[f"{M}x{N}x{K}"] = {"padded_to": [Mp, Np, Kp], "unpadded_us": round(t_u * 1e3, 2),
                              "padded_us": round(t_p * 1e3, 2), "unpadded_tflops": _tf(fl, t_u),
                              "padded_tflops": _tf(fl, t_p),
                              "no_padding_gain_pct": round(100 * (t_p / t_u - 1), 2)}
    return out


def compute_units(dev, reps=10):
    """The report's "Compute Units" argument: Stream-K (all tiles split, no
    grid floor) on FP16 3840x4096x4096 and 1920x2000x2000, 256x128 tiles,
    with g = 8 .. 256 workgroups (one per CU); the data-parallel grid beside
    it uses every CU."""
    ws = api.Workspace(dev)
    ws.get(96 << 20, torch.cuda.current_stream().cuda_stream)
    out = {}
    for M, N, K in [(3840, 4096, 4096), (1920, 2000, 2000)]:
        A = _uniform((M, K), 2, dev).half()
        Bt = _uniform((N, K), 3, dev).half()
        o = torch.empty((M, N), device=dev)
        gs = [8, 16, 32, 64, 120, 128, 192, 240, 256]
        cfgs = [api.Config(tile=(256, 128), mode="sk", num_cu=g, min_iters=1) for g in gs]
        cfgs.append(api.Config(tile=(256, 128), mode="dp"))
        ts = _time_all([(lambda c: (lambda: api.gemm(A, Bt.t(), out=o, config=c,
                                                       workspace=ws)))(c) for c in cfgs], reps)
        fl = 2.0 * M * N * K
        out[f"{M}x{N}x{K}"] = {"stream_k_tflops_by_cus": {str(g): _tf(fl, t) for g, t in
                                                          zip(gs, ts[:-1])},
                              "dp_tflops": _tf(fl, ts[-1])}
    return out


def hybrid_variants(dev, reps=10, tile=(256, 128)):
    """Data-parallel + Stream-K splits on FP16 (256 CUs): the two-tile rule
    (S = T mod g + g), the one-tile remainder (S = T mod g: Stream-K only for
    the last, partial wave), all tiles Stream-K, the auto policy and the
    data-parallel grid."""
    ws = api.Workspace(dev)
    ws.get(96 << 20, torch.cuda.current_stream().cuda_stream)
    cus, _ = api.device_query(api.Config(tile=tile), torch.float16)
    out = {"tile": list(tile)}
    for M, N, K in [(3840, 4096, 4096), (1920, 2000, 2000), (480, 512, 512)]:
        A = _uniform((M, K), 2, dev).half()
        Bt = _uniform((N, K), 3, dev).half()
        o = torch.empty((M, N), device=dev)
        T = -(-M // tile[0]) * -(-N // tile[1])
        cfgs = {"two_tile": api.Config(tile=tile, mode="hybrid"),
                "one_tile": api.Config(tile=tile, mode="hybrid", dp_tiles=T - T % cus),
                "all_stream_k": api.Config(tile=tile, mode="sk"),
                "auto": api.Config(tile=tile, mode="auto"),
                "dp": api.Config(tile=tile, mode="dp")}
        ts = _time_all([(lambda c: (lambda: api.gemm(A, Bt.t(), out=o, config=c,
                                                       workspace=ws)))(c) for c in cfgs.values()],
                       reps)
        fl = 2.0 * M * N * K
        row = {"tiles": T}
        for (name, c), t in zip(cfgs.items(), ts):
            row[name] = {"stream_k_tiles": api.plan([(M, N, K)], torch.float16, c)["S"],
                         "tflops": _tf(fl, t)}
        out[f"{M}x{N}x{K}"] = row
    return out


def run_all(dev, extra=False, only=None, c5_tile=None):
    """Every configuration (`extra` adds the experiments), or the named ones;
    c5_tile runs c5 in auto mode on that tile instead of the tuner's pick."""
    out = {}
    todo = [("c1", c1), ("c3", c3), ("c4", c4), ("c5", lambda d: c5(d, tile=c5_tile)),
            ("per_dtype", per_dtype), ("mxfp8", mxfp8), ("mxfp4", mxfp4), ("mxfp6", mxfp6),
            ("epilogue", epilogue)]
    if extra or only:
        todo += [("packing", packing), ("padding", padding), ("compute_units", compute_units),
                 ("hybrid_variants", hybrid_variants)]
    if only:
        unknown = set(only) - {n for n, _ in todo}
        if unknown:
            raise SystemExit(f"unknown configuration(s): {sorted(unknown)}")
        todo = [(n, f) for n, f in todo if n in only]
    for name, fn in todo:
        out[name] = fn(dev)
        print(f"# {name}: {json.dumps(out[name])}", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    return out


def main():
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--extra", action="store_true", help="also the report's experiments")
    ap.add_argument("--only", default="", help="comma-separated names, e.g. c1,c5")
    ap.add_argument("--c5-tile", default="", help="e.g. 128x128: no tuner for c5")
    a = ap.parse_args()
    only = [x for x in a.only.split(",") if x] or None
    tile = tuple(int(v) for v in a.c5_tile.split("x")) if a.c5_tile else None
    print(json.dumps(run_all(torch.device("cuda", 0), extra=a.extra, only=only,
                             c5_tile=tile)))


if __name__ == "__main__":
    main()
