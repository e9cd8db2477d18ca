"""The benchmark's measurement conventions against the numbers the report
prints (CPU only; tests/golden/paper_numbers.json).

* Table 1 (Results section): each row's TFLOP/s equals 2*M*N*K over its
  time, and its GB/s equals A, B and C counted once at 2 bytes an element
  over its time, both within the rounding of the printed ms (0.4%);
* the arithmetic intensity quoted in the Methodology section ("1337") is
  the same flop count over the same bytes at 3840x4096x4096 (1335.65);
* the report's Figure 1 utilisation (Background section): 9 equal tiles on
  4 cores keep 75% of the core slots busy.
"""
import json
import os

from paper_2407_00044_amd import metrics

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                   "paper_numbers.json")))


def test_table1_tflops_and_gbs_conventions():
    for row in GOLD["table1"]:
        M, N, K, ms = row["M"], row["N"], row["K"], row["ms"]
        tf = metrics.tflops(metrics.gemm_flops(M, N, K), ms)
        assert abs(tf / row["tflops"] - 1) < 4e-3, (row["label"], tf)
        gb = metrics.gbs(M, N, K, ms)
        assert abs(gb / row["gbs"] - 1) < 4e-3, (row["label"], gb)
    # a dropped factor of two in the flop count or bytes counted at 4 bytes
    # would be far outside that band
    row = GOLD["table1"][0]
    assert abs(metrics.tflops(row["M"] * row["N"] * row["K"], row["ms"]) / row["tflops"]
               - 1) > 0.4


def test_arithmetic_intensity_closed_form():
    ai = GOLD["arithmetic_intensity"]
    v = metrics.arithmetic_intensity(ai["M"], ai["N"], ai["K"])
    assert abs(v - 1335.65) < 0.01
    assert abs(v / ai["printed"] - 1) < 2e-3


def test_figure1_utilisation():
    f = GOLD["figure1_dp_utilisation"]
    assert metrics.dp_efficiency(f["tiles"], f["cores"]) == f["utilisation"]
    # the headline workload: 480 tiles of 256x128 on 256 CUs in two waves
    assert metrics.dp_efficiency(480, 256) == 0.9375
