"""Register budget of the built kernels, read from the compiler's
resource-usage remarks that the build writes beside the objects: the
kernels of every tile below 256x256 must not spill, and the 16-bit and e4m3
256x256 kernels must keep to the few spills they have outside the MAC loop.
A kernel change that raises register pressure elsewhere in the kernel shows
up here before it shows up as a slowdown."""
import glob
import os
import re

import pytest

BUILD = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "_build")


def _spills():
    files = glob.glob(os.path.join(BUILD, "sk_inst_*.resources.txt"))
    if not files:
        pytest.skip("no build remarks (run the build first)")
    out = {}
    for f in files:
        name = None
        for line in open(f):
            m = re.search(r"Function Name: (\S+)", line)
            if m:
                name = m.group(1)
            m = re.search(r"VGPRs Spill: (\d+)", line)
            if m and name:
                out[name] = int(m.group(1))
    return out


def _cfg(name):
    # ..._ZN2sk14sk_gemm_kernelINS_3CfgILi<DT>ELi<LA>ELi<LB>ELi<BM>ELi<BN>ELi<WGM>ELi<NW>EEEEE...
    return tuple(int(x) for x in re.findall(r"Li(\d+)E", name)[:7])


def test_no_spills_below_256x256():
    for name, n in _spills().items():
        dt, la, lb, bm, bn, wgm, nw = _cfg(name)
        if (bm, bn) != (256, 256):
            assert n == 0, (name, n)


def test_16bit_256x256_spill_budget():
    for name, n in _spills().items():
        dt, la, lb, bm, bn, wgm, nw = _cfg(name)
        if (bm, bn) == (256, 256) and dt in (1, 2):
            assert n <= 40, (name, n)


def test_e4m3_256x256_spill_budget():
    # e4m3 on 256x256: a step's fragments take 48 registers beside the 128
    # of the accumulators; with two steps in flight the layouts read through
    # transposing LDS reads spilled 122-440 registers inside the MAC loop,
    # so those read each step just before its MFMAs
    for name, n in _spills().items():
        dt, la, lb, bm, bn, wgm, nw = _cfg(name)
        if (bm, bn) == (256, 256) and dt == 3:
            assert n <= 70, (name, n)
