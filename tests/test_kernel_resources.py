"""Every device kernel of the library compiles without register spills
(no scratch memory), with the library's own compile flags for gfx950.  The
BF16x3 kernels' occupancy (three 256-thread workgroups, one 512-thread
workgroup and four 256-thread workgroups per CU for the Pi build's 128 x 128
and 256 x 256 forms and the W^c contraction) depends on their register
counts staying below 168, 256 and 128 VGPRs; those are checked too.  Cross-compiles with hipcc; no GPU needed."""
import concurrent.futures as cf
import importlib.util
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _build_module():
    spec = importlib.util.spec_from_file_location(
        "gw_build", os.path.join(ROOT, "paper_2107_10423_amd", "build.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def _resources(src, flags, hipcc):
    with tempfile.TemporaryDirectory() as d:
        cmd = [hipcc, *flags, "--cuda-device-only", "-c", src, "-o", os.path.join(d, "k.o"),
               "-Rpass-analysis=kernel-resource-usage"]
        r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    out, name = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            out[name] = {}
            continue
        m = re.search(r"remark:\s+(VGPRs|ScratchSize \[bytes/lane\]|VGPRs Spill): (\d+)", line)
        if m and name:
            out[name][m.group(1)] = int(m.group(2))
    return out


@pytest.fixture(scope="module")
def kernels():
    b = _build_module()
    if not os.path.exists(b.HIPCC):
        pytest.skip("hipcc not available")
    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        parts = list(ex.map(lambda s: _resources(s, b.FLAGS, b.HIPCC), b.sources()))
    res = {}
    for p in parts:
        res.update(p)
    return res


def test_no_kernel_uses_scratch(kernels):
    assert len(kernels) > 20
    bad = {k: v for k, v in kernels.items()
           if v.get("ScratchSize [bytes/lane]", 0) or v.get("VGPRs Spill", 0)}
    assert not bad, bad


def test_bf16x3_kernels_keep_their_occupancy(kernels):
    vg = {k: v["VGPRs"] for k, v in kernels.items() if "bf16x3" in k}
    pi = [v for k, v in vg.items() if "k_pi_bf16x3" in k and "wide" not in k]
    wide = [v for k, v in vg.items() if "k_pi_bf16x3_wide" in k]
    wc = [v for k, v in vg.items() if "k_wc_bf16x3" in k and "wide" not in k]
    wcw = [v for k, v in vg.items() if "k_wc_bf16x3_wide" in k]
    assert pi and wc and wide and wcw
    assert max(pi) <= 168, vg      # three 256-thread workgroups per CU
    assert max(wide + wcw) <= 256, vg   # one 512-thread workgroup (two wavefronts per SIMD)
    assert max(wc) <= 128, vg      # four
