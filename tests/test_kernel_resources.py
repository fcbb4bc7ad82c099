"""Every kernel of the library compiles for gfx950 without spills to memory.

A spilled vector register lives in scratch memory, and scratch accesses
share the in-order completion counter with the kernels' global loads and
stores: one spill inside a batch loop makes every batch wait on it. Scalar
registers the compiler runs short of are kept in lanes of a vector register
instead (v_writelane / v_readlane, no memory), which is allowed as long as
no scratch memory is used. The compiler's per-kernel resource remarks give
the counts; this test compiles each source for the device only (no GPU
needed) and checks them.
"""
import concurrent.futures as cf
import os
import re
import subprocess

import pytest

from paper_1803_11449_amd import build as lib_build

pytestmark = pytest.mark.slow


def resource_remarks(src):
    """{kernel: {field: value}} from hipcc's kernel-resource-usage remarks."""
    cmd = [lib_build._hipcc(), *lib_build.HIPCC_FLAGS, "--offload-device-only",
           "-Rpass-analysis=kernel-resource-usage", "-c", os.path.join(lib_build.CSRC, src),
           "-o", os.devnull]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    out, cur = {}, None
    for line in res.stderr.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            cur = out.setdefault(m.group(1), {})
            continue
        m = re.search(r"remark:\s+(VGPRs Spill|SGPRs Spill|ScratchSize \[bytes/lane\]|VGPRs|"
                      r"Occupancy \[waves/SIMD\]): (\d+)", line)
        if m and cur is not None:
            cur[m.group(1).split(" [")[0]] = int(m.group(2))
    return out


@pytest.mark.skipif(not os.path.exists(lib_build._hipcc()), reason="hipcc not installed")
def test_no_kernel_spills():
    with cf.ThreadPoolExecutor(max_workers=len(lib_build.SOURCES)) as ex:
        found = dict(zip(lib_build.SOURCES, ex.map(resource_remarks, lib_build.SOURCES)))
    kernels = {k: v for per in found.values() for k, v in per.items()}
    # the hot kernels are all there, with their remarks
    for name in ("k_bin_count", "k_bin_scatter", "k_bin_apply", "k_bin_merge", "k_join",
                 "k_hot_scan_lez", "k_update"):
        assert any(name in k for k in kernels), name
    assert all("VGPRs Spill" in v and "ScratchSize" in v for v in kernels.values())
    bad = {k: v for k, v in kernels.items() if v["VGPRs Spill"] or v["ScratchSize"]}
    assert not bad, bad
    # the capped count instantiations keep 8 waves per SIMD
    for r, ppt in ((5, 6), (5, 5), (4, 6), (7, 4)):
        name = f"_ZN4ddhf11k_bin_countILi{r}ELi{ppt}EEEvPKNS_6UpdJobEj"
        assert kernels[name]["Occupancy"] == 8, (r, ppt, kernels[name])
