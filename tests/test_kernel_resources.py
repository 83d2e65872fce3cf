"""Register budget of the hot kernels, from the compiler's resource report (CPU).

A code change that pushes the inner PCG's banded tiles or the row-staged SG
operator into spilling vector registers to scratch memory costs far more than
any arithmetic it saves (a sweep that spilled 134 to 198 registers ran the
inner solves 2.6 times slower). The kernels are compiled for gfx950 exactly as
the library build does and their reported VGPR spills and scratch sizes are
held to the current budget."""

import os
import re
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

# kernel name pattern -> (max VGPR spills, max scratch bytes per lane)
BUDGET = {
    "k_pcg.hip": {
        r"pcg_kernelIdNS0_8BandTileIdLi128ELi15ELi16EEELi1ELb0E": (12, 64),
        r"pcg_kernelIfNS0_8BandTileIfLi256ELi15ELi16EEELi1ELb0E": (12, 64),
        r"pcg_kernelIdNS0_8BandTileIdLi64ELi15ELi16EEELi1ELb0E": (12, 64),
        r"pcg_kernelIfNS0_8BandTileIfLi128ELi15ELi16EEELi1ELb0E": (12, 64),
    },
    "k_sgop.hip": {
        r"sgop_stage_kernel": (4, 32),
    },
}


def _report(src):
    from paper_1205_1864_amd import build as bld
    cmd = [bld.hipcc(), *bld.COMMON, "-x", "hip", "-c", os.path.join(bld.CSRC, src), "-o", os.devnull,
           "-Rpass-analysis=kernel-resource-usage"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    kernels, cur = {}, None
    for line in res.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            kernels[cur] = {}
            continue
        m = re.search(r"remark:\s+([A-Za-z ]+?)(?: \[bytes/lane\])?: (\d+)", line)
        if cur and m:
            kernels[cur][m.group(1).strip()] = int(m.group(2))
    return kernels


@pytest.mark.parametrize("src", sorted(BUDGET))
def test_hot_kernels_within_register_budget(src):
    if shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("hipcc not found")
    kernels = _report(src)
    for pat, (max_spill, max_scratch) in BUDGET[src].items():
        hits = [k for k in kernels if re.search(pat, k)]
        assert hits, f"no kernel matches {pat}"
        for k in hits:
            r = kernels[k]
            assert r.get("VGPRs Spill", 0) <= max_spill and r.get("ScratchSize", 0) <= max_scratch, (k, r)
