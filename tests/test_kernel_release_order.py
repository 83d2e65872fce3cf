"""Release order of the inner solver's column arrivals, from the gfx950 assembly (CPU).

A block publishes a column phase by an L2 write-back (the device-scope release)
followed by an atomic add to the column's arrival counter. The write-back is a
memory operation of its own: unless the wave waits for it, the atomic can be
seen by another block before the data is in memory, and that block then reads
stale halo values or partial sums (wrong iterates, or owners of one column that
disagree on stopping). The compiler drops its wait after the write-back when
the wave has nothing else outstanding, so the kernel states the wait itself;
this test holds every write-back of every instantiation to it."""

import os
import re
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_every_l2_writeback_is_waited_for_before_the_arrival():
    if shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("hipcc not found")
    from paper_1205_1864_amd import build as bld
    cmd = [bld.hipcc(), *bld.COMMON, "-x", "hip", "--cuda-device-only", "-S", "-o", "-",
           os.path.join(bld.CSRC, "k_pcg.hip")]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    lines = res.stdout.splitlines()
    sites, missing = 0, []
    for i, line in enumerate(lines):
        if "buffer_wbl2" not in line:
            continue
        sites += 1
        waited = False
        for nxt in lines[i + 1:i + 80]:
            if re.search(r"s_waitcnt\b.*vmcnt\(0\)", nxt):
                waited = True
                break
            if "global_atomic" in nxt or "s_endpgm" in nxt:
                break
        if not waited:
            missing.append(i)
    assert sites > 0, "no device-scope release found in the inner solver"
    assert not missing, f"{len(missing)} of {sites} L2 write-backs reach an atomic unwaited (lines {missing[:5]})"
