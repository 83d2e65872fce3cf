"""The library's host code under AddressSanitizer, on the CPU.

The three host sources are compiled with g++ and -fsanitize=address (the
kernels are linked from the normal build, uninstrumented) into a small
program, tests/host_asan/sg_host_checks.cpp, that drives the C interface
without a GPU: workspace queries over the option space, every rejected
argument, and the host table building of sg_setup, sg_batch_setup and
sg_logn_setup up to their first HIP call, which must fail with SG_EDEVICE.
Leak detection is on. Skipped where a HIP device is present."""

import concurrent.futures as cf
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ROCM = "/opt/rocm"
HOST_SOURCES = ("sg_capi.cpp", "sg_batch.cpp", "sg_lognormal.cpp")
CXXFLAGS = ["-std=c++17", "-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer",
            "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include", f"-I{os.path.join(ROOT, 'include')}"]


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, f"{' '.join(cmd)}\n{res.stdout}\n{res.stderr}"


def test_host_code_under_address_sanitizer(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.exists(f"{ROCM}/lib/libamdhip64.so"):
        pytest.skip("g++ or the HIP runtime is missing")
    from paper_1205_1864_amd import build as bld
    if not bld.built_from_current_sources():
        bld.build()
    kernels = sorted(os.path.join(bld.BUILD, os.path.basename(p) + ".o")
                     for p in bld._sources() if p.endswith(".hip"))
    assert kernels and all(os.path.exists(k) for k in kernels)
    srcs = [os.path.join(bld.CSRC, f) for f in HOST_SOURCES]
    srcs.append(os.path.join(HERE, "host_asan", "sg_host_checks.cpp"))
    objs = [str(tmp_path / (os.path.basename(s) + ".o")) for s in srcs]
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        list(ex.map(lambda so: _run([gxx, *CXXFLAGS, "-c", so[0], "-o", so[1]]), zip(srcs, objs)))
    exe = str(tmp_path / "sg_host_checks")
    _run([gxx, "-fsanitize=address", "-o", exe, *objs, *kernels, f"-L{ROCM}/lib", "-lamdhip64",
          f"-Wl,-rpath,{ROCM}/lib"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    if res.returncode == 77:
        pytest.skip("a HIP device is present: the checks hand the library host buffers as workspace")
    assert res.returncode == 0, res.stdout[-4000:] + res.stderr[-4000:]
    assert "0 failures" in res.stdout and "AddressSanitizer" not in res.stderr
