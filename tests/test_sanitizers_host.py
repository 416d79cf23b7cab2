"""Address and undefined-behaviour sanitizers on the host code (no GPU):
the oracle (every routine on many small texts, cross-checked) and the
library's host side (sizing, binding, build planners, argument errors),
each built with -fsanitize=address,undefined and run to completion.
Device code is compiled as usual: the sanitizers apply to the host pass
only (-Xarch_host before each -fsanitize on the hipcc lines)."""
import glob
import os
import subprocess
import concurrent.futures as cf

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CLANG = "/opt/rocm/llvm/bin/clang++"
HIPCC = "/opt/rocm/bin/hipcc"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-2000:]}\n{r.stderr[-4000:]}"
    return r


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_checks")
    _run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "oracle"), "-o", exe,
          os.path.join(HERE, "oracle_checks.c"), os.path.join(ROOT, "oracle", "wt_oracle.c"),
          os.path.join(ROOT, "oracle", "wt_oracle_par.c")])
    r = _run([exe], env=dict(ENV, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", OMP_NUM_THREADS="4"),
             timeout=300)
    assert "oracle sanitizer checks ok" in r.stdout


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_library_host_side_under_sanitizers(tmp_path):
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_1702_07578_amd", "csrc", "*.hip")))
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer"]

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _run([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature",
              "-Xclang", "-packed-fp32-ops", *san, "-c", src, "-o", obj])
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(compile_one, srcs))
    drv = str(tmp_path / "drv.o")
    _run([CLANG, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-I", os.path.join(ROOT, "include"),
          "-I", "/opt/rocm/include", "-D__HIP_PLATFORM_AMD__", "-c", os.path.join(HERE, "host_abi_checks.cpp"),
          "-o", drv])
    exe = str(tmp_path / "host_abi_checks")
    _run([CLANG, "-fsanitize=address,undefined", "-o", exe, drv, *objs, "-L/opt/rocm/lib", "-lamdhip64",
          "-Wl,-rpath,/opt/rocm/lib"])
    r = _run([exe], env=ENV, timeout=300)
    assert "host sanitizer checks ok" in r.stdout
