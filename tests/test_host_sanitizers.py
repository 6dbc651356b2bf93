"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the
CPU: the oracle (every entry point, through tests/hostbuild/oracle_driver.c)
and the library's host-side code (argument checks, variant tables, defaults,
the mean-mode recommendation, through tests/hostbuild/abi_driver.cpp).  The
library is compiled host-only (no device image): the driver calls only paths
that return before any kernel launch, so the device-image symbols the host
objects reference are never used (the link leaves them unresolved)."""
import concurrent.futures as cf
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HB = os.path.join(ROOT, "tests", "hostbuild")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (cmd, r.stdout[-2000:], r.stderr[-4000:])
    return r


def test_oracle_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if not gcc:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_driver")
    o = os.path.join(ROOT, "oracle")
    _run([gcc, "-O1", "-g", "-std=c11", "-D_POSIX_C_SOURCE=200809L", *SAN, "-I", o, "-o", exe,
          os.path.join(HB, "oracle_driver.c"), *(os.path.join(o, f) for f in
                                                 ("planck.c", "opacity.c", "solve.c")),
          "-lm", "-lpthread"])
    r = _run([exe], env=dict(ENV, ASAN_OPTIONS="detect_leaks=1"))
    assert "oracle driver: ok" in r.stdout


def test_library_host_code_under_sanitizers(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc"
    clang = "/opt/rocm/llvm/bin/clang++"
    if not (os.path.exists(hipcc) and os.path.exists(clang)):
        pytest.skip("hipcc / clang++ not available")
    from paper_2407_18304_amd import build as B
    inc = os.path.join(ROOT, "include")
    srcs = [os.path.join(B.CSRC, s) for s in B.LIBS["libmgrhd.so"]]

    def host_obj(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _run([hipcc, "--offload-arch=gfx950", "--offload-host-only", "-O1", "-g", "-std=c++17",
              "-fPIC", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
              "-fsanitize=undefined", "-fno-omit-frame-pointer", "-I", inc, "-c", "-o", obj, src])
        return obj

    with cf.ThreadPoolExecutor(8) as ex:
        objs = list(ex.map(host_obj, srcs))
    drv = str(tmp_path / "abi_driver.o")
    _run([clang, "-O1", "-g", "-std=c++17", *SAN, "-I", inc, "-c", "-o", drv,
          os.path.join(HB, "abi_driver.cpp")])
    exe = str(tmp_path / "abi_driver")
    _run([clang, *SAN, "-o", exe, drv, *objs, "-L/opt/rocm/lib", "-lamdhip64",
          "-Wl,-rpath,/opt/rocm/lib", "-Wl,--unresolved-symbols=ignore-all"])
    r = _run([exe], env=ENV, timeout=120)
    assert "abi driver: ok" in r.stdout
