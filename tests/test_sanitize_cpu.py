"""CPU: the FP64 oracle and the host side of the library built under
AddressSanitizer and UndefinedBehaviorSanitizer, each driven by a small
program (tests/sanitize/) over random cases and the argument checks.  The
library's host code (api.hip) is compiled with the sanitizers on the host
side only and linked with the device objects of the regular build; the
driver makes no call that reaches the HIP runtime, so no GPU is needed."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="verify_asan_link_order=0:detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, cwd):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0, f"{' '.join(cmd)} failed ({r.returncode}):\n{r.stdout[-2000:]}\n{r.stderr[-4000:]}"
    return r


def test_oracle_under_asan_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    exe = str(tmp_path / "oracle_asan")
    _run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-Wall",
          os.path.join(SAN, "oracle_driver.c"), os.path.join(ROOT, "oracle", "stkde_oracle.c"), "-lm", "-o", exe],
         str(tmp_path))
    r = _run([exe], str(tmp_path))
    assert "cases ok" in r.stdout


def test_library_host_code_under_asan_ubsan(tmp_path):
    from paper_1705_09366_amd import build as B
    objdir = os.path.join(ROOT, "paper_1705_09366_amd", "_build")
    others = [os.path.join(objdir, s + ".o") for s in B.SOURCES if s != "api.hip"]
    if not all(os.path.exists(o) for o in others):
        pytest.fail("the library's objects are missing: run __graft_entry__.build() first")
    cc = B.hipcc()
    # sanitizers on the host side only (each -fsanitize= after -Xarch_host)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all"]
    api = str(tmp_path / "api.o")
    drv = str(tmp_path / "drv.o")
    exe = str(tmp_path / "host_asan")
    _run([cc, "-O1", "-g", "-std=c++20", f"--offload-arch={B.ARCH}", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops", *san, "-I", os.path.join(ROOT, "include"), "-I", B.CSRC, "-c",
          os.path.join(B.CSRC, "api.hip"), "-o", api], str(tmp_path))
    _run([cc, "-O1", "-g", "-std=c++20", *san, "-I", os.path.join(ROOT, "include"), "-c",
          os.path.join(SAN, "host_driver.cpp"), "-o", drv], str(tmp_path))
    _run([cc, f"--offload-arch={B.ARCH}", *san, drv, api, *others, "-o", exe], str(tmp_path))
    r = _run([exe], str(tmp_path))
    assert "ok" in r.stdout
