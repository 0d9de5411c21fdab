"""AddressSanitizer and UndefinedBehaviorSanitizer on the CPU: the FP64 oracle
(every decoder, option and dump, through tests/sanitize/oracle_driver.c) and
the host side of the C ABI (handles, validation, sizing and error paths,
through tests/sanitize/abi_host_driver.c), each built with the sanitizers and
run with leak detection.  The library's device code is compiled as usual; the
sanitizers instrument host code only."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
SAN = ROOT / "tests" / "sanitize"
CSRC = ROOT / "paper_2305_05286_amd" / "csrc"
ENV = {**os.environ, "ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0",
       "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(map(str, cmd))}\n{r.stdout}\n{r.stderr}"
    return r


def test_oracle_under_asan_ubsan(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    exe = tmp_path / "oracle_san"
    run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fno-omit-frame-pointer",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         str(SAN / "oracle_driver.c"), str(ROOT / "oracle" / "cbp_oracle.c"), "-lm", "-o", str(exe)])
    r = run([str(exe)], env=ENV)
    assert "oracle driver: ok" in r.stdout


def test_abi_host_side_under_asan_ubsan(tmp_path):
    from paper_2305_05286_amd import build
    clang = Path("/opt/rocm/llvm/bin/clang")
    if not (Path(build.HIPCC).exists() and clang.exists()):
        pytest.skip("ROCm toolchain not available")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = [f for f in build.FLAGS if f != "-O3"] + ["-O1", "-g"]

    def compile_one(src):
        obj = tmp_path / (Path(src).stem + ".o")
        run([build.HIPCC, *flags, *san, "-c", str(CSRC / src), "-o", str(obj)])
        return obj

    with ThreadPoolExecutor(max_workers=len(build.SOURCES)) as ex:
        objs = list(ex.map(compile_one, build.SOURCES))
    drv = tmp_path / "drv.o"
    run([str(clang), "-O1", "-g", "-fsanitize=address,undefined", f"-I{ROOT / 'include'}",
         "-c", str(SAN / "abi_host_driver.c"), "-o", str(drv)])
    exe = tmp_path / "abi_san"
    run([str(clang) + "++", "-fsanitize=address,undefined", str(drv), *map(str, objs),
         "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", str(exe)])
    r = run([str(exe)], env=ENV)
    assert "abi host driver: ok" in r.stdout
