"""The emulation harness built with AddressSanitizer and
UndefinedBehaviorSanitizer (host code: the device headers compiled by the
host compiler behind the stand-in hip/hip_runtime.h), run as a separate
executable: products of several schedule classes, a staged class, the
Toeplitz tile and the sparse barrel equal the C oracle, with no sanitizer
report (the LDS stand-in has each kernel's exact LDS size, so an access past
it is a heap overflow)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_emulation_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "emu_asan")
    emu = os.path.join(ROOT, "tests", "emu")
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
    oracle_o = str(tmp_path / "oracle.o")
    subprocess.check_call(["/opt/rocm/llvm/bin/clang", "-O1", "-g", "-std=c99", "-c"] + san +
                          [os.path.join(ROOT, "oracle", "gf2x_oracle.c"), "-o", oracle_o])
    subprocess.check_call(["/opt/rocm/llvm/bin/clang++", "-O1", "-g", "-std=c++17", "-pthread",
                           "-Wno-unknown-pragmas"] + san +
                          ["-I", emu, "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_2201_10473_amd", "csrc"),
                           os.path.join(emu, "emu.cpp"), os.path.join(emu, "asan_main.cpp"), oracle_o, "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    proc = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, env=env, timeout=1200)
    print(proc.stdout[-3000:])
    assert proc.returncode == 0, proc.stdout[-3000:]
    assert "ALL OK" in proc.stdout
    assert "ERROR: AddressSanitizer" not in proc.stdout and "runtime error" not in proc.stdout
