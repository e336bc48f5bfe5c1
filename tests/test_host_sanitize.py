"""The library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU: tests/host_fuzz/fuzz_host.cpp
includes the host source, feeds seeded random pools (well-formed and
mutated) to the pool validation and random forward maps (rotations,
anisotropic and extreme scales, singular ones) to the frame-table builder,
and checks every return code.  A sanitizer report aborts the program."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host_fuzz", "fuzz_host.cpp")
HIP_INC = "/opt/rocm/include"
HIP_LIB = "/opt/rocm/lib"


@pytest.fixture(scope="module")
def fuzz_bin(tmp_path_factory):
    if not shutil.which("g++") or not os.path.isdir(HIP_INC) or not os.path.exists(os.path.join(HIP_LIB, "libamdhip64.so")):
        pytest.skip("g++ or the HIP runtime headers / library are not available")
    out = str(tmp_path_factory.mktemp("fuzz") / "fuzz_host")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-D__HIP_PLATFORM_AMD__", "-I", HIP_INC,
           "-I", os.path.join(ROOT, "paper_1911_06001_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-Wno-subobject-linkage", SRC, "-o", out, "-L", HIP_LIB, "-lamdhip64", "-Wl,-rpath," + HIP_LIB]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=300)
    return out


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_host_code_is_clean_under_sanitizers(fuzz_bin, seed):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    p = subprocess.run([fuzz_bin, str(seed), "3000"], capture_output=True, text=True, timeout=300, env=env)
    assert p.returncode == 0, p.stdout + p.stderr
    fields = dict(zip(p.stdout.split()[0::2], map(int, p.stdout.split()[1::2])))
    # both well-formed and malformed pools were seen, and tables were built
    assert fields["accepted"] > 1000 and fields["rejected"] > 100 and fields["tables"] > 1000, p.stdout
    assert fields["candidates"] > 1000, p.stdout
