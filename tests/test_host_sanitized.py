"""The library's host logic under AddressSanitizer and UBSan, without a GPU:
the C ABI's sources are compiled with the sanitizers on their host code only
(device code is compiled as usual and never runs here), linked with the
robustness driver tests/host_abi_fuzz.c, and fed seeded random and damaged
arguments: header parsing, size and workspace queries, relative bounds, batch
job validation, and the argument checks and launch preparation of
compression, decompression and the field range.  Every call must return and
the sanitizers must report nothing."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2508_10305_amd", "csrc")
SOURCES = ("api", "batch", "encode", "decode", "aux", "generic")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"


@pytest.fixture(scope="module")
def fuzz_exe(tmp_path_factory):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm compilers not found")
    d = str(tmp_path_factory.mktemp("host_sanitized"))
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    san_host = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=undefined"]

    def compile_one(name):
        obj = os.path.join(d, name + ".o")
        cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
               "-ffp-contract=off", *san_host, "-Xclang", "-target-feature", "-Xclang",
               "-packed-fp32-ops", *inc, "-c", os.path.join(CSRC, name + ".hip"), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stderr[-3000:]
        return obj

    with ThreadPoolExecutor(max_workers=min(6, os.cpu_count() or 1)) as pool:
        objs = list(pool.map(compile_one, SOURCES))
    drv = os.path.join(d, "host_abi_fuzz.o")
    r = subprocess.run([CLANG, "-O1", "-g", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=undefined", *inc, "-c",
                        os.path.join(ROOT, "tests", "host_abi_fuzz.c"), "-o", drv],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-3000:]
    exe = os.path.join(d, "host_abi_fuzz")
    r = subprocess.run([CLANG + "++", "-fsanitize=address,undefined", "-o", exe, drv, *objs,
                        "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-3000:]
    yield exe
    shutil.rmtree(d, ignore_errors=True)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_host_entry_points_are_memory_safe(fuzz_exe, seed):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([fuzz_exe, str(seed), "300"], capture_output=True, text=True, timeout=300,
                       env=env)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    assert "300 cases" in r.stdout
