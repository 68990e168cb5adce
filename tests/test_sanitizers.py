"""AddressSanitizer and UndefinedBehaviorSanitizer builds, run on the CPU: the FP64 oracle
(gcc) on small problems of every kind, and the host-only paths of the C-ABI (hipcc with the
sanitizers on the host side only; no call reaches the device). CPU only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
OBJDIR = os.path.join(ROOT, "paper_1512_01383_amd", "_build")
SAN_HOST = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined"]


def _run(exe, env_extra):
    env = dict(os.environ, **env_extra)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr
    return r.stdout


def test_oracle_under_asan_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_san")
    cmd = [gcc, "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-D_GNU_SOURCE", "-fopenmp", "-Wall",
           "-Werror=incompatible-pointer-types", "-Werror=implicit-function-declaration",
           *SAN_HOST, "-I", os.path.join(ROOT, "oracle"), os.path.join(HERE, "oracle_driver.c"),
           os.path.join(ROOT, "oracle", "oracle.c"), "-lm", "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    out = _run(exe, {"ASAN_OPTIONS": "detect_leaks=1", "UBSAN_OPTIONS": "print_stacktrace=1",
                     "OMP_NUM_THREADS": "2"})
    assert "oracle sanitizer run ok" in out


def test_c_abi_host_paths_under_asan_ubsan(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc"
    clang = "/opt/rocm/llvm/bin/clang"
    objs = [os.path.join(OBJDIR, n) for n in ("pdhg_iter.o", "aux.o", "adjoint.o", "steps.o", "stereo.o", "temporal.o")]
    if not (os.path.exists(hipcc) and os.path.exists(clang) and all(os.path.exists(o) for o in objs)):
        pytest.skip("needs hipcc and the objects of a library build (run build() first)")
    from paper_1512_01383_amd import build as B
    host_san = [a for f in SAN_HOST for a in ("-Xarch_host", f)]
    capi_o = str(tmp_path / "capi_san.o")
    subprocess.run([hipcc, *B.HIPCC_FLAGS, *host_san, "-g", "-c",
                    os.path.join(ROOT, "paper_1512_01383_amd", "csrc", "capi.hip"), "-o", capi_o],
                   check=True, capture_output=True)
    drv_o = str(tmp_path / "abi_driver.o")
    subprocess.run([clang, "-std=c11", "-O1", "-g", *SAN_HOST, "-I", os.path.join(ROOT, "include"), "-c",
                    os.path.join(HERE, "abi_driver.c"), "-o", drv_o], check=True, capture_output=True)
    exe = str(tmp_path / "abi_san")
    subprocess.run([hipcc, f"--offload-arch={B.ARCH}", *host_san, drv_o, capi_o, *objs, "-o", exe],
                   check=True, capture_output=True)
    # the HIP runtime itself is not instrumented: its allocations are left out of the leak check
    out = _run(exe, {"ASAN_OPTIONS": "detect_leaks=0", "UBSAN_OPTIONS": "print_stacktrace=1"})
    assert "abi sanitizer run ok" in out
