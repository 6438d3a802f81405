"""Host AddressSanitizer and UndefinedBehaviorSanitizer runs (CPU only).

Two native parts run on the host and are checked here with the sanitizers
(the device code is never instrumented):

- the oracle's C core (oracle/pa_oracle.c), built with gcc's sanitizers and
  driven by tests/sanitize_oracle_driver.c over ragged inputs; its hash of
  every result must equal that of an uninstrumented -O2 build;
- libpa's host code, built with the library's own flags plus host-side
  sanitizers and driven by tests/sanitize_libpa_driver.cpp in its host mode:
  configuration checks, workspace layouts, creation failures and NULL handles,
  none of which needs a device.

Run as a script, this file builds the instrumented libpa driver into a
directory, for the driver's device mode (every entry point on small runs and
batches) on a GPU machine:

    python tests/test_host_sanitizers.py <dir>
    ASAN_OPTIONS=detect_leaks=0 <dir>/sanitize_libpa_driver device
"""
import concurrent.futures
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

ORACLE_C = os.path.join(ROOT, "oracle", "pa_oracle.c")
ORACLE_DRIVER = os.path.join(HERE, "sanitize_oracle_driver.c")
LIBPA_DRIVER = os.path.join(HERE, "sanitize_libpa_driver.cpp")

# gcc / clang++ lines for host-only code (no .hip file on them)
GCC_SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
# hipcc lines: every sanitizer flag applies to the host side only
HIP_HOST_SANITIZE = [
    "-Xarch_host", "-g",
    "-Xarch_host", "-fsanitize=address",
    "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-sanitize-recover=all",
    "-Xarch_host", "-fno-omit-frame-pointer",
]
SAN_ENV = {
    "ASAN_OPTIONS": "detect_leaks=1:exitcode=23",
    "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1:exitcode=24",
}


def _run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    if r.returncode != 0:
        raise RuntimeError("%s failed (%d):\n%s\n%s" % (" ".join(cmd), r.returncode, r.stdout,
                                                        r.stderr))
    return r


def _rocm_root() -> str:
    from paper_2102_06611_amd import build
    return os.path.dirname(os.path.dirname(os.path.realpath(build.hipcc())))


def _clangxx() -> str:
    llvm = os.path.join(_rocm_root(), "llvm", "bin", "clang++")
    for cand in (llvm, "/opt/rocm/llvm/bin/clang++", shutil.which("amdclang++")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("clang++ of the ROCm toolchain not found")


def build_libpa_driver(out_dir: str) -> str:
    """libpa's sources with the library's flags plus host sanitizers, linked
    with the driver; returns the executable's path."""
    from paper_2102_06611_amd import build
    os.makedirs(out_dir, exist_ok=True)

    def compile_one(src):
        obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
        _run([build.hipcc()] + build.flags() + HIP_HOST_SANITIZE +
             ["-c", os.path.join(build.CSRC, src), "-o", obj])
        return obj

    with concurrent.futures.ThreadPoolExecutor(max_workers=len(build.SOURCES)) as ex:
        objs = list(ex.map(compile_one, build.SOURCES))
    drv_obj = os.path.join(out_dir, "sanitize_libpa_driver.o")
    _run([_clangxx(), "-O1", "-g", "-std=c++17", "-D__HIP_PLATFORM_AMD__",
          "-I" + os.path.join(_rocm_root(), "include"),
          "-I" + build.INCLUDE, "-fno-omit-frame-pointer"] + GCC_SANITIZE +
         ["-c", LIBPA_DRIVER, "-o", drv_obj])
    exe = os.path.join(out_dir, "sanitize_libpa_driver")
    _run([build.hipcc(), "--offload-arch=" + build.ARCH] + HIP_HOST_SANITIZE +
         ["-o", exe, drv_obj] + objs)
    return exe


@pytest.mark.timeout(120)
def test_oracle_c_under_asan_and_ubsan(tmp_path):
    san = str(tmp_path / "oracle_san")
    plain = str(tmp_path / "oracle_plain")
    common = ["-std=c11", "-ffp-contract=off", ORACLE_DRIVER, ORACLE_C]
    _run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer"] + GCC_SANITIZE + ["-o", san] + common)
    _run(["gcc", "-O2", "-o", plain] + common)
    r_san = _run([san], env=dict(os.environ, **SAN_ENV))
    r_plain = _run([plain])
    assert "runtime error" not in r_san.stderr and "Sanitizer" not in r_san.stderr, r_san.stderr
    assert r_san.stdout.strip() == r_plain.stdout.strip()
    assert len(r_san.stdout.strip()) == 16


@pytest.mark.timeout(600)
def test_libpa_host_code_under_asan_and_ubsan(tmp_path):
    exe = build_libpa_driver(str(tmp_path / "libpa_san"))
    # no device here: HIP finds none, and the host mode never asks for one
    env = dict(os.environ, **SAN_ENV)
    r = _run([exe, "host"], env=env)
    assert r.stdout.strip().endswith("host checks ok"), r.stdout
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr


if __name__ == "__main__":
    print(build_libpa_driver(sys.argv[1] if len(sys.argv) > 1 else "libpa_sanitize_build"))
