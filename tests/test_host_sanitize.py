"""Host code under AddressSanitizer, UndefinedBehaviorSanitizer and LeakSanitizer (CPU).

* libnfft's host code (plan.cpp, runtime.cpp) is rebuilt with the sanitizers on its
  host side only and linked with the library's device objects into a driver
  (tests/sanitize/plan_alloc_faults.c) that checks argument errors, the error of a
  valid plan on a machine without a device (NFFT_ERR_HIP), and -- with the HIP
  allocation call interposed -- that an allocation failing at any point of plan
  creation returns NFFT_ERR_NOMEM and frees everything allocated before it.
* The C part of the oracle and the CPU timing baseline run small problems through
  every entry point under the same sanitizers (tests/sanitize/oracle_and_baseline.c).

Only meaningful without a GPU (the interposed allocator hands out host memory), so the
module is skipped where a device is present.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/lib/llvm/bin/clang"
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="4")
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]

pytestmark = pytest.mark.skipif(os.path.exists("/dev/kfd"),
                                reason="host-only sanitizer checks run on machines without a GPU")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (cmd[0], r.stdout[-2000:], r.stderr[-4000:])
    return r


def test_plan_creation_under_sanitizers(tmp_path):
    from paper_2208_00049_amd import build
    objs = {s: os.path.join(build.BUILD, os.path.splitext(s)[0] + ".o") for s in build.SOURCES}
    if not all(os.path.exists(o) for o in objs.values()):
        build.build()
    csrc = os.path.join(ROOT, "paper_2208_00049_amd", "csrc")
    inc = ["-I", os.path.join(ROOT, "include")]
    san_objs = []
    for src in ("plan.cpp", "runtime.cpp"):
        o = str(tmp_path / (src + ".o"))
        _run([HIPCC, "-x", "hip"] + build.COMMON[:1] + ["-O1", "-g", "-std=c++17", "-fPIC"] +
             HOST_SAN + build.COMMON[4:9] + inc + ["-c", os.path.join(csrc, src), "-o", o])
        san_objs.append(o)
    drv = str(tmp_path / "drv.o")
    _run([CLANG, "-g", "-O1", "-fsanitize=address,undefined", "-D__HIP_PLATFORM_AMD__",
          "-I", "/opt/rocm/include"] + inc +
         ["-c", os.path.join(ROOT, "tests", "sanitize", "plan_alloc_faults.c"), "-o", drv])
    exe = str(tmp_path / "plan_alloc_faults")
    rest = [objs[s] for s in build.SOURCES if s not in ("plan.cpp", "runtime.cpp")]
    _run([HIPCC] + build.COMMON[:1] + HOST_SAN + ["-o", exe, drv] + san_objs + rest)
    supp = tmp_path / "lsan.supp"
    # leaks of the HIP runtime's own initialisation are not the library's
    supp.write_text("leak:libamdhip64\nleak:libhsa-runtime64\nleak:libhsakmt\nleak:libdrm\n")
    env = dict(SAN_ENV, LSAN_OPTIONS="suppressions=%s" % supp)
    r = _run([exe], env=env, timeout=300)
    assert "injected failures returning NFFT_ERR_NOMEM" in r.stdout
    assert "fails 0" in r.stdout


def test_oracle_and_baseline_under_sanitizers(tmp_path):
    flags = ["-g", "-O1", "-fopenmp", "-fsanitize=address,undefined", "-fno-omit-frame-pointer"]
    o1, o2, o3 = (str(tmp_path / n) for n in ("drv.o", "ndft.o", "cpu_nfft.o"))
    _run(["gcc"] + flags + ["-c", os.path.join(ROOT, "tests", "sanitize", "oracle_and_baseline.c"),
                            "-o", o1])
    _run(["gcc"] + flags + ["-c", os.path.join(ROOT, "oracle", "ndft.c"), "-o", o2])
    _run(["g++", "-std=c++17"] + flags + ["-c", os.path.join(ROOT, "baseline", "cpu_nfft.cpp"),
                                          "-o", o3])
    exe = str(tmp_path / "oracle_and_baseline")
    _run(["g++", "-fopenmp", "-fsanitize=address,undefined", "-o", exe, o1, o2, o3, "-lm"])
    r = _run([exe], env=SAN_ENV, timeout=300)
    assert "fails 0" in r.stdout
