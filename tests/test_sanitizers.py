"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only).

* The oracle (oracle/smc_oracle.c) is rebuilt with gcc -fsanitize=address,
  undefined and its pins (the oracle test modules) run against that build in
  a child Python with gcc's ASan runtime preloaded.
* The library's host runtime (runtime.cpp: argument validation, threshold
  tables, handle bookkeeping) is rebuilt with the sanitizers on its host
  code only (-Xarch_host), linked with the unchanged device objects, and the
  host ABI checks run against it with clang's ASan runtime preloaded.

Any sanitizer report aborts the child (halt_on_error, no recovery from UB),
which fails the test.  Leak checking is off: the interpreter itself keeps
allocations alive until exit."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = {
    "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0:exitcode=97",
    "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1:exitcode=98",
}


def _run(cmd, env, timeout):
    e = dict(os.environ)
    e.update(env)
    p = subprocess.run(cmd, cwd=ROOT, env=e, capture_output=True, text=True, timeout=timeout)
    tail = (p.stdout[-3000:] + "\n" + p.stderr[-3000:])
    assert p.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in p.stderr and "runtime error:" not in p.stderr, tail
    return p


def test_oracle_pins_under_asan_ubsan(tmp_path):
    libasan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                             text=True).stdout.strip()
    if not os.path.isabs(libasan) or not os.path.exists(libasan):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-fopenmp", "-ffp-contract=off",
                    "-fno-fast-math", "-fPIC", "-shared", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    "-o", lib, os.path.join(ROOT, "oracle", "smc_oracle.c"), "-lm"], check=True)
    env = dict(SAN_ENV, LD_PRELOAD=libasan, SMC_ORACLE_LIB=lib, OMP_NUM_THREADS="4")
    # the child really runs the instrumented build under the ASan runtime
    _run([sys.executable, "-c", "import oracle; oracle.lib(); m = open('/proc/self/maps').read(); "
          f"assert 'libasan' in m and {lib!r} in m, 'sanitized oracle not loaded'"], env, timeout=120)
    _run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
          "tests/test_oracle_rng.py", "tests/test_oracle_thresholds.py",
          "tests/test_oracle_ising.py", "tests/test_oracle_continuous.py",
          "tests/test_oracle_chains.py", "tests/test_oracle_rules.py",
          "tests/test_oracle_schedule_pins.py"], env, timeout=900)


def _clang_asan_runtime():
    import glob
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_host_runtime_under_asan_ubsan(tmp_path):
    rt = _clang_asan_runtime()
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if rt is None or not os.path.exists(hipcc):
        pytest.skip("hipcc or clang's AddressSanitizer runtime is not installed")
    from paper_1107_5463_amd import build as pkg_build
    objdir = os.path.join(ROOT, "paper_1107_5463_amd", "_build")
    if not all(os.path.exists(os.path.join(objdir, os.path.splitext(s)[0] + ".o"))
               for s in pkg_build.SOURCES):
        pkg_build.build()
    obj = str(tmp_path / "runtime_san.o")
    flags = [f for f in pkg_build.flags() if f != "-O3"] + ["-O1", "-g"]
    subprocess.run([hipcc] + flags + ["-Xarch_host", "-fsanitize=address",
                                      "-Xarch_host", "-fsanitize=undefined",
                                      "-Xarch_host", "-fno-sanitize-recover=undefined",
                                      "-Xarch_host", "-fno-omit-frame-pointer",
                                      "-x", "hip", "-c",
                                      os.path.join(ROOT, "paper_1107_5463_amd", "csrc", "runtime.cpp"),
                                      "-o", obj], check=True, capture_output=True)
    objs = [os.path.join(objdir, os.path.splitext(s)[0] + ".o") for s in pkg_build.SOURCES
            if s != "runtime.cpp"] + [obj]
    lib = str(tmp_path / "libsmc_san.so")
    subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC",
                    "-Xarch_host", "-shared-libsan", "-Xarch_host", "-fsanitize=address",
                    "-Xarch_host", "-fsanitize=undefined", "-o", lib] + objs, check=True,
                   capture_output=True)
    env = dict(SAN_ENV, LD_PRELOAD=rt, SMC_LIBRARY=lib)
    _run([sys.executable, "-c", "import paper_1107_5463_amd as s; s.load_library(); "
          "m = open('/proc/self/maps').read(); "
          f"assert 'libclang_rt.asan' in m and {lib!r} in m, 'sanitized library not loaded'"],
         env, timeout=120)
    _run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
          "tests/test_abi_host.py", "-m", "not gpu"], env, timeout=600)
