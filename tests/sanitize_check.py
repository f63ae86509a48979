"""CPU sanitizer runs, by hand (not collected by pytest; CPU only):

    python tests/sanitize_check.py

1. The oracle's CPU pins under AddressSanitizer and UndefinedBehaviorSanitizer:
   builds oracle/pfo.c with gcc -fsanitize=address,undefined (no recovery from
   undefined behaviour) into a temporary library, and runs
   tests/test_oracle_*.py against it through PFO_LIBRARY with the ASan runtime
   preloaded into the (uninstrumented) Python interpreter.
2. The host code of the HIP library (parameter validation, workspace layout,
   status strings) under the same sanitizers: the three sources are built with
   the sanitizer flags for the host compilation only (the gfx950 code is
   unchanged), and tests/test_abi_cpu.py runs against that library with
   clang's ASan runtime preloaded.
Leak detection is off: the interpreter itself keeps memory until exit.
Exits non-zero if either run fails.
"""
import os
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def main():
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True,
                          check=True).stdout.strip()
    with tempfile.TemporaryDirectory() as tmp:
        lib = os.path.join(tmp, "libpfo_sanitized.so")
        subprocess.run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=undefined", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
                        "-fopenmp", "-fPIC", "-shared", os.path.join(ROOT, "oracle", "pfo.c"), "-o", lib, "-lm"],
                       check=True)
        tests = sorted(os.path.join(ROOT, "tests", f) for f in os.listdir(os.path.join(ROOT, "tests"))
                       if f.startswith("test_oracle_") and f.endswith(".py"))
        env = dict(os.environ, PFO_LIBRARY=lib, LD_PRELOAD=asan,
                   ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", *tests], cwd=ROOT, env=env)
        return r.returncode


HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]

DRIVER = """
import sys
sys.path.insert(0, {root!r})
from paper_2207_09431_amd import pflbm
pflbm.LIB_PATH = {lib!r}
pflbm._lib = None
import pytest
sys.exit(pytest.main(["-q", "-p", "no:cacheprovider", {test!r}]))
"""


def host_library():
    sys.path.insert(0, ROOT)
    from paper_2207_09431_amd import build as pbuild
    asan = subprocess.run(["hipcc", "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                          text=True, check=True).stdout.strip()
    flags = [f for f in pbuild.hipcc_flags() if f != "-O3"] + ["-O1", "-g"] + HOST_SAN
    with tempfile.TemporaryDirectory() as tmp:
        objs = []
        for src in pbuild.SOURCES:
            obj = os.path.join(tmp, src.replace(".hip", ".o"))
            subprocess.run(["hipcc", *flags, "-c", os.path.join(pbuild.CSRC, src), "-o", obj], check=True)
            objs.append(obj)
        lib = os.path.join(tmp, "libpflbm_sanitized.so")
        subprocess.run(["hipcc", f"--offload-arch={pbuild.ARCH}", "-shared", "-fPIC", "-shared-libsan",
                        "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", *objs, "-o", lib],
                       check=True)
        env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1")
        code = DRIVER.format(root=ROOT, lib=lib, test=os.path.join(ROOT, "tests", "test_abi_cpu.py"))
        r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env)
        return r.returncode


if __name__ == "__main__":
    rc_oracle = main()
    rc_host = host_library()
    print(f"oracle pins: {'pass' if rc_oracle == 0 else 'FAIL'}; HIP library host code: "
          f"{'pass' if rc_host == 0 else 'FAIL'}", flush=True)
    sys.exit(1 if rc_oracle or rc_host else 0)
