"""The oracle's CPU pins under AddressSanitizer and UndefinedBehaviorSanitizer,
run by hand (not collected by pytest; CPU only):

    python tests/sanitize_check.py

Builds oracle/pfo.c with gcc -fsanitize=address,undefined (no recovery from
undefined behaviour) into a temporary library, and runs tests/test_oracle_*.py
against it through PFO_LIBRARY with the ASan runtime preloaded into the
(uninstrumented) Python interpreter.  Leak detection is off: the interpreter
itself keeps memory until exit.  Exits with the test run's status.
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


if __name__ == "__main__":
    sys.exit(main())
