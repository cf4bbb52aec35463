"""Runs the CPU test suite against AddressSanitizer / UndefinedBehaviorSanitizer
builds of the host-side code (CPU only; the GPU code is not instrumented):

  * the FP64 oracle (oracle/rg_oracle.c: pthreads, manual index arithmetic,
    adjacency tables) built with gcc -fsanitize=address,undefined;
  * the library's host code (argument validation, size computations, the
    serving pool and admission accounting, descriptor handling in
    paper_2001_09792_amd/csrc/*.hip) built with hipcc, the sanitizer flags
    applied to the host compilation only (-Xarch_host).

Both builds go to a temporary directory; the tests load them through
RG_ORACLE_LIBRARY / RG_LIBRARY, with the sanitizer runtime preloaded.
Usage:  python tests/run_sanitizers.py [pytest args...]
(default: the CPU tests of the oracle, the ABI, the serving host logic and
the scene generators).  Exit status: pytest's.
"""
import os
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = "-fsanitize=address,undefined"
DEFAULT_TESTS = ["tests/test_oracle_triangle.py", "tests/test_oracle_ties.py", "tests/test_oracle_invariants.py",
                 "tests/test_oracle_shading.py", "tests/test_oracle_masks.py", "tests/test_oracle_alpha.py",
                 "tests/test_abi.py", "tests/test_serve.py"]


CLANG = "/opt/rocm/llvm/bin/clang"   # one sanitizer runtime for both builds: clang's


def build_oracle(out: str) -> str:
    lib = os.path.join(out, "liboracle_san.so")
    subprocess.check_call([CLANG, "-O1", "-g", "-fno-omit-frame-pointer", "-std=c11", "-D_GNU_SOURCE",
                           "-ffp-contract=off", "-fno-fast-math", SAN, "-fno-sanitize-recover=undefined",
                           "-shared-libasan", "-shared", "-fPIC", "-pthread",
                           os.path.join(ROOT, "oracle", "rg_oracle.c"), "-o", lib, "-lm"])
    return lib


def build_library(out: str) -> str:
    sys.path.insert(0, os.path.join(ROOT, "paper_2001_09792_amd"))
    import _build
    lib = os.path.join(out, "librg_san.so")
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    flags = [f for f in _build.FLAGS if f != "-O3"] + [
        "-O1", "-g", "-fno-omit-frame-pointer",
        "-Xarch_host", "-fsanitize=address",
        "-Xarch_host", "-fsanitize=undefined",
        "-Xarch_host", "-fno-sanitize-recover=undefined",
        "-Xarch_host", "-shared-libasan"]
    srcs = [os.path.join(_build.CSRC, s) for s in _build.SOURCES]
    subprocess.check_call([hipcc] + flags + srcs + ["-o", lib])
    return lib


def main(argv):
    out = tempfile.mkdtemp(prefix="rg_san_")
    print("[sanitizers] building the oracle", flush=True)
    olib = build_oracle(out)
    print("[sanitizers] building the library's host code", flush=True)
    rlib = build_library(out)
    # the library's host code is built by clang: its ASan runtime serves both
    runtime = subprocess.check_output([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"], text=True).strip()
    env = dict(os.environ, RG_ORACLE_LIBRARY=olib, RG_LIBRARY=rlib, LD_PRELOAD=runtime,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    args = argv or DEFAULT_TESTS
    cmd = [sys.executable, "-m", "pytest", "-q", "-m", "not gpu", "-p", "no:cacheprovider"] + args
    print("[sanitizers] " + " ".join(cmd), flush=True)
    return subprocess.call(cmd, cwd=ROOT, env=env)


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
