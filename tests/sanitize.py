"""CPU sanitizer run: the oracle (oracle/fewha_oracle.c) and the library's host code (plan and C-ABI
layers of libfewha.so) built with AddressSanitizer and UndefinedBehaviorSanitizer, then the
`-m "not gpu"` suite run against those builds.  Works on a copy of the tree in a temporary
directory, so the normal builds are never touched.  Device code is built as usual (the
sanitizers apply to host code only).  Exit status: pytest's (0 = clean).

    python tests/sanitize.py [extra pytest arguments]
"""
import glob
import os
import shutil
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from paper_2009_00946_amd import build as B  # noqa: E402

LLVM = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm")
SAN = ["-fsanitize=address", "-fsanitize=undefined"]


def asan_runtime():
    libs = sorted(glob.glob(os.path.join(LLVM, "lib", "clang", "*", "lib", "linux", "libclang_rt.asan-x86_64.so")))
    if not libs:
        raise RuntimeError("clang's ASan runtime not found under %s" % LLVM)
    return libs[-1]


def main(extra):
    tmp = tempfile.mkdtemp(prefix="fewha_san_")
    try:
        dst = os.path.join(tmp, "repo")
        shutil.copytree(ROOT, dst, ignore=shutil.ignore_patterns(".git", "_work", "gpurun_out", "*.so", "__pycache__"))
        # oracle: clang (one sanitizer runtime for the whole process), OpenMP from the same toolchain
        orc = os.path.join(dst, "oracle")
        subprocess.check_call([os.path.join(LLVM, "bin", "clang"), "-O1", "-g", "-fno-omit-frame-pointer", "-std=c99",
                               "-fopenmp", "-fPIC", "-shared"] + SAN + ["-o", os.path.join(orc, "liboracle.so"),
                               os.path.join(orc, "fewha_oracle.c"), "-lm"])
        # library: host code sanitized, each sanitizer flag bound to the host pass
        host_san = []
        for f in SAN:
            host_san += ["-Xarch_host", f]
        lib = os.path.join(dst, "paper_2009_00946_amd", "libfewha.so")
        cmd = B.command(lib)
        cmd = [c.replace(os.path.join(ROOT, ""), os.path.join(dst, "")) for c in cmd]
        cmd = cmd[:1] + ["-g", "-Xarch_host", "-fno-omit-frame-pointer"] + host_san + cmd[1:]
        subprocess.check_call(cmd)
        for p in (lib, os.path.join(orc, "liboracle.so")):  # both carry the instrumentation
            syms = subprocess.run(["nm", "-D", p], capture_output=True, text=True, check=True).stdout
            if "__asan_report" not in syms or "__ubsan_handle" not in syms:
                raise RuntimeError("%s was built without the sanitizers" % p)
        # keep the freshly built libraries (the binding and the oracle would rebuild when older
        # than their sources)
        now = os.path.getmtime(lib) + 5
        for p in (lib, os.path.join(orc, "liboracle.so")):
            os.utime(p, (now, now))
        env = dict(os.environ)
        env["LD_PRELOAD"] = asan_runtime()
        env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:halt_on_error=1"
        env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
        env["PYTHONDONTWRITEBYTECODE"] = "1"
        env["FEWHA_SANITIZE"] = "1"
        r = subprocess.run([sys.executable, "-m", "pytest", "tests", "-m", "not gpu", "-x", "-q", "-p", "no:cacheprovider"]
                           + list(extra), cwd=dst, env=env)
        return r.returncode
    finally:
        shutil.rmtree(tmp, ignore_errors=True)


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
