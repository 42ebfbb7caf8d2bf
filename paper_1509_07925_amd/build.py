"""Compile libmbf.so (HIP for gfx950 + host C++) in-tree with hipcc.

Usage: python -m paper_1509_07925_amd.build   (or build() from Python)
       python -m paper_1509_07925_amd.build --sanitize   (host ASan/UBSan build + CPU tests)
"""

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmbf.so")
ARCH = os.environ.get("MBF_OFFLOAD_ARCH", "gfx950")
# Host-code AddressSanitizer + UndefinedBehaviorSanitizer build (libmbf_asan.so):
# the host side of every file instrumented, device code untouched.
SAN_DIR = os.path.join(HERE, "_build_asan")
SAN_LIB = os.path.join(HERE, "libmbf_asan.so")
# (device code is built as in the plain build)
SAN = ["-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
       "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=undefined"]
SAN_HOST = ["-O1", "-g"]

COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-variable", "-Wno-unused-function",
          "-Wno-unused-result", "-I", os.path.join(HERE, "..", "include")]
# Device code: no packed-FP32 instructions (some of their forms have given
# wrong results on this hardware).
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]
HOST_ONLY = ["-march=x86-64-v3", "-fcx-limited-range", "-ffp-contract=fast", "-fno-math-errno", "-fno-signed-zeros", "-fno-trapping-math", "-fassociative-math", "-freciprocal-math"]


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _rocm():
    return os.environ.get("ROCM_PATH", "/opt/rocm")


def _compile(src, sanitize=False):
    obj = os.path.join(SAN_DIR if sanitize else OUT_DIR, os.path.basename(src) + ".o")
    extra = SAN if sanitize else []
    if src.endswith(".hip"):
        cmd = [_hipcc(), "-x", "hip"] + COMMON + DEVICE + extra + ["-c", src, "-o", obj]
    else:
        cmd = [_hipcc()] + COMMON + HOST_ONLY + extra + (SAN_HOST if sanitize else []) + [
            "-D__HIP_PLATFORM_AMD__", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(verbose=False, sanitize=False):
    """Compile and link libmbf.so (sanitize: libmbf_asan.so, see SAN)."""
    out_dir, lib = (SAN_DIR, SAN_LIB) if sanitize else (OUT_DIR, LIB)
    os.makedirs(out_dir, exist_ok=True)
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".cpp", ".hip")))
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, sanitize), srcs))
    tmp = lib + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs + [
        "-L" + os.path.join(_rocm(), "lib"), "-Wl,-rpath," + os.path.join(_rocm(), "lib"), "-lrocsolver", "-lrocblas",
        "-lpthread"]
    if sanitize:
        cmd += ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-shared-libsan"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, lib)
    if verbose:
        print("built", lib)
    return lib


def asan_runtime():
    """Path of the compiler's shared AddressSanitizer runtime (LD_PRELOAD for Python)."""
    r = subprocess.run([_hipcc().replace("hipcc", "amdclang++"), "-print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("AddressSanitizer runtime not found")
    return path


def sanitized_tests(pytest_args=("tests", "-x", "-q", "-m", "not gpu")):
    """Build libmbf_asan.so and run the CPU tests against it (MBF_LIB) in a
    child process with the sanitizer runtime preloaded.  Leak detection is
    off: the Python interpreter itself is not instrumented."""
    lib = build(verbose=True, sanitize=True)
    env = dict(os.environ)
    env["MBF_LIB"] = lib
    env["LD_PRELOAD"] = asan_runtime()
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    root = os.path.dirname(HERE)
    return subprocess.call([sys.executable, "-m", "pytest"] + list(pytest_args), cwd=root, env=env)


if __name__ == "__main__":
    if "--sanitize" in sys.argv[1:]:
        sys.exit(sanitized_tests())
    build(verbose=True)
    sys.exit(0)
