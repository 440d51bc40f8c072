"""Build libmfq.so (HIP kernels + C ABI) for gfx950, in-tree.

    python -m paper_1910_13247_amd.build      # or build() from Python

Each source compiles to an object under _build/ in parallel, then one shared library is linked
next to this file.  Packed FP32 instruction selection is disabled for all device code.

    python -m paper_1910_13247_amd.build --sanitize   # or build(sanitize=True)

builds the same library with AddressSanitizer and UndefinedBehaviorSanitizer on the host code
only (device code is compiled as usual) into _build/sanitize/libmfq.so.  Load it in a process
that preloads the ASan runtime (sanitizer_env() gives the environment) and point MFQ_LIBRARY at it.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libmfq.so")
ARCH = "gfx950"

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-function",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(ROOT, "include")]


# host-only sanitizers: each flag applies to the host compilation pass alone
SANITIZE = "-Xarch_host -fsanitize=address,undefined -Xarch_host -fno-sanitize-recover=undefined".split() + \
    "-Xarch_host -fno-omit-frame-pointer".split()
SAN_BUILD = os.path.join(BUILD, "sanitize")
SAN_LIB = os.path.join(SAN_BUILD, "libmfq.so")


def sources():
    out = []
    for f in sorted(os.listdir(CSRC)):
        if f.endswith((".hip", ".cpp")):
            out.append(os.path.join(CSRC, f))
    return out


def _compile(src, sanitize=False):
    obj = os.path.join(SAN_BUILD if sanitize else BUILD, os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [HIPCC] + COMMON + (SANITIZE if sanitize else []) + lang + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj, r.stderr


def build(verbose=False, jobs=None, sanitize=False):
    """Compile every source and link paper_1910_13247_amd/libmfq.so (or, with sanitize, the
    host-sanitized _build/sanitize/libmfq.so); returns its path."""
    out_dir = SAN_BUILD if sanitize else BUILD
    os.makedirs(out_dir, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(lambda s: _compile(s, sanitize), srcs))
    objs = [o for o, _ in results]
    if verbose:
        for _, err in results:
            if err.strip():
                print(err, file=sys.stderr)
    out = SAN_LIB if sanitize else LIB
    tmp = out + ".tmp"
    san = (SANITIZE + ["-shared-libasan"]) if sanitize else []
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}"] + san + ["-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    return out


def sanitizer_env(base=None):
    """Environment for a process that loads the host-sanitized library: the ASan runtime
    preloaded (the interpreter itself is not instrumented), MFQ_LIBRARY pointing at the library,
    every UBSan finding fatal, leak checking off (the interpreter's own allocations)."""
    r = subprocess.run([HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    rt = r.stdout.strip()
    if r.returncode != 0 or not os.path.exists(rt):
        raise RuntimeError("the ASan runtime of the HIP toolchain was not found")
    env = dict(os.environ if base is None else base)
    env["LD_PRELOAD"] = rt
    env["MFQ_LIBRARY"] = SAN_LIB
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    return env


if __name__ == "__main__":
    print(build(verbose=True, sanitize="--sanitize" in sys.argv[1:]))
