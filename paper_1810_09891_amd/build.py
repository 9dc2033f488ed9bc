"""Build the HIP library ``paper_1810_09891_amd/lib/libnfft_mi355x.so`` for gfx950.

Each ``csrc/*.hip`` file is compiled to an object with hipcc (in parallel) and the
objects are linked into one shared library that exports the C ABI of
``include/nfft_mi355x.h``.  Always rebuilds when called.  (The LDS throughput probe under
``calib/`` is measurement tooling and is built by ``profiling.py lds-probe`` instead.)

``build_host_sanitized()`` builds a second copy under ``_build/host_sanitized/`` whose host
code (plan set-up, workspace layout, batching, tuning caches, argument checks) carries
AddressSanitizer and UndefinedBehaviorSanitizer.  It is for host-side tests on the CPU only,
loaded with the ASan runtime preloaded; its kernels are never launched, so its device code is
compiled without optimisation (a quarter of the compile time).
"""
import concurrent.futures
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OBJ = os.path.join(ROOT, "_build", "obj")
LIBDIR = os.path.join(PKG, "lib")
LIB = os.path.join(LIBDIR, "libnfft_mi355x.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

CFLAGS = [
    "-O3",
    "-std=c++17",
    "-fPIC",
    "--offload-arch=" + ARCH,
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
    "-I" + os.path.join(ROOT, "include"),
]


def _compile(src):
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    cmd = [HIPCC] + CFLAGS + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr[-20000:]))
    warn = [l for l in r.stderr.splitlines() if "warning" in l and "packed-fp32-ops" not in l]
    return obj, warn


def build(verbose=False, jobs=None):
    os.makedirs(OBJ, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    jobs = jobs or min(len(srcs), os.cpu_count() or 4, 8)
    objs = []
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        for obj, warn in ex.map(_compile, srcs):
            objs.append(obj)
            if verbose:
                for w in warn:
                    print(w)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr[-20000:]))
    os.replace(tmp, LIB)
    return LIB


HOST_SAN_DIR = os.path.join(ROOT, "_build", "host_sanitized")
HOST_SAN_LIB = os.path.join(HOST_SAN_DIR, "libnfft_mi355x.so")
# sanitizers for the host pass only (each flag after -Xarch_host); the device pass unoptimised
HOST_SAN_FLAGS = ["-Xarch_host", "-O1", "-Xarch_host", "-g", "-Xarch_host", "-fno-omit-frame-pointer",
                  "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_device", "-O0"]


def host_asan_runtime():
    """The clang ASan runtime that a process loading the host-sanitized library preloads."""
    hits = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def build_host_sanitized(jobs=None):
    """Build ``_build/host_sanitized/libnfft_mi355x.so``; kept when its stamp (a hash of the
    sources and flags) is current.  Returns the library path."""
    import hashlib
    srcs = sorted(glob.glob(os.path.join(CSRC, "*"))) + [os.path.join(ROOT, "include", "nfft_mi355x.h")]
    h = hashlib.sha256(" ".join(CFLAGS + HOST_SAN_FLAGS).encode())
    for f in srcs:
        with open(f, "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    stamp = os.path.join(HOST_SAN_DIR, "stamp")
    if os.path.exists(HOST_SAN_LIB) and os.path.exists(stamp) and open(stamp).read() == h.hexdigest():
        return HOST_SAN_LIB
    os.makedirs(HOST_SAN_DIR, exist_ok=True)
    hip = sorted(glob.glob(os.path.join(CSRC, "*.hip")))

    def comp(src):
        obj = os.path.join(HOST_SAN_DIR, os.path.basename(src) + ".o")
        cmd = [HIPCC] + CFLAGS + HOST_SAN_FLAGS + ["-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr[-20000:]))
        return obj

    jobs = jobs or min(len(hip), os.cpu_count() or 4, 8)
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(comp, hip))
    # the objects carry their device code; the host link adds the shared sanitizer runtimes
    clangxx = os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "lib", "llvm", "bin", "clang++")
    if not os.path.exists(clangxx):
        clangxx = "/opt/rocm/lib/llvm/bin/clang++"
    tmp = HOST_SAN_LIB + ".tmp%d" % os.getpid()
    cmd = [clangxx, "-shared", "-fPIC", "-fsanitize=address,undefined", "-shared-libsan", "-o", tmp] + objs + [
        "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr[-20000:]))
    os.replace(tmp, HOST_SAN_LIB)
    with open(stamp, "w") as fh:
        fh.write(h.hexdigest())
    return HOST_SAN_LIB


if __name__ == "__main__":
    if "--host-sanitized" in sys.argv:
        print(build_host_sanitized())
    else:
        print(build(verbose="-v" in sys.argv))
