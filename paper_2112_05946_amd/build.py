"""Build libfrsg.so (HIP for gfx950 + C++ host code) in-tree with hipcc."""

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfrsg.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-fPIC", "-std=c++17", "-I" + INCLUDE, "-I" + CSRC]
# packed FP32 instructions are kept out of every device code object
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


def sources():
    out = []
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".cpp")):
            out.append(os.path.join(CSRC, name))
    return out


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC] + COMMON
    if src.endswith(".hip"):
        cmd += DEVICE + ["-x", "hip"]
    cmd += ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in (r.stderr or "").splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), err))
    return obj


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


# Host code checked by AddressSanitizer and UndefinedBehaviorSanitizer: the host
# sources (problem validation, operator tables, meshes, workspace layout) are
# compiled with both, the device sources are the objects of the normal build
# (the flags reach the host pass only), and the result is a separate library
# that a process loads after preloading the sanitizer runtime.
SAN_LIB = os.path.join(BUILD, "libfrsg_san.so")
SAN_LINK = "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined".split()
SAN_FLAGS = "-O1 -g -fno-omit-frame-pointer -Xarch_host -fno-sanitize-recover=undefined".split() + SAN_LINK


def sanitizer_runtime():
    """Path of the clang AddressSanitizer runtime that hipcc's host compiler links against."""
    r = subprocess.run([HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = (r.stdout or "").strip()
    if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path):
        return path
    root = "/opt/rocm/llvm/lib/clang"
    for ver in sorted(os.listdir(root)) if os.path.isdir(root) else []:
        cand = os.path.join(root, ver, "lib", "linux", "libclang_rt.asan-x86_64.so")
        if os.path.exists(cand):
            return cand
    return None


def _fresh(obj, src):
    """True when obj is newer than src and every header the sources include."""
    if not os.path.exists(obj):
        return False
    t = os.path.getmtime(obj)
    deps = [src] + [os.path.join(d, f) for d in (CSRC, INCLUDE) for f in os.listdir(d) if f.endswith((".h", ".hpp"))]
    return all(os.path.getmtime(d) < t for d in deps)


def build_sanitized(verbose=False, reuse_device_objects=False):
    """Build libfrsg_san.so: sanitized host sources linked with the normal device objects
    (reused from the normal build when they are newer than their sources and headers)."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    dev = [s for s in srcs if s.endswith(".hip")]
    host = [s for s in srcs if s.endswith(".cpp")]

    def compile_host(src):
        obj = os.path.join(BUILD, os.path.basename(src) + ".san.o")
        cmd = [HIPCC] + [f for f in COMMON if f != "-O3"] + SAN_FLAGS + ["-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), r.stderr))
        return obj

    def compile_dev(src):
        obj = os.path.join(BUILD, os.path.basename(src) + ".o")
        return obj if reuse_device_objects and _fresh(obj, src) else _compile(src)

    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        dev_objs = list(ex.map(compile_dev, dev))
        host_objs = list(ex.map(compile_host, host))
    tmp = SAN_LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH] + SAN_LINK + ["-o", tmp] + dev_objs + host_objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, SAN_LIB)
    if verbose:
        print("built", SAN_LIB)
    return SAN_LIB


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "sanitized":
        build_sanitized(verbose=True)
    else:
        build(verbose=True)
    sys.exit(0)
