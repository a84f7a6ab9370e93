"""Builds the HIP library librz.so in-tree for gfx950 with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "librz.so")
SOURCES = ["csrc/refelem.cpp", "csrc/topology.cpp", "csrc/multigrid.cpp", "csrc/kernels.hip", "csrc/capi.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay off in every device pass
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # MFMA accumulators in ordinary VGPRs (no AGPR copies around loop-carried sums)
    "-mllvm", "-amdgpu-mfma-vgpr-form=1",
    "-I", os.path.join(ROOT, "include"),
]


def build(verbose=False, jobs=4):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        objs.append(obj)
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [hipcc] + HIPCC_FLAGS + lang + ["-c", os.path.join(HERE, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l and "warning: feature flag" not in l]
        if p.returncode != 0:
            failed.append(src)
            print("\n".join(lines), file=sys.stderr)
        elif verbose and lines:
            print("\n".join(lines))
    if failed:
        raise RuntimeError("hipcc failed for " + ", ".join(failed))
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def build_host_sanitized(out_dir, verbose=False, jobs=4, reuse_kernels=True):
    """The library with its host code built with AddressSanitizer and
    UndefinedBehaviorSanitizer (the device code as usual), for
    the CPU tests of the host-only entry points (reference tables,
    numbering, patch lists, argument and mesh checks).  Load it with the
    sanitizer runtime preloaded (see sanitizer_runtime) and RZ_LIBRARY set to
    the returned path.  With reuse_kernels the up-to-date in-tree object of
    the device kernels (whose host side is only their launchers) is linked
    in instead of being rebuilt."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(out_dir, exist_ok=True)
    flags = [f for f in HIPCC_FLAGS if f != "--offload-arch=gfx950"]
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined", "-O1", "-g"]
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(out_dir, os.path.basename(src) + ".o")
        if src == "csrc/kernels.hip" and reuse_kernels:
            # the device kernels and their thin launchers: the in-tree object
            # when it is newer than every source it includes
            built = os.path.join(HERE, "_build", "kernels.hip.o")
            deps = [os.path.join(HERE, "csrc", f) for f in ("kernels.hip", "kernels.hpp")]
            if os.path.exists(built) and all(os.path.getmtime(built) > os.path.getmtime(d) for d in deps):
                objs.append(built)
                continue
        objs.append(obj)
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [hipcc, "--offload-arch=gfx950"] + flags + san + lang + ["-c", os.path.join(HERE, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            failed.append(src)
            print(out.decode(errors="replace"), file=sys.stderr)
    if failed:
        raise RuntimeError("hipcc failed for " + ", ".join(failed))
    lib = os.path.join(out_dir, "librz_hostsan.so")
    subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
                    "-Xarch_host", "-fsanitize=undefined", "-shared-libasan", "-o", lib] + objs, check=True)
    return lib


def sanitizer_runtime():
    """Path of the clang AddressSanitizer runtime that a Python process must
    preload to load the host-sanitizer build."""
    out = subprocess.run(["/opt/rocm/llvm/bin/clang", "-print-file-name=libclang_rt.asan-x86_64.so"],
                         capture_output=True, text=True, check=True).stdout.strip()
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
