"""Build libbq.so (HIP, gfx950 only) in-tree.

Every call recompiles.  Flags: -O3, C++17, and -packed-fp32-ops disabled for
the device code (hipcc's host pass warns that it does not know the feature;
that warning is harmless); the slice GEMMs also keep MFMA accumulators in
VGPRs (EXTRA).
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libbq.so")
SOURCES = ["bq_engine.cpp", "bq_kernels.hip", "bq_split.hip", "bq_split_f8.hip", "bq_crt.hip", "bq_heev.hip",
           "bq_noalloc.hip"]
# The eigensolves of bq_heev call rocSOLVER (with rocBLAS for its handle).
LIBS = ["-L/opt/rocm/lib", "-lrocsolver", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC]
# Slice GEMMs: MFMA accumulators in ordinary VGPRs.  The level sums are
# updated by chains of MFMAs of different lengths; with AGPR accumulators the
# register allocator rotates them between registers and copies them back
# every k-step, with VGPR accumulators every MFMA accumulates in place.
EXTRA = {"bq_split.hip": ["-Xarch_device", "-mllvm=-amdgpu-mfma-vgpr-form=1"]}


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{out}")
    if verbose and out.strip():
        print(out)


def build(verbose: bool = False) -> str:
    from concurrent.futures import ThreadPoolExecutor

    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    cmds, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmds.append([HIPCC, *COMMON, *EXTRA.get(src, []), *lang, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    # One compiler process per source, at most as many as there are CPUs.
    with ThreadPoolExecutor(max_workers=max(1, min(len(cmds), os.cpu_count() or 1, 8))) as ex:
        for f in [ex.submit(_run, c, verbose) for c in cmds]:
            f.result()
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, *LIBS, "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
