"""Build librqrcp.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_1505_08115_amd.build_lib   (or call build()).
"""
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "librqrcp.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep packed-FP32 instructions out of all generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def sources():
    return sorted(glob.glob(os.path.join(PKG, "csrc", "*.hip")))


def _compile(hipcc, src, obj, verbose):
    flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    cmd = [hipcc, *flags, "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"), "-c", src,
           "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    errs = "\n".join(l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l)
    return res.returncode, errs


def build(verbose=False):
    """Compile every source to an object in parallel (one hipcc per file),
    then link the shared library; every call compiles afresh."""
    from concurrent.futures import ThreadPoolExecutor
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    srcs = sources()
    objs = [os.path.join(objdir, os.path.basename(s) + ".o") for s in srcs]
    jobs = max(1, min(len(srcs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(lambda so: _compile(hipcc, so[0], so[1], verbose), zip(srcs, objs)))
    for src, (rc, errs) in zip(srcs, results):
        if rc != 0:
            raise RuntimeError(f"hipcc failed on {os.path.basename(src)}:\n" + errs)
        if verbose and errs.strip():
            print(errs, file=sys.stderr)
    out_tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", out_tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + res.stderr)
    os.replace(out_tmp, LIB)
    build_driver(hipcc, verbose)
    return LIB


DRIVER_SRC = os.path.join(PKG, "driver", "rqrcp_bench.hip")
DRIVER = os.path.join(PKG, "rqrcp_bench")


def build_driver(hipcc, verbose=False):
    """The standalone C-ABI driver (linked against the in-tree librqrcp.so)."""
    flags = [f for f in HIPCC_FLAGS if f not in ("-shared", "-fPIC")]
    cmd = [hipcc, *flags, "-I", os.path.join(ROOT, "include"), DRIVER_SRC, "-L", PKG, "-lrqrcp",
           "-Wl,-rpath,$ORIGIN", "-o", DRIVER + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        errs = "\n".join(l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l)
        raise RuntimeError("hipcc failed on the driver:\n" + errs)
    os.replace(DRIVER + ".tmp", DRIVER)
    return DRIVER


if __name__ == "__main__":
    print(build(verbose=True))
