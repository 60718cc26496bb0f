"""Build the HIP library libbras.so for gfx950 in-tree (hipcc, no torch extension).

Usage: python -m paper_2607_12138_amd.build [--jobs N]
"""
import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libbras.so")
ARCH = os.environ.get("BRAS_OFFLOAD_ARCH", "gfx950")

SOURCES = [
    ("host_mesh.cpp", ["-ffp-contract=off"]),
    ("host_fe.cpp", []),
    ("capi.cpp", []),
    ("setup.hip", []),
    ("apply.hip", []),
    ("csr.hip", []),
    ("spgemm.hip", []),
    ("lane_packed_f64.hip", []),
    ("lane_packed_f32.hip", []),
    ("lane_metric3.hip", []),
    ("lane_metric6_v0.hip", []),
    ("lane_metric6_v1.hip", []),
    ("lane_metric6_v2.hip", []),
    ("elem_mfma.hip", []),
    ("pcg.hip", []),
    ("pcg_small.hip", []),
    ("bf16.hip", []),
    ("noalloc.hip", []),
    ("microbench.hip", []),
    ("patch_setup.cpp", []),
    ("patch.hip", []),
    ("patch_scaled.hip", []),
    ("patch_packed_f32.hip", []),
    ("patch_packed_f64.hip", []),
    ("patch_metric3.hip", []),
    ("patch_metric6.hip", []),
]

COMMON = [
    "-O3", "-fPIC", "-std=c++17", "--offload-arch=" + ARCH,
    # packed FP32 instructions are disabled for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def compile_one(src, extra):
    obj = os.path.join(BUILD, src + ".o")
    cmd = [hipcc(), "-c", os.path.join(CSRC, src), "-o", obj] + COMMON + extra
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    warn = (r.stderr or "").strip()
    return obj, warn


def _up_to_date(src):
    """The object of src is newer than src and every header it may include."""
    obj = os.path.join(BUILD, src + ".o")
    if not os.path.exists(obj):
        return False
    deps = [os.path.join(CSRC, src), os.path.join(os.path.dirname(HERE), "include", "bras.h")]
    deps += [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".h")]
    t = os.path.getmtime(obj)
    return all(os.path.getmtime(d) < t for d in deps)


def build(jobs=8, verbose=False, incremental=False):
    """Compile every source (incremental: only those whose object is out of
    date) and link libbras.so."""
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = []
        for s, e in SOURCES:
            if incremental and _up_to_date(s):
                futs.append(None)
                objs.append(os.path.join(BUILD, s + ".o"))
            else:
                futs.append(ex.submit(compile_one, s, e))
                objs.append(None)
        for k, f in enumerate(futs):
            if f is None:
                continue
            obj, warn = f.result()
            objs[k] = obj
            if verbose and warn:
                print(warn, file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=8)
    ap.add_argument("-v", "--verbose", action="store_true")
    ap.add_argument("--incremental", action="store_true", help="recompile only out-of-date objects")
    a = ap.parse_args()
    print(build(a.jobs, a.verbose, a.incremental))
