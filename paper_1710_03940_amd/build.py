"""Build libdfamg.so (HIP for gfx950 + host C++) in-tree with hipcc.

Usage: python -m paper_1710_03940_amd.build [--force]
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libdfamg.so")
# (source, extra flags, object name)
UNITS = [
    ("host_plan.cpp", [], "host_plan.o"),
    ("device.hip", [], "device.o"),
    ("launch_outer.hip", [], "launch_outer.o"),
    ("launch_vcycle.hip", ["-DDFAMG_VT_DOUBLE"], "launch_vcycle_f64.o"),
    ("launch_vcycle.hip", [], "launch_vcycle_f32.o"),
    ("dense_inverse.hip", [], "dense_inverse.o"),
    # the setup kernels reproduce the host's rounding: no fused multiply-adds
    ("setup_device.hip", ["-ffp-contract=off"], "setup_device.o"),
]
HEADERS = ["host_plan.hpp", "kernels.hpp", "kernels_fgmres.hpp", "kernels_schur.hpp", "kernels_bsmooth.hpp",
           "kernels_coarse_setup.hpp", "devmat.hpp", "dense_inverse.hpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # hand-written code must not rely on packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I" + INCLUDE, "-I" + CSRC,
]


def _stale():
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = [os.path.join(CSRC, u[0]) for u in UNITS] + [os.path.join(CSRC, h) for h in HEADERS]
    deps.append(os.path.join(INCLUDE, "dfamg.h"))
    return any(os.path.getmtime(d) > t for d in deps)


def build(force=True, verbose=True, jobs=None):
    """Compile the library (always when force=True); translation units are
    compiled in parallel."""
    from concurrent.futures import ThreadPoolExecutor
    if not force and not _stale():
        return LIB
    jobs = jobs or min(len(UNITS), max(1, (os.cpu_count() or 4)))
    cmds = []
    for src, extra, objname in UNITS:
        obj = os.path.join(CSRC, objname)
        cmd = [HIPCC] + [f for f in FLAGS if f != "-shared"] + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
        cmds.append((cmd, obj))

    def run(c):
        if verbose:
            print(" ".join(c[0]), flush=True)
        subprocess.check_call(c[0])
        return c[1]

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(run, cmds))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lrocblas", "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    build(force=True)
    print(LIB)
