"""Build libttice.so (gfx950) from csrc/ with hipcc.

Usage: python -m paper_2211_12487_amd.build   (or __graft_entry__.build())
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = ["csrc/kernels.hip", "csrc/eig.hip", "csrc/proj.hip", "csrc/proj_lp.hip", "csrc/proj_short.hip", "csrc/ttice.hip", "csrc/server.hip",
       "csrc/lanczos.hip", "csrc/gemm_mx.hip", "csrc/gemm_mx_lp.hip"]
OUT = os.path.join(HERE, "libttice.so")
ARCH = os.environ.get("TTICE_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "--offload-arch=" + ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-fvisibility=hidden",
    "-Wall",
    "-Wno-unused-function",
    # packed FP32 instructions stay off in every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


def build(verbose: bool = True) -> str:
    """Compile every source to an object in parallel (one hipcc each: the
    sources share no device code), then link the shared library."""
    from concurrent.futures import ThreadPoolExecutor
    import tempfile
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    srcs = [os.path.join(HERE, s) for s in SRC]
    tmp = OUT + ".tmp"
    with tempfile.TemporaryDirectory(prefix="ttice_build_") as td:
        objs = [os.path.join(td, os.path.basename(s) + ".o") for s in srcs]
        cmds = [[hipcc] + [f for f in FLAGS if f != "-shared"] + ["-c", s, "-o", o] for s, o in zip(srcs, objs)]
        if verbose:
            for c in cmds:
                print(" ".join(c), flush=True)
        jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
        with ThreadPoolExecutor(jobs) as ex:
            for r in ex.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds):
                if r.stdout or r.stderr:
                    print(r.stdout + "\n".join(l for l in r.stderr.splitlines()
                                                if "packed-fp32-ops" not in l), flush=True)
                if r.returncode != 0:
                    raise subprocess.CalledProcessError(r.returncode, r.args)
        link = [hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC"] + objs + ["-o", tmp]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.run(link, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    build()
    sys.exit(0)
