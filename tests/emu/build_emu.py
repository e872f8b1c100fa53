"""Build the host-emulation variant of libttice (tests only): the library's
own .hip sources compiled by g++ against tests/emu/hipemu.h, with
AddressSanitizer, so kernel indexing and host logic can be checked on a
machine without a GPU.  Output: a path under the given directory."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRCS = [os.path.join(ROOT, "paper_2211_12487_amd", "csrc", f) for f in ("kernels.hip", "eig.hip", "proj.hip", "proj_short.hip", "ttice.hip", "server.hip",
                                                                          "lanczos.hip", "gemm_mx.hip")]


def asan_runtime() -> str:
    return subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True, text=True,
                          check=True).stdout.strip()


def build(outdir: str, asan: bool = True) -> str:
    os.makedirs(outdir, exist_ok=True)
    out = os.path.join(outdir, "libttice_emu.so")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fPIC", "-shared", "-pthread", "-w",
           "-I", HERE, "-I", os.path.join(ROOT, "include")]
    if os.environ.get("TTICE_EMU_DEBUG"):
        cmd += ["-DTTICE_EMU_DEBUG", "-include", "cstdio"]
    if asan:
        cmd += ["-fsanitize=address", "-fno-omit-frame-pointer"]
    objs = []
    for src in SRCS + [os.path.join(HERE, "hipemu.cpp"), os.path.join(HERE, "eig_probe.cpp"),
                          os.path.join(HERE, "proj_probe.cpp"), os.path.join(HERE, "proj_lp_stub.cpp"),
                          os.path.join(HERE, "gemm_probe.cpp"), os.path.join(HERE, "gemm_mx_lp_stub.cpp")]:
        obj = os.path.join(outdir, os.path.basename(src) + ".o")
        lang = ["-x", "c++"] if src.endswith(".hip") else []
        subprocess.run(cmd + ["-c"] + lang + [src, "-o", obj], check=True)
        objs.append(obj)
    subprocess.run(cmd + objs + ["-o", out], check=True)
    return out


if __name__ == "__main__":
    import sys
    import tempfile
    print(build(sys.argv[1] if len(sys.argv) > 1 else tempfile.mkdtemp(prefix="ttice_emu_")))
