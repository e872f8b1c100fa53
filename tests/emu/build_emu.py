"""Build the host-emulation variant of libttice (tests only): the library's
own .hip sources compiled by g++ against tests/emu/hipemu.h, with
AddressSanitizer, so kernel indexing and host logic can be checked on a
machine without a GPU.  Output: a path under the given directory."""
import concurrent.futures
import os
import re
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRCS = [os.path.join(ROOT, "paper_2211_12487_amd", "csrc", f) for f in ("kernels.hip", "eig.hip", "proj.hip", "proj_short.hip", "ttice.hip", "server.hip",
                                                                          "lanczos.hip", "gemm_mx.hip")]


def asan_runtime() -> str:
    return subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True, text=True,
                          check=True).stdout.strip()


_SHARED = re.compile(r"__shared__\s+([^;]*);")


def _declarators(decl: str):
    """Names declared by the text between __shared__ and its semicolon (type,
    attributes, then one or more declarators separated by top-level commas)."""
    depth, parts, cur = 0, [], ""
    for ch in decl:
        depth += ch in "([{"
        depth -= ch in ")]}"
        if ch == "," and depth == 0:
            parts.append(cur)
            cur = ""
        else:
            cur += ch
    parts.append(cur)
    names = []
    for k, part in enumerate(parts):
        head = part.split("[")[0].strip()
        names.append(re.findall(r"[A-Za-z_][A-Za-z_0-9]*", head)[-1])
    return names


def with_lds_marks(text: str) -> str:
    """Each static LDS declaration followed by HIPEMU_LDS(name) for every name
    it declares (hipemu.h fills them with 0xff at the start of each block)."""
    def mark(m):
        return m.group(0) + "".join(f" HIPEMU_LDS({n});" for n in _declarators(m.group(1)))
    return _SHARED.sub(mark, text)


def build(outdir: str, asan: bool = True) -> str:
    os.makedirs(outdir, exist_ok=True)
    out = os.path.join(outdir, "libttice_emu.so")
    csrc = os.path.join(ROOT, "paper_2211_12487_amd", "csrc")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fPIC", "-shared", "-pthread", "-w",
           "-I", HERE, "-I", os.path.join(ROOT, "include"), "-I", csrc]
    if os.environ.get("TTICE_EMU_DEBUG"):
        cmd += ["-DTTICE_EMU_DEBUG", "-include", "cstdio"]
    if asan:
        cmd += ["-fsanitize=address", "-fno-omit-frame-pointer"]
    jobs = []
    for src in SRCS + [os.path.join(HERE, "hipemu.cpp"), os.path.join(HERE, "eig_probe.cpp"),
                          os.path.join(HERE, "proj_probe.cpp"), os.path.join(HERE, "proj_lp_stub.cpp"),
                          os.path.join(HERE, "gemm_probe.cpp"), os.path.join(HERE, "gemm_mx_lp_stub.cpp")]:
        obj = os.path.join(outdir, os.path.basename(src) + ".o")
        if src.endswith(".hip"):
            # the marked copy sits in outdir; its quoted includes resolve
            # through -I csrc
            marked = os.path.join(outdir, os.path.basename(src) + ".cpp")
            with open(src) as f, open(marked, "w") as g:
                g.write(f'#line 1 "{src}"\n' + with_lds_marks(f.read()))
            src = marked
        jobs.append(cmd + ["-c", src, "-o", obj])
    with concurrent.futures.ThreadPoolExecutor(max_workers=4) as pool:
        for r in pool.map(lambda c: subprocess.run(c, capture_output=True, text=True), jobs):
            if r.returncode != 0:
                raise RuntimeError("emulation build failed:\n" + r.stdout + r.stderr)
    subprocess.run(cmd + [j[-1] for j in jobs] + ["-o", out], check=True)
    return out


if __name__ == "__main__":
    import sys
    import tempfile
    print(build(sys.argv[1] if len(sys.argv) > 1 else tempfile.mkdtemp(prefix="ttice_emu_")))
