"""Host-emulation run of the library's own HIP sources (CPU tier).

tests/emu/build_emu.py compiles paper_2211_12487_amd/csrc/*.hip with g++
against a small HIP emulation layer and AddressSanitizer; the parity cases
of tests/emu/emu_cases.py then run against the oracle in subprocesses with
the ASan runtime preloaded.  This checks kernel indexing and the engine's
control flow (including failure injection) without a GPU; the GPU tier
checks the same cases on the device."""
import os
import subprocess
import sys
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "emu"))

import build_emu  # noqa: E402
from emu_cases import CASES  # noqa: E402


@pytest.fixture(scope="module")
def emu_lib():
    td = tempfile.mkdtemp(prefix="ttice_emu_")
    return build_emu.build(td, asan=True)


def test_emulated_kernels_match_oracle(emu_lib):
    env = dict(os.environ)
    env["LD_PRELOAD"] = build_emu.asan_runtime()
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    script = os.path.join(HERE, "emu", "emu_cases.py")
    procs = {name: subprocess.Popen([sys.executable, script, emu_lib, name], env=env,
                                    stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
             for name in CASES}
    failures = []
    for name, p in procs.items():
        out, _ = p.communicate(timeout=900)
        if p.returncode != 0:
            failures.append(f"--- {name} (rc={p.returncode})\n{out[-3000:]}")
    assert not failures, "\n".join(failures)
