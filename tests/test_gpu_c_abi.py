"""The C ABI from plain C: tests/c/psweep_abi_demo.c (built by the build step)
allocates with hipMalloc, sweeps a case with a known answer (a textured wall
exactly on one plane) and checks it, with no Python in the path."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c", "psweep_abi_demo")


def test_c_program_sweeps_a_known_wall():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert os.path.exists(EXE), "tests/c/psweep_abi_demo is built by __graft_entry__.build()"
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "PASS" in r.stdout
