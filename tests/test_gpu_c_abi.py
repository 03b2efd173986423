"""The C ABI from a plain C program (tests/c/abi_solve.c, built by
build()): lower triangle uploaded, completed on the device, lowest
eigenpairs of a dense Hermitian matrix with a known spectrum, checked on
the host."""
import os
import subprocess

import pytest

from tests.gpu_util import torch_cuda

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c", "abi_solve")


def test_plain_c_program_solves_through_the_abi():
    torch_cuda()
    assert os.path.exists(EXE), "tests/c/abi_solve is missing: run __graft_entry__.build()"
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().splitlines()[-1] == "ok"
