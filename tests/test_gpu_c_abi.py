"""The C ABI from a plain C program (tests/c_abi/solve_from_c.c, built by
__graft_entry__.build()): no Python binding and no torch in the process; the program
checks the solve on the host against the library's right-hand side and operator."""
import json
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "c_abi", "solve_from_c")


def test_plain_c_program_solves_through_the_abi():
    if not os.path.exists(EXE):
        pytest.fail("tests/c_abi/solve_from_c is not built: run __graft_entry__.build()")
    print("running", EXE, flush=True)
    out = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    print(out.stdout, out.stderr, flush=True)
    assert out.returncode == 0, (out.stdout, out.stderr)
    rec = json.loads(out.stdout.strip().splitlines()[-1])
    assert rec["ok"] == 1 and rec["status"] == 0
    assert rec["host_rel_resid"] <= 1.05e-10
    assert rec["outer_iters"] >= 2          # mixed precision: FP64 refinement steps
