"""The residue (CRT) kernels' integer and float steps, replayed on the host
in the same precisions (tests/crt_arith_check.c), against exact residues:
exhaustively over every int32 |x| <= 2^26 for all fifteen moduli, plus the
fold of larger sums and the exact pieces of operands up to 2^53."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(__file__)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_crt_reduction_steps_exact(tmp_path):
    exe = str(tmp_path / "crt_arith_check")
    src = os.path.join(HERE, "crt_arith_check.c")
    subprocess.run(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", src, "-o", exe, "-lm"],
                   check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("0 mismatches")
