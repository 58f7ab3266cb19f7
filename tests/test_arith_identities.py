"""Exhaustive host checks of two arithmetic identities of the GPU kernels (CPU only).

tests/arith_identities.c restates the packed zigzag undo (unzigzag_pk: every
pair of zigzag values below 2^12, q = 0..4, against the definition of
Sec. 3.2) and the division by 255 of the interpolation (div255: every float
in [0, 255] against the IEEE quotient) and compares them case by case.  The
kernels themselves are covered on the GPU by the parity tests; this pins the
identities their comments state.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(not shutil.which("gcc"), reason="needs gcc")
def test_arith_identities_hold_exhaustively(tmp_path):
    exe = str(tmp_path / "arith_identities")
    # ISO C (no contraction of a * b + c into a fused operation), OpenMP over the host's cores
    subprocess.run(["gcc", "-std=c11", "-O2", "-fopenmp", os.path.join(HERE, "arith_identities.c"), "-o", exe, "-lm"],
                   check=True, timeout=120)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "unzigzag_pk: 83886080 cases, 0 differ" in r.stdout, r.stdout
    assert "div255: 1132396545 cases, 0 differ" in r.stdout, r.stdout
