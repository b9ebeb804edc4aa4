"""The C ABI from plain C: tests/native/abi_roundtrip.c links libpyrit.so and
the HIP runtime only (no Python, no torch) and encodes, decodes, runs a
one-item batch in both launch forms and checks two error paths."""
import os
import subprocess

import pytest

from tests.native import build as native_build


@pytest.mark.gpu
def test_c_consumer_round_trip():
    exe = native_build.EXE
    if not os.path.exists(exe):
        exe = native_build.build_abi_roundtrip()
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert r.stdout.strip().endswith("ok")
