"""The pins reject a wrong oracle: each planted mistake (OR_MUTANT in
oracle/pyrit_oracle.c, built into a separate library) makes the pin suite
fail.  Runs on the CPU only."""
import concurrent.futures as cf
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    1: "table base x instead of the smallest primitive element",
    2: "antilog index off by one in the product",
    3: "antilog index off by one in the inverse",
    4: "Cauchy points Y_j = j + 1 instead of m + j",
    5: "slices read in reverse bit order",
    6: "last data block dropped from every sum",
    7: "Gauss-Jordan without the row swap",
    8: "erased parity not re-encoded after recovery",
    9: "survivor rows of C taken in reverse column order",
}


def _run(mutant, tmp):
    env = dict(os.environ, PYRIT_ORACLE_MUTANT=str(mutant), PYRIT_ORACLE_DIR=str(tmp))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu", os.path.join(ROOT, "tests", "test_oracle.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    failed = [ln for ln in r.stdout.splitlines() if ln.startswith("FAILED")]
    return r.returncode, failed


def test_every_planted_mistake_fails_a_pin(tmp_path):
    with cf.ThreadPoolExecutor(max(1, min(4, (os.cpu_count() or 2) // 2))) as ex:
        res = dict(zip(MUTANTS, ex.map(lambda m: _run(m, tmp_path), MUTANTS)))
    survivors = {m: MUTANTS[m] for m, (rc, _) in res.items() if rc != 1}
    assert not survivors, f"planted mistakes not caught by any pin: {survivors}"
    for m, (rc, failed) in res.items():
        assert failed, (m, MUTANTS[m])


@pytest.mark.parametrize("mutant", [0])
def test_unmutated_build_passes(mutant):
    import oracle
    assert oracle._MUTANT == 0
