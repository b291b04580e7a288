"""Mutation check of the oracle pins: plant a mistake in the oracle (a
compile-time switch in the C source), rebuild it into a temporary library
and require that the pin suite rejects it.  Everything runs on the CPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = [
    "ORC_PLANT_AB_SIGN",          # wrong sign of alpha-beta doubles
    "ORC_PLANT_AB_INDEX",         # (pr|qs) instead of (pq|rs): transposed operand
    "ORC_PLANT_SS_EXCHANGE",      # (pq|rs) + (ps|rq): wrong exchange sign
    "ORC_PLANT_DROP_SS_SINGLE",   # dropped same-spin term of single excitations
    "ORC_PLANT_SINGLE_NOSIGN",    # phase of single excitations ignored
    "ORC_PLANT_DROP_AB_DIAG",     # dropped alpha-beta Coulomb term of the diagonal
    "ORC_PLANT_KEEP_GE",          # keep rule |I| >= tau instead of |I| > tau
    "ORC_PLANT_DIAG_ROWSUM",      # diagonal: the j == I filter dropped (whole row summed)
    "ORC_PLANT_DIAG_UNSCREENED",  # diagonal: screened units counted
    "ORC_PLANT_GAS_LEVEL",        # two-space restriction: level counted from n, not the boundary
]

PINS = ("reference_energy or hermiticity or noninteracting or kronecker or rotation "
        "or swap or strict or term_counts_integral or diag_ or gas_")


@pytest.mark.parametrize("macro", MUTANTS)
def test_pins_reject_planted_mistake(macro, tmp_path):
    sys.path.insert(0, ROOT)
    from oracle.build import build
    lib = build(out=str(tmp_path / f"liboracle_{macro}.so"), defines=[macro])
    env = dict(os.environ, ISCI_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-k", PINS],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1, f"pins did not catch {macro}:\n{r.stdout[-2000:]}"
    assert "failed" in r.stdout


# Mistakes planted in the numpy part of the oracle (an environment switch
# read when the module loads).
PY_MUTANTS = [
    "D2_AB_NO_BETA_SIGN",    # two-body alpha-beta block: beta replacement sign dropped
    "D2_AA_SWAP_QS",         # two-body alpha-alpha block: annihilator indices q and s exchanged
    "D1_HALF_SIGN",          # phase of a+_p ignored (only a_q's counted)
    "D1_LONG_ROW",           # alpha dot over the longer row: reads past the shorter one
    "D1_BETA_PAST_ALPHA",    # beta replacement signed by the alpha creators it passes
]


@pytest.mark.parametrize("plant", PY_MUTANTS)
def test_density_pins_reject_planted_mistake(plant):
    env = dict(os.environ, ISCI_ORACLE_PLANT=plant)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-k", "density"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1, f"pins did not catch {plant}:\n{r.stdout[-2000:]}"
    assert "failed" in r.stdout
