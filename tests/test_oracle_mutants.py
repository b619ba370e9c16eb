"""Each planted mistake in the oracle (a wrong sign, a dropped term, a wrong
kept-index rule, a wrong slice radix, a missing conjugate, a transposed
output) must make at least one pin fail.  Mistakes are planted only in the CPU
oracle, through the ORACLE_PLANT_* build macros."""

import os

import pytest

import tests.test_oracle as pins
from oracle import contract as oc

PIN_SET = [
    pins.test_cfg1_every_amplitude_matches_statevector,
    pins.test_open_outputs_match_statevector,
    lambda o: pins.test_rrg_matches_bruteforce(o, 0),
    lambda o: pins.test_hyperedges_outputs_nonbinary_match_bruteforce(o, 0),
    pins.test_matrix_chain_is_matmul,
    pins.test_outer_dot_and_batch,
    pins.test_slice_id_radix_matches_projection,
    lambda o: pins.test_grad_matches_bruteforce_environments(o, 0),
    pins.test_grad_circuit_statevector_environments,
]


def _failing_pins(lib):
    failed = 0
    for pin in PIN_SET:
        try:
            pin(lib)
        except (AssertionError, oc.OracleError, ValueError):
            failed += 1
    return failed


@pytest.mark.parametrize("mutant", ["SIGN", "DROP", "KEPT", "SLICE", "CONJ", "ROOT"])
def test_planted_mistake_is_caught(tmp_path, mutant):
    path = str(tmp_path / f"liboracle_{mutant}.so")
    oc.build(force=True, path=path, defines=[f"ORACLE_PLANT_{mutant}"])
    try:
        oc.use_library(path)
        assert _failing_pins(oc) >= 1
    finally:
        oc.use_library(None)


def test_clean_build_passes_every_pin():
    oc.use_library(None)
    assert _failing_pins(oc) == 0
    assert os.path.exists(oc._LIB)
