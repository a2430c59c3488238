"""The FP64 oracle against its pins (CPU only), and a mutation check showing
that each plausible mistake in the oracle trips at least one pin."""
import os

import numpy as np
import pytest

import oracle
from tests import oracle_pins


@pytest.mark.parametrize("pin", oracle_pins.ALL_PINS, ids=lambda p: p.__name__)
def test_oracle_pin(orc, pin):
    pin(orc)


def test_oracle_rejects_bad_shapes(orc):
    x = np.zeros((4, 4))
    for n0, n1 in [(5, 1), (1, 5), (0, 2), (2, 0)]:
        with pytest.raises(ValueError):
            orc.swdft2d(x, n0, n1)
    with pytest.raises(ValueError):
        orc.swdft2d(x, 2, 2, windows=(np.array([3]), np.array([0])))


def test_oracle3d_rejects_bad_shapes(orc):
    x = np.zeros((4, 4, 4))
    for n in [(5, 1, 1), (1, 5, 1), (1, 1, 5), (0, 2, 2)]:
        with pytest.raises(ValueError):
            orc.swdft3d(x, *n)
    with pytest.raises(ValueError):
        orc.swdft3d(x, 2, 2, 2, windows=(np.array([0]), np.array([0]), np.array([3])))


MUTANTS = {
    1: "inverse twiddle sign",
    2: "last window column dropped",
    3: "window transposed",
    4: "off-by-one column",
    5: "k0 and k1 swapped",
    6: "adjoint without conjugate",
    7: "adjoint window range off by one",
    8: "3D: last slice of every window dropped",
    9: "3D: k1 and k2 swapped",
    10: "3D: axis-2 roots of the wrong length",
    11: "3D adjoint without conjugate",
    12: "3D adjoint axis-1 window range off by one",
}


@pytest.mark.parametrize("mutation", sorted(MUTANTS), ids=lambda m: MUTANTS[m])
def test_pins_catch_mutant(tmp_path, mutation):
    path = oracle.compile_library(str(tmp_path / f"liboracle_m{mutation}.so"), mutation=mutation,
                                  openmp=False)
    mutant = oracle.Oracle(path)
    failed = []
    for pin in oracle_pins.ALL_PINS:
        try:
            pin(mutant)
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, f"no pin caught mutation {mutation} ({MUTANTS[mutation]})"
