"""Each planted mistake in the oracle (a dropped term, a wrong sign, a
swapped operand, a wrong index rule) must trip at least one pin.

The mistakes are compiled into separate builds of the oracle with
``-DPSREF_MUTANT=n``; the default build has none of them."""
import os

import pytest

import pins
from oracle import psref

MUTANTS = {
    1: "curl: sign of one component",
    2: "projection: k(k.v)/|k|^2 term dropped",
    3: "dealiasing: 9|k|^2 <= N^2 kept",
    4: "spectrum: weight 2 on the kx = N/2 plane",
    5: "RK2: second stage evaluated at z^n",
    6: "nonlinear term: 1/N^3 normalisation dropped",
    7: "MHD: sign of the induction term",
    8: "inverse transform: forward twiddles",
    9: "curl: Nyquist derivative not zeroed",
    10: "nonlinear term: w x u instead of u x w",
    11: "RK2: first stage with dt instead of dt/2",
    12: "spectrum: shells by floor(|k|)",
    13: "rotation: Coriolis term not projected",
    14: "rotation: Omega x u instead of 2 Omega x u",
    15: "box: viscous term with the index |n|^2",
    16: "box: curl without the factors 2 pi / L",
    17: "grid: dealiasing sphere of nx on every axis",
    18: "MHD: nu and eta swapped in the cross term of the resistive coupling",
    19: "MHD diagnostics: b taken as (z- - z+)/2",
    20: "MHD diagnostics: u = z+ + z- without the 1/2",
}


@pytest.mark.parametrize("n", sorted(MUTANTS), ids=lambda n: f"m{n}")
def test_mutant_is_caught(n, tmp_path):
    lib = psref.build(mutant=n, out=os.path.join(str(tmp_path), f"libpsref_m{n}.so"))
    o = psref.Oracle(lib)
    caught = []
    for pin in pins.ALL_PINS:
        try:
            pin(o)
        except Exception:  # a pin that cannot even run on the output also fails
            caught.append(pin.__name__)
    assert caught, f"mutant {n} ({MUTANTS[n]}) passed every pin"
