"""The CPU oracle against its pins (see ``pins.py``): no GPU needed.  The
product pins run with the oracle's plain loop and again with its OpenMP loop
over rows (8 threads), the configuration the GPU parity tests use."""
import pytest

import pins

PRODUCT_PINS = [pins.pin_golden_products, pins.pin_dense_bruteforce, pins.pin_minplus_two_walks,
                pins.pin_scipy_int64, pins.pin_numpy_fp64, pins.pin_stencil_small_boundary,
                pins.pin_identity_and_relabel, pins.pin_int64_invariants, pins.pin_minplus_invariants,
                pins.pin_boolean_bit_slices, pins.pin_transpose, pins.pin_stencil_closed_form,
                pins.pin_general_update]


@pytest.mark.parametrize("pin", pins.ALL_PINS + [pins.pin_stencil_closed_form],
                         ids=lambda f: f.__name__)
def test_pin(orc, pin):
    pin(orc)


@pytest.mark.parametrize("pin", PRODUCT_PINS, ids=lambda f: f.__name__)
def test_pin_threaded(orc, pin, monkeypatch):
    monkeypatch.setattr(pins, "NTHREADS", 8)
    pin(orc)
