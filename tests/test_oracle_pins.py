"""The CPU oracle against its pins (see ``pins.py``): no GPU needed."""
import pytest

import pins


@pytest.mark.parametrize("pin", pins.ALL_PINS + [pins.pin_stencil_closed_form],
                         ids=lambda f: f.__name__)
def test_pin(orc, pin):
    pin(orc)
