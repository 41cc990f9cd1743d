"""Pins for the SER metric (METHODS, reconstruction and analysis)."""
import numpy as np
import pytest

import oracle


def test_ser_hand_cases():
    x = np.ones((1, 4, 4, 2), complex)
    assert oracle.ser(x * 1.1, x) == pytest.approx(20.0, abs=1e-12)
    assert oracle.ser(x + 0.01j, x) == pytest.approx(40.0, abs=1e-12)
    assert oracle.rel_err(x * 1.001, x) == pytest.approx(1e-3, rel=1e-9)
