"""Pins of the oracle's Radau IIA tableau and Crout factor (not gpu)."""
import math

import numpy as np
import pytest

from oracle import tableau


def test_s1_is_backward_euler():
    A, b, c = tableau.radau_iia(1)
    assert np.allclose(A, [[1.0]]) and np.allclose(b, [1.0]) and np.allclose(c, [1.0])


def test_s2_textbook_values():
    # Radau IIA order 3 (Hairer & Wanner, Solving ODEs II, Table IV.5.5)
    A, b, c = tableau.radau_iia(2)
    assert np.allclose(A, [[5 / 12, -1 / 12], [3 / 4, 1 / 4]], atol=1e-15)
    assert np.allclose(b, [3 / 4, 1 / 4], atol=1e-15)
    assert np.allclose(c, [1 / 3, 1.0], atol=1e-15)


def test_s3_textbook_values():
    # Radau IIA order 5 (Hairer & Wanner, Solving ODEs II, Table IV.5.6)
    r6 = math.sqrt(6.0)
    Aref = np.array([
        [(88 - 7 * r6) / 360, (296 - 169 * r6) / 1800, (-2 + 3 * r6) / 225],
        [(296 + 169 * r6) / 1800, (88 + 7 * r6) / 360, (-2 - 3 * r6) / 225],
        [(16 - r6) / 36, (16 + r6) / 36, 1 / 9]])
    A, b, c = tableau.radau_iia(3)
    assert np.allclose(A, Aref, atol=1e-14)
    assert np.allclose(b, Aref[2], atol=1e-14)
    assert np.allclose(c, [(4 - r6) / 10, (4 + r6) / 10, 1.0], atol=1e-14)


@pytest.mark.parametrize("s", [1, 2, 3, 4, 5])
def test_order_conditions_and_stiff_accuracy(s):
    A, b, c = tableau.radau_iia(s)
    for q in range(1, 2 * s):          # quadrature order 2s-1: sum b c^{q-1} = 1/q
        assert abs(b @ c ** (q - 1) - 1.0 / q) < 1e-13
    assert abs(b @ c ** (2 * s - 1) - 1.0 / (2 * s)) > 1e-6   # and not 2s
    assert np.allclose(A.sum(axis=1), c, atol=1e-13)
    assert np.allclose(A[-1], b) and abs(c[-1] - 1.0) < 1e-15


@pytest.mark.parametrize("s", [1, 2, 3])
def test_stability_function_order_and_l_stability(s):
    A, b, _ = tableau.radau_iia(s)
    errs = [abs(tableau.stability_function(A, b, z) - math.exp(z)) for z in (0.1, 0.05)]
    # local error of an order-p method: O(z^{p+1}) with p = 2s-1
    slope = math.log(errs[0] / errs[1]) / math.log(2.0)
    assert abs(slope - 2 * s) < 0.15
    assert abs(tableau.stability_function(A, b, -1e9)) < 1e-8


@pytest.mark.parametrize("s", [1, 2, 3, 4, 5])
def test_crout(s):
    A, _, _ = tableau.radau_iia(s)
    L, U = tableau.crout(A)
    assert np.allclose(L @ U, A, atol=1e-14)
    assert np.allclose(np.triu(L, 1), 0) and np.allclose(np.tril(U, -1), 0)
    assert np.allclose(np.diag(U), 1.0)
    if s <= 3:
        assert np.all(np.diag(L) > 0)


def test_crout_s2_pivots():
    A, _, _ = tableau.radau_iia(2)
    L, _ = tableau.crout(A)
    assert np.allclose(np.diag(L), [5 / 12, 2 / 5], atol=1e-15)
