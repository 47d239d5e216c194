"""Pins of the 1-D LGL SBP operator (Notation section, Definition "SBP")."""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

from oracle import operators


@pytest.mark.parametrize("p", list(range(1, 16)))
def test_sbp_definition(p):
    op = operators.SBP1D(p)
    x = op.x
    # 1. exact on monomials up to degree p
    for j in range(p + 1):
        lhs = op.D @ x ** j
        rhs = j * x ** (j - 1) if j > 0 else np.zeros_like(x)
        assert np.abs(lhs - rhs).max() < 1e-12 * max(1, p * p)
    # 2. P symmetric positive definite (diagonal, positive weights), sum = 2
    assert np.all(op.w > 0)
    assert abs(op.w.sum() - 2.0) < 1e-14
    # 3. Q + Q^T = E, S skew
    assert np.abs(op.Q + op.Q.T - op.E).max() < 1e-13 * max(1, p)
    assert np.abs(op.S + op.S.T).max() < 1e-13 * max(1, p)
    # Lobatto quadrature exact to degree 2p - 1
    for k in range(2 * p):
        exact = (1.0 - (-1.0) ** (k + 1)) / (k + 1)
        assert abs((op.w * x ** k).sum() - exact) < 1e-14


def test_textbook_p1_p2():
    op = operators.SBP1D(1)
    assert np.allclose(op.x, [-1, 1], atol=0, rtol=0)
    assert np.allclose(op.w, [1, 1], atol=1e-16)
    assert np.allclose(op.D, [[-0.5, 0.5], [-0.5, 0.5]], atol=1e-16)
    op = operators.SBP1D(2)
    assert np.allclose(op.x, [-1, 0, 1], atol=1e-16)
    assert np.allclose(op.w, [1 / 3, 4 / 3, 1 / 3], atol=1e-16)
    assert np.allclose(op.D, [[-1.5, 2, -0.5], [-0.5, 0, 0.5], [0.5, -2, 1.5]], atol=1e-15)


def test_textbook_lgl_p3_p4():
    LD = np.longdouble
    op = operators.SBP1D(3)
    a = 1 / np.sqrt(LD(5))
    assert np.abs(op.x_ld - np.array([-1, -a, a, 1], dtype=LD)).max() < 1e-18
    assert np.abs(op.w_ld - np.array([1, 5, 5, 1], dtype=LD) / 6).max() < 1e-18
    op = operators.SBP1D(4)
    b = np.sqrt(LD(3) / 7)
    assert np.abs(op.x_ld - np.array([-1, -b, 0, b, 1], dtype=LD)).max() < 1e-18
    assert np.abs(op.w_ld - np.array([LD(1) / 10, LD(49) / 90, LD(32) / 45, LD(49) / 90, LD(1) / 10])).max() < 1e-18


@pytest.mark.parametrize("p", [3, 5, 8, 12])
def test_derivative_matches_vandermonde(p):
    """Collocation derivative against an independent construction D = V_x V^{-1} in the Legendre basis."""
    op = operators.SBP1D(p)
    V = npleg.legvander(op.x, p)
    Vx = np.stack([npleg.legval(op.x, npleg.legder(np.eye(p + 1)[k])) for k in range(p + 1)], axis=1)
    D = Vx @ np.linalg.inv(V)
    assert np.abs(D - op.D).max() < 1e-11 * p * p
