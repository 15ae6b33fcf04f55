"""Pins of the oracle's algebraic interpolation (Sec. 2.3): the pivot-block
inverse, the contraction V = A[:, tau] P and the interpolation basis.

* The inverse on matrices whose inverses are known in closed form (2 x 2
  real and complex, a permutation that needs row exchanges, a triangular
  matrix) and M P = I on a seeded complex matrix.
* The contraction with P a permutation or a diagonal picks and scales
  columns exactly; a 2 x 2 product checked by hand.
* Interpolation reproduces every column of an exactly rank-k matrix
  (A = B C): V A[t~, :] = A to rounding, and the pivot rows of V are the
  identity.  A matrix of higher rank is not reproduced (the pin would catch
  an inverse or product that ignores part of A).
"""
import numpy as np
import pytest

import oracle


def test_inverse_closed_forms():
    M = np.array([[4.0, 7.0], [2.0, 6.0]])
    assert np.allclose(oracle.inverse(M), np.array([[6.0, -7.0], [-2.0, 4.0]]) / 10.0,
                       rtol=0, atol=1e-15)
    C = np.array([[1.0, 1j], [0.0, 2.0]])
    assert np.allclose(oracle.inverse(C), np.array([[1.0, -0.5j], [0.0, 0.5]]), rtol=0, atol=1e-15)
    Pm = np.array([[0.0, 1.0, 0.0], [0.0, 0.0, 1.0], [1.0, 0.0, 0.0]])
    assert np.array_equal(oracle.inverse(Pm), Pm.T)  # needs row exchanges, exact
    T = np.array([[2.0, 0.0, 0.0], [3.0, 4.0, 0.0], [1.0, 5.0, 8.0]])
    Ti = np.array([[0.5, 0.0, 0.0], [-0.375, 0.25, 0.0], [0.171875, -0.15625, 0.125]])
    assert np.allclose(oracle.inverse(T), Ti, rtol=0, atol=1e-15)
    assert oracle.inverse(np.array([[-4.0]]))[0, 0] == -0.25


def test_inverse_residual_seeded():
    rng = np.random.Generator(np.random.PCG64(3))
    M = rng.standard_normal((40, 40)) + 1j * rng.standard_normal((40, 40))
    P = oracle.inverse(M)
    assert np.abs(M @ P - np.eye(40)).max() <= 1e-12
    assert np.abs(P @ M - np.eye(40)).max() <= 1e-12


def test_inverse_singular_rejected():
    with pytest.raises(ValueError):
        oracle.inverse(np.array([[1.0, 2.0], [2.0, 4.0]]) * 0.0)


def test_contract_picks_and_scales_columns():
    rng = np.random.Generator(np.random.PCG64(4))
    A = rng.standard_normal((9, 12)) + 1j * rng.standard_normal((9, 12))
    tau = np.array([7, 2, 11])
    perm = np.array([[0.0, 0.0, 1.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    # column j of V is sum_l A[:, tau_l] P[l, j]
    assert np.array_equal(oracle.contract(A, tau, perm), A[:, [2, 11, 7]])
    D = np.diag([2.0, -0.5, 4.0])
    assert np.array_equal(oracle.contract(A, tau, D), A[:, tau] * np.array([2.0, -0.5, 4.0]))
    A2 = np.array([[1.0, 2.0, 3.0], [4.0, 5.0, 6.0]])
    P2 = np.array([[1.0, 2.0], [3.0, 4.0]])
    # A2[:, [2, 0]] = [[3, 1], [6, 4]];  times P2 = [[6, 10], [18, 28]]
    assert np.array_equal(oracle.contract(A2, [2, 0], P2).real, np.array([[6.0, 10.0], [18.0, 28.0]]))


@pytest.mark.parametrize("cplx", [False, True])
def test_interpolation_reproduces_rank_k(cplx):
    rng = np.random.Generator(np.random.PCG64(5 + cplx))
    n, acols, k = 50, 30, 7
    B = rng.standard_normal((n, k)) + (1j * rng.standard_normal((n, k)) if cplx else 0)
    C = rng.standard_normal((k, acols)) + (1j * rng.standard_normal((k, acols)) if cplx else 0)
    A = B @ C
    prow = np.array([3, 17, 22, 29, 31, 40, 44])
    tau = np.array([0, 5, 9, 12, 18, 21, 27])
    V, P = oracle.interp_basis(A, prow, tau)
    assert np.abs(V[prow] - np.eye(k)).max() <= 1e-12
    assert np.abs(V @ A[prow, :] - A).max() <= 1e-11 * np.abs(A).max()
    assert np.abs(P @ A[np.ix_(prow, tau)] - np.eye(k)).max() <= 1e-12
    # one rank more: the k pivots can no longer reproduce A
    A1 = A + np.outer(rng.standard_normal(n), rng.standard_normal(acols))
    V1, _ = oracle.interp_basis(A1, prow, tau)
    assert np.abs(V1 @ A1[prow, :] - A1).max() > 1e-3 * np.abs(A1).max()
