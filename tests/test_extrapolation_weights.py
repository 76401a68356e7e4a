"""Host-side weights of the learned start's extrapolation in time
(paper_1610_03918_amd.unet.extrapolation_coefficients): the polynomial through
the last K solutions, or the least-squares polynomial of a lower degree
through them.  Pinned by what fixes them: exact reproduction of every
polynomial up to the degree, minimum sum of squares among the weights that do
so (the least-squares estimate is the best linear unbiased one), and the
weights written out by hand for small cases."""
from math import comb

import numpy as np
import pytest

from paper_1610_03918_amd.unet import extrapolation_coefficients


@pytest.mark.parametrize("K", [1, 2, 3, 4, 5, 6, 8])
def test_interpolation_weights_are_binomial(K):
    w = extrapolation_coefficients(K)
    assert w == [(-1) ** (k + 1) * comb(K, k) for k in range(1, K + 1)]
    assert extrapolation_coefficients(K, K - 1) == w


@pytest.mark.parametrize("K,D", [(5, 3), (6, 3), (8, 3), (8, 2), (6, 2), (5, 0), (7, 4)])
def test_least_squares_weights_reproduce_polynomials_with_least_norm(K, D):
    w = np.array(extrapolation_coefficients(K, D))
    t = -np.arange(1, K + 1, dtype=np.float64)
    for j in range(D + 1):
        # value at t = 0 of t^j: 1 for j = 0, else 0
        assert abs(float(w @ t ** j) - (1.0 if j == 0 else 0.0)) < 1e-9 * K ** j, (K, D, j)
    # any other weights reproducing degree <= D differ by a vector orthogonal
    # to 1, t, .., t^D, and have a larger sum of squares
    V = np.vander(t, D + 1, increasing=True)
    null = np.linalg.svd(V.T)[2][D + 1:]
    r = np.random.default_rng(K * 10 + D)
    for _ in range(5):
        u = w + null.T @ r.standard_normal(null.shape[0])
        assert float(u @ u) > float(w @ w)


def test_small_cases_by_hand():
    # constant fit: the mean of the last K solutions
    assert np.allclose(extrapolation_coefficients(5, 0), [0.2] * 5, rtol=0, atol=1e-12)
    # straight line through 3 points at t = -1, -2, -3, evaluated at 0: 4/3, 1/3, -2/3
    assert np.allclose(extrapolation_coefficients(3, 1), [4 / 3, 1 / 3, -2 / 3], rtol=0, atol=1e-12)
    # cubic through 6 points
    assert np.allclose(extrapolation_coefficients(6, 3), [8 / 3, -4 / 3, -4 / 3, 1 / 3, 4 / 3, -2 / 3],
                       rtol=0, atol=1e-10)
    with pytest.raises(ValueError):
        extrapolation_coefficients(4, 4)
