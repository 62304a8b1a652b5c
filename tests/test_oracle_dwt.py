"""Pins of the oracle's wavelet transform W (Eq. (fewha): orthonormal, compactly supported).

Nothing here re-derives the oracle's code: each check is a property the Daubechies-3
periodic transform must have (filter identities, orthogonality at every level size,
vanishing moments, closed forms for constant fields, band orientation, the Haar reduction
of a length-2 periodic level).
"""
import numpy as np
import pytest

from oracle import db3
from oracle.oracle import dwt1, dwt2, level_of


def test_db3_filter_identities():
    h = db3()
    assert abs(h.sum() - np.sqrt(2)) < 1e-15
    assert abs((h * h).sum() - 1) < 1e-15
    # double-shift orthogonality
    assert abs(np.dot(h[:-2], h[2:])) < 1e-15
    assert abs(np.dot(h[:-4], h[4:])) < 1e-15
    # three vanishing moments of the high-pass partner: sum (-1)^n n^p h_n = 0, p = 0, 1, 2
    n = np.arange(6)
    for p in range(3):
        assert abs(np.sum((-1.0) ** n * n ** p * h)) < 1e-13
    # extremal (minimum) phase: no zero of H outside the unit circle
    assert np.all(np.abs(np.roots(h)) < 1 + 1e-5)
    # literature values of db3 (Daubechies 1988), 8 digits
    ref = [0.33267055, 0.80689151, 0.45987750, -0.13501102, -0.08544127, 0.03522629]
    assert np.allclose(h, ref, atol=5e-9)


@pytest.mark.parametrize("N", [2, 4, 6, 8, 16, 64])
def test_dwt1_orthogonal_every_length(N):
    F = np.stack([dwt1(e) for e in np.eye(N)], axis=1)   # analysis matrix
    assert np.abs(F @ F.T - np.eye(N)).max() < 1e-14
    G = np.stack([dwt1(e, inverse=True) for e in np.eye(N)], axis=1)
    assert np.abs(G - F.T).max() < 1e-15                   # synthesis is the transpose


def test_dwt1_length2_is_haar():
    x = np.array([3.0, -1.25])
    a, d = dwt1(x)
    assert abs(a - (x[0] + x[1]) / np.sqrt(2)) < 1e-15
    assert abs(d - (x[0] - x[1]) / np.sqrt(2)) < 1e-15


def test_dwt1_highpass_kills_quadratics_away_from_wrap():
    N = 64
    m = np.arange(N, dtype=float)
    for x in (np.ones(N), m, 0.01 * m * m - 0.3 * m + 2):
        out = dwt1(x)
        d = out[N // 2:]
        k = np.arange(N // 2)
        inner = 2 * k + 5 < N
        assert np.abs(d[inner]).max() < 1e-11 * max(1, np.abs(x).max())
        assert np.abs(d[~inner]).max() > 1e-6 or np.ptp(x) == 0


@pytest.mark.parametrize("n,J", [(4, 1), (4, 2), (8, 3), (16, 2), (16, 4), (32, 4), (32, 5)])
def test_dwt2_orthogonal(n, J):
    W = np.stack([dwt2(e.reshape(n, n), J).ravel() for e in np.eye(n * n)], axis=1)
    assert np.abs(W @ W.T - np.eye(n * n)).max() < 1e-14
    x = np.random.default_rng(3).standard_normal((n, n))
    assert np.abs(dwt2(dwt2(x, J), J, inverse=True) - x).max() < 1e-14


@pytest.mark.parametrize("n,J", [(32, 4), (64, 6), (16, 4)])
def test_constant_field(n, J):
    c = dwt2(np.full((n, n), 1.7), J)
    m = n >> J
    assert np.allclose(c[:m, :m], 1.7 * 2 ** J, rtol=0, atol=1e-12)
    c[:m, :m] = 0
    assert np.abs(c).max() < 1e-12


def test_band_orientation():
    """A field that varies only along x (columns) has no y-detail: the bottom-left and
    bottom-right bands vanish at every level; the top-right (x-detail) band does not."""
    n, J = 32, 3
    rng = np.random.default_rng(5)
    fx = np.tile(rng.standard_normal(n), (n, 1))          # row = y, col = x
    c = dwt2(fx, J)
    for s in range(1, J + 1):
        m = n >> s
        assert np.abs(c[m:2 * m, :m]).max() < 1e-13       # x-low / y-high
        assert np.abs(c[m:2 * m, m:2 * m]).max() < 1e-13  # HH
        assert np.abs(c[:m, m:2 * m]).max() > 1e-3        # x-high / y-low
    cy = dwt2(fx.T.copy(), J)
    for s in range(1, J + 1):
        m = n >> s
        assert np.abs(cy[:m, m:2 * m]).max() < 1e-13
        assert np.abs(cy[m:2 * m, :m]).max() > 1e-3


def test_level_map():
    n, J = 32, 3
    assert level_of(n, J, 0, 0) == (3, 0)
    assert level_of(n, J, 3, 3) == (3, 0)
    assert level_of(n, J, 0, 4) == (3, 1)
    assert level_of(n, J, 4, 0) == (3, 2)
    assert level_of(n, J, 5, 7) == (3, 3)
    assert level_of(n, J, 0, 8) == (2, 1)
    assert level_of(n, J, 31, 31) == (1, 3)
    assert level_of(n, J, 16, 3) == (1, 2)
    assert level_of(n, J, 15, 16) == (1, 1)


def test_kronecker_structure_one_level():
    """A single 2D level equals F X F^T with the 1D analysis matrix F (rows along x first)."""
    n = 16
    F = np.stack([dwt1(e) for e in np.eye(n)], axis=1)
    X = np.random.default_rng(9).standard_normal((n, n))
    assert np.abs(dwt2(X, 1) - F @ X @ F.T).max() < 1e-13
