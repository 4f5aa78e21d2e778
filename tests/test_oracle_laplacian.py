"""Pins of the oracle's 25-point Laplacian (paper Section III; neighbour sets
of Section IV-C; centre counted once as in Section IV-C).

Each test is chosen so that a plausible slip (a wrong weight, a dropped
tap, a transposed axis, a wrong spacing) fails it."""
import numpy as np
import pytest

from _pins import golden_coefficients, kron_laplacian, rel_l2


def _coords(n, h):
    """Coordinates of padded indices 0..n+7 (interior 4..n+3), centred."""
    i = np.arange(n + 8) - 4
    return (i - (n - 1) / 2.0) * h


def _grid(shape, h):
    nz, ny, nx = shape
    dx, dy, dz = h
    z = _coords(nz, dz)[:, None, None]
    y = _coords(ny, dy)[None, :, None]
    x = _coords(nx, dx)[None, None, :]
    return z, y, x


# Polynomial with per-variable degree <= 9 and mixed terms.
_TERMS = [  # (coef, px, py, pz)
    (0.7, 9, 0, 0), (-0.3, 0, 9, 0), (0.45, 0, 0, 9), (0.2, 9, 7, 0), (-0.1, 3, 9, 8),
    (0.05, 8, 8, 9), (1.3, 2, 1, 0), (-0.8, 0, 5, 4), (0.25, 6, 0, 3), (2.0, 0, 0, 0),
    (0.6, 1, 1, 1),
]


def _poly_and_lap(z, y, x):
    p = 0.0
    lap = 0.0
    for a, i, j, k in _TERMS:
        p = p + a * x ** i * y ** j * z ** k
        if i >= 2:
            lap = lap + a * i * (i - 1) * x ** (i - 2) * y ** j * z ** k
        if j >= 2:
            lap = lap + a * j * (j - 1) * x ** i * y ** (j - 2) * z ** k
        if k >= 2:
            lap = lap + a * k * (k - 1) * x ** i * y ** j * z ** (k - 2)
    return p, lap


@pytest.mark.parametrize("h", [(0.21, 0.17, 0.13), (0.1, 0.1, 0.1)])
def test_polynomial_exactness(oracle_lib, h):
    shape = (9, 10, 12)
    z, y, x = _grid(shape, h)
    p, lap = _poly_and_lap(z, y, x)
    p = np.broadcast_to(p, tuple(s + 8 for s in shape)).copy()
    lap = np.broadcast_to(lap, tuple(s + 8 for s in shape))[4:-4, 4:-4, 4:-4]
    got = oracle_lib.laplacian(p, h)
    scale = np.abs(p).max() / min(h) ** 2
    assert np.abs(got - lap).max() <= 1e-12 * scale


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_degree10_error_is_predicted(oracle_lib, axis):
    # For u = q^10 along one axis the rule returns 90 q^8 - 1152 h^8 exactly
    # (the only non-vanishing moment beyond degree 9 is the 10th).
    h = (0.23, 0.19, 0.29)  # (dx, dy, dz): distinct so that an axis swap shows
    shape = (11, 9, 10)
    z, y, x = _grid(shape, h)
    q = [z, y, x][axis]
    hq = [h[2], h[1], h[0]][axis]
    p = np.broadcast_to(q ** 10, tuple(s + 8 for s in shape)).copy()
    exact = np.broadcast_to(90.0 * q ** 8, p.shape)[4:-4, 4:-4, 4:-4]
    got = oracle_lib.laplacian(p, h)
    err = got - exact
    pred = -1152.0 * hq ** 8
    scale = np.abs(p).max() / hq ** 2 * 1e-14
    assert np.abs(err - pred).max() <= max(scale, 1e-9 * abs(pred))


def _gaussian(z, y, x, sig):
    r2 = x * x + y * y + z * z
    return np.exp(-r2 / (2 * sig * sig))


def _gauss_lap(z, y, x, sig):
    r2 = x * x + y * y + z * z
    return (r2 / sig ** 4 - 3.0 / sig ** 2) * np.exp(-r2 / (2 * sig * sig))


def _gauss_d10(q, sig):
    # 10th derivative of exp(-q^2/(2 s^2)) along q: (-1/s)^10 He_10(q/s) g
    from numpy.polynomial import hermite_e as H

    t = q / sig
    return (1.0 / sig ** 10) * H.hermeval(t, [0] * 10 + [1]) * np.exp(-t * t / 2)


def test_eighth_order_convergence_and_error_constant(oracle_lib):
    # Ghost layer filled with the analytic Gaussian, so only truncation error
    # remains: observed order -> 8 and the error -> -(h^8/3150) sum_a d^10u/dq_a^10.
    sig = 1.0
    errs, hs = [], []
    for n in (32, 48, 64, 96):
        h = 8.0 * sig / n
        hh = (h, h, h)
        z, y, x = _grid((n, n, n), hh)
        u = _gaussian(z, y, x, sig)
        got = oracle_lib.laplacian(u, hh)
        ex = _gauss_lap(z, y, x, sig)[4:-4, 4:-4, 4:-4]
        errs.append(np.abs(got - ex).max())
        hs.append(h)
    zz, yy, xx = z[4:-4], y[:, 4:-4], x[:, :, 4:-4]
    pred = -(h ** 8 / 3150.0) * (_gauss_d10(zz, sig) * np.exp(-(yy ** 2 + xx ** 2) / 2)
                                 + _gauss_d10(yy, sig) * np.exp(-(zz ** 2 + xx ** 2) / 2)
                                 + _gauss_d10(xx, sig) * np.exp(-(zz ** 2 + yy ** 2) / 2))
    assert rel_l2(got - ex, pred) < 0.03
    orders = [np.log(errs[i] / errs[i + 1]) / np.log(hs[i] / hs[i + 1]) for i in range(3)]
    for o in orders:
        assert 7.5 < o < 8.5, orders


def test_kronecker_sum_brute_force(oracle_lib):
    # Independent construction: the Laplacian as a Kronecker sum of 1-D
    # banded operators built from the published weights, zero ghost layer.
    rng = np.random.default_rng(7)
    nz, ny, nx = 7, 9, 11
    h = (1.3, 0.9, 1.7)
    u = rng.standard_normal((nz, ny, nx))
    pad = np.zeros((nz + 8, ny + 8, nx + 8))
    pad[4:-4, 4:-4, 4:-4] = u
    got = oracle_lib.laplacian(pad, h)
    L = kron_laplacian(nz, ny, nx, h, golden_coefficients())
    ref = (L @ u.ravel()).reshape(u.shape)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
