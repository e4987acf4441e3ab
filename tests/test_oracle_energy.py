"""Pins of how the oracle assembles the energy E and the update (Sec. 2, Eq. 1;
Sec. 3, final energy equation):

    phi_{n+1} = phi_n + dt * E,   E = mu * R + delta(phi) * (nu * kappa - F_d)

Each pin switches all terms but one (or two) off through the coefficients and
rebuilds what is left from facts that do not come from the oracle: closed
forms of the curvature and Laplacian of spheres and cones, the double-well
rate taken from a numerical derivative of its potential, and the fitting
energies as brute-force double sums with a Gaussian built from scipy's taps.
The profiles are chosen so that delta(phi) varies by orders of magnitude over
the checked voxels, so a term put inside or outside the Dirac factor by
mistake changes the result by far more than the tolerance.
"""
import math

import numpy as np
import pytest
from scipy.ndimage import gaussian_filter, gaussian_filter1d

import oracle

DW = oracle.DOUBLE_WELL
SW = oracle.SINGLE_WELL


def P(sigma=1.0, lambda1=0.0, lambda2=0.0, nu=0.0, mu=0.0, dt=0.1, eps=1.0, eta=1e-10):
    return oracle.params_array(sigma, lambda1, lambda2, nu, mu, dt, eps, eta)


def dirac(phi, eps):
    """Derivative of the arctan Heaviside, written out here."""
    return eps / (math.pi * (eps * eps + phi * phi))


def grid(n):
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    return x.astype(float), y.astype(float), z.astype(float)


def rate_from_one_step(I, phi0, params, reg=DW):
    phi1, _ = oracle.evolve(I, phi0, params, 1, reg=reg)
    return (phi1 - phi0) / params[5]


def test_regulariser_alone_is_not_weighted_by_dirac():
    """lambda = nu = 0, mu = 1 on phi = 0.02 x^2: (phi1 - phi0)/dt equals the
    double-well R built from the potential's numerical derivative, although
    delta(phi) falls from 1/pi to 5e-5 along the profile."""
    nx = 64
    shape = (3, 3, nx)
    xs = np.arange(nx, dtype=float)
    phi0 = np.broadcast_to(0.02 * xs * xs, shape).copy()
    I = np.full(shape, 0.5)

    def pot(s):
        return np.where(s <= 1, (1 - np.cos(2 * np.pi * s)) / (2 * np.pi) ** 2, (s - 1) ** 2 / 2)

    def rate(s):
        h = 1e-6
        dp = (pot(s + h) - pot(s - h)) / (2 * h)
        return np.where(s > 0, dp / np.where(s > 0, s, 1), 1.0) - 1.0

    g = 0.04 * xs                      # the central difference of 0.02 x^2 is exact
    V = rate(np.abs(g)) * g
    want = np.zeros(nx)
    for i in range(1, nx - 1):
        want[i] = (phi0[1, 1, i + 1] + phi0[1, 1, i - 1] - 2 * phi0[1, 1, i]) + (V[i + 1] - V[i - 1]) / 2
    for mu in (1.0, 0.3):
        got = rate_from_one_step(I, phi0, P(mu=mu))[1, 1]
        ok = np.abs(g[2:-2] - 1.0) > 0.05   # skip the kink of the potential at s = 1
        assert np.max(np.abs(got[2:-2] - mu * want[2:-2])[ok]) < 1e-6
    d = dirac(phi0[1, 1, 2:-2], 1.0)
    assert d.max() / d.min() > 1e3


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_curvature_alone_is_weighted_by_dirac(sign):
    """mu = lambda = 0, nu = 1 on an offset sphere's signed distance:
    (phi1 - phi0) / (dt delta(phi0)) = kappa = 2/r (sign flips with phi),
    second order in 1/r (the curvature pin's bar)."""
    n = 40
    x, y, z = grid(n)
    r = np.sqrt((x - 20.3) ** 2 + (y - 19.7) ** 2 + (z - 20.2) ** 2)
    phi0 = sign * (r - 10.0)
    I = np.full(phi0.shape, 0.5)
    p = P(nu=1.0, eps=1.0)
    k = rate_from_one_step(I, phi0, p) / dirac(phi0, 1.0)
    rel = np.abs(k * r / (2.0 * sign) - 1.0)
    e6 = rel[(r >= 6) & (r < 7)].max()
    e12 = rel[(r >= 12) & (r < 13)].max()
    assert e6 < 0.05
    assert e12 < e6 / 2.5
    # nu scales the term linearly
    k2 = rate_from_one_step(I, phi0, P(nu=2.5, eps=1.0)) / dirac(phi0, 1.0)
    sel = (r >= 6) & (r < 16)
    assert np.max(np.abs(k2[sel] - 2.5 * k[sel])) < 1e-9


def test_cone_regulariser_outside_and_curvature_inside_dirac():
    """Constant image (no data force) and the cone phi = a (r0 - r), a = 2:
    the double-well flux is (1 - 1/a) grad phi, so R = -2 (a - 1)/r, and
    kappa = -2/r.  Then (phi1 - phi0)/dt = -2 mu (a - 1)/r - 2 nu delta(phi0)/r
    where delta(phi0) spans two orders of magnitude."""
    n = 40
    x, y, z = grid(n)
    r = np.sqrt((x - 19.6) ** 2 + (y - 20.3) ** 2 + (z - 19.8) ** 2)
    a, r0, eps = 2.0, 9.0, 0.5
    phi0 = a * (r0 - r)
    I = np.full(phi0.shape, 0.37)
    mu, nu = 1.0, 0.8
    got = rate_from_one_step(I, phi0, P(sigma=1.5, mu=mu, nu=nu, lambda1=1.0, lambda2=1.0,
                                        eps=eps))
    d = dirac(phi0, eps)
    t_reg = -2.0 * mu * (a - 1.0) / r
    t_curv = -2.0 * nu * d / r
    sel = (r >= 6) & (r < 12)
    err = np.abs(got - (t_reg + t_curv))[sel]
    assert np.all(err <= 0.05 * (np.abs(t_reg) + np.abs(t_curv))[sel])
    assert d[sel].max() / d[sel].min() > 100
    # each misplacement moves the rate by more than twice that bar everywhere
    scale = (np.abs(t_reg) + np.abs(t_curv))[sel]
    wrong_inside = d * t_reg + t_curv                          # delta (mu R + nu kappa)
    wrong_outside = t_reg + t_curv / d                         # nu kappa outside delta
    assert np.min(np.abs(got - wrong_inside)[sel] / scale) > 0.1
    assert np.min(np.abs(got - wrong_outside)[sel] / scale) > 0.1


def scipy_kernel3d(sigma):
    R = int(3.0 * sigma + 0.5)
    d = np.zeros(4 * R + 1)
    d[2 * R] = 1.0
    w = gaussian_filter1d(d, sigma, truncate=3.0, mode="constant")[R:3 * R + 1]
    return R, w[:, None, None] * w[None, :, None] * w[None, None, :]


def brute_same_conv(u, R, K):
    nz, ny, nx = u.shape
    up = np.pad(u, R)
    out = np.zeros_like(u)
    for c in range(2 * R + 1):
        for b in range(2 * R + 1):
            for a in range(2 * R + 1):
                out += K[c, b, a] * up[c:c + nz, b:b + ny, a:a + nx]
    return out


@pytest.mark.parametrize("l1,l2", [(1.3, 0.7), (0.0, 2.0)])
def test_data_force_alone_is_minus_dirac_times_fitting_energy(l1, l2):
    """mu = nu = 0: (phi1 - phi0)/(dt delta(phi0)) = -(l1 e1 - l2 e2), with
    H, f_i and e_i(x) = sum_y K(y - x) (I(x) - f_i(y))^2 all rebuilt here by
    brute force on a 9^3 volume (K from scipy's taps, zero padding)."""
    shape = (9, 9, 9)
    sigma, eps = 1.0, 0.8
    r = np.random.default_rng(41)
    I = r.uniform(0, 1, size=shape)
    phi0 = 20.0 * gaussian_filter(r.normal(size=shape), 1.5, mode="reflect")
    R, K = scipy_kernel3d(sigma)
    H = 0.5 * (1.0 + (2.0 / math.pi) * np.arctan(phi0 / eps))
    f1 = brute_same_conv(H * I, R, K) / brute_same_conv(H, R, K)
    f2 = brute_same_conv((1 - H) * I, R, K) / brute_same_conv(1 - H, R, K)
    e = []
    for fit in (f1, f2):
        ei = np.zeros(shape)
        for z in range(9):
            for y in range(9):
                for x in range(9):
                    acc = 0.0
                    for zz in range(max(0, z - R), min(9, z + R + 1)):
                        for yy in range(max(0, y - R), min(9, y + R + 1)):
                            for xx in range(max(0, x - R), min(9, x + R + 1)):
                                acc += K[zz - z + R, yy - y + R, xx - x + R] * \
                                    (I[z, y, x] - fit[zz, yy, xx]) ** 2
                    ei[z, y, x] = acc
        e.append(ei)
    want = -(l1 * e[0] - l2 * e[1])
    d = dirac(phi0, eps)
    got = rate_from_one_step(I, phi0, P(sigma=sigma, lambda1=l1, lambda2=l2, eps=eps))
    assert np.max(np.abs(got / d - want)) < 1e-10
    assert d.max() / d.min() > 10
