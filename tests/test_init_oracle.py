"""Pins of the oracle's initialisation (Sec. 4.3): determinant-of-Hessian
seeds in each z slice and fast sweeping (Zhao 2005) of the distance to them.

Each pin is fixed by something other than the oracle's own code: a
library convolution, exact derivatives of quadratics, the geometry of a
Gaussian blob, and a fast-marching solution of the same upwind equations
(written here as a plain Dijkstra-type loop) that the converged sweep must
reproduce."""
import heapq
import math

import numpy as np
import pytest

import oracle

scipy_ndimage = pytest.importorskip("scipy.ndimage")


def gauss_weights(sigma):
    R = math.ceil(3 * sigma - 1e-9)
    k = np.arange(-R, R + 1, dtype=np.float64)
    w = np.exp(-k * k / (2 * sigma * sigma))
    return w / w.sum()


def fast_marching(shape, seeds):
    """Dijkstra-type solution of the first-order upwind (Godunov) equations
    of |grad u| = 1 on the unit grid: a trial point takes the largest set of
    accepted axis minima v with x = root of sum (x - v)^2 = 1 above them."""
    u = np.full(shape, math.inf)
    done = np.zeros(shape, bool)
    heap = []
    for s in seeds:
        u[s] = 0.0
        heapq.heappush(heap, (0.0, s))

    def solve(p):
        vals = []
        for ax in range(3):
            best = math.inf
            for step in (-1, 1):
                q = list(p)
                q[ax] += step
                if 0 <= q[ax] < shape[ax] and done[tuple(q)]:
                    best = min(best, u[tuple(q)])
            if best < math.inf:
                vals.append(best)
        vals.sort()
        for m in range(len(vals), 0, -1):
            a = vals[:m]
            s1, s2 = sum(a), sum(v * v for v in a)
            disc = s1 * s1 - m * (s2 - 1)
            if disc >= 0:
                x = (s1 + math.sqrt(disc)) / m
                if x > a[-1]:
                    return x
        return math.inf

    while heap:
        d, p = heapq.heappop(heap)
        if done[p] or d > u[p]:
            continue
        done[p] = True
        for ax in range(3):
            for step in (-1, 1):
                q = list(p)
                q[ax] += step
                if 0 <= q[ax] < shape[ax] and not done[tuple(q)]:
                    q = tuple(q)
                    x = solve(q)
                    if x < u[q]:
                        u[q] = x
                        heapq.heappush(heap, (x, q))
    return u


def seeded(shape, seeds):
    u = np.full(shape, oracle.FAR)
    for s in seeds:
        u[s] = 0.0
    return u


# --- fast sweeping ---------------------------------------------------------

@pytest.mark.parametrize("shape,n_seeds,seed", [((7, 8, 9), 1, 1), ((7, 8, 9), 3, 2),
                                                ((5, 11, 6), 5, 3), ((9, 4, 10), 2, 4)])
def test_fast_sweep_converges_to_fast_marching(shape, n_seeds, seed):
    rng = np.random.default_rng(seed)
    seeds = {tuple(int(rng.integers(0, e)) for e in shape) for _ in range(n_seeds)}
    got = oracle.fast_sweep(seeded(shape, seeds), rounds=2)
    want = fast_marching(shape, seeds)
    assert np.max(np.abs(got - want)) < 1e-12
    # one more round changes nothing: the discrete solution is reached
    assert np.array_equal(oracle.fast_sweep(got, rounds=1), got)


def test_fast_sweep_single_seed_bounds():
    shape = (9, 10, 11)
    s = (4, 3, 6)
    one = oracle.fast_sweep(seeded(shape, [s]), rounds=1)
    assert np.array_equal(one, oracle.fast_sweep(seeded(shape, [s]), rounds=2))
    z, y, x = np.indices(shape)
    dz, dy, dx = np.abs(z - s[0]), np.abs(y - s[1]), np.abs(x - s[2])
    euclid = np.sqrt(dz ** 2 + dy ** 2 + dx ** 2)
    manhattan = dz + dy + dx
    on_axis = (dz == 0).astype(int) + (dy == 0) + (dx == 0) >= 2
    assert np.array_equal(one[on_axis], euclid[on_axis])      # exact along the axes
    assert np.all(one >= euclid - 1e-12)                       # upwind overestimates
    assert np.all(one <= manhattan + 1e-12)
    assert one[s[0], s[1] + 1, s[2] + 1] == pytest.approx(1 + math.sqrt(0.5), abs=1e-15)


def test_fast_sweep_seed_plane_gives_exact_distance():
    shape = (6, 7, 12)
    u = np.full(shape, oracle.FAR)
    u[:, :, 3] = 0.0
    d = oracle.fast_sweep(u, rounds=1)
    want = np.broadcast_to(np.abs(np.arange(12) - 3).astype(np.float64), shape)
    assert np.array_equal(d, want)


# --- determinant-of-Hessian seeds -----------------------------------------

@pytest.mark.parametrize("sigma", [1.0, 1.7, 2.5])
def test_slice_smoothing_matches_library_correlation(sigma):
    rng = np.random.default_rng(11)
    I = rng.random((3, 17, 23))
    w = gauss_weights(sigma)
    want = scipy_ndimage.correlate1d(I, w, axis=2, mode="constant", cval=0.0)
    want = scipy_ndimage.correlate1d(want, w, axis=1, mode="constant", cval=0.0)
    assert np.max(np.abs(oracle.smooth_slices(I, sigma) - want)) < 1e-14


def test_slice_hessian_exact_on_quadratics():
    a, b, c, d, e = 0.7, -1.3, 0.45, 2.0, -0.5
    y, x = np.indices((9, 12), dtype=np.float64)
    L = np.stack([a * x * x + b * y * y + c * x * y + d * x + e * y + k for k in range(3)])
    Lxx, Lyy, Lxy = oracle.slice_hessian(L)
    inner = (slice(None), slice(1, -1), slice(1, -1))
    assert np.allclose(Lxx[inner], 2 * a, atol=1e-11)
    assert np.allclose(Lyy[inner], 2 * b, atol=1e-11)
    assert np.allclose(Lxy[inner], c, atol=1e-11)


def test_slice_hessian_boundary_reflects_about_the_edge_voxel():
    rng = np.random.default_rng(12)
    L = rng.random((2, 5, 6))
    Lxx, Lyy, Lxy = oracle.slice_hessian(L)
    nz, ny, nx = L.shape

    def at(z, yy, xx):   # ghost -1 -> 1, n -> n - 2
        yy = -yy if yy < 0 else (2 * (ny - 1) - yy if yy > ny - 1 else yy)
        xx = -xx if xx < 0 else (2 * (nx - 1) - xx if xx > nx - 1 else xx)
        return L[z, yy, xx]

    for z in range(nz):
        for yy in range(ny):
            for xx in range(nx):
                c = at(z, yy, xx)
                assert Lxx[z, yy, xx] == pytest.approx(at(z, yy, xx + 1) - 2 * c + at(z, yy, xx - 1))
                assert Lyy[z, yy, xx] == pytest.approx(at(z, yy + 1, xx) - 2 * c + at(z, yy - 1, xx))
                assert Lxy[z, yy, xx] == pytest.approx(
                    (at(z, yy + 1, xx + 1) - at(z, yy - 1, xx + 1) - at(z, yy + 1, xx - 1) +
                     at(z, yy - 1, xx - 1)) / 4)


def tube(shape, centre, radius, amp):
    nz, ny, nx = shape
    y, x = np.indices((ny, nx), dtype=np.float64)
    blob = amp * np.exp(-((x - centre[1]) ** 2 + (y - centre[0]) ** 2) / (2 * radius ** 2))
    return np.broadcast_to(blob, shape).copy()


def test_bright_tube_gives_one_seed_per_slice_at_its_centre():
    shape = (4, 31, 37)
    I = 0.1 + tube(shape, (14, 20), 2.0, 1.0)
    m, doh, tr = oracle.blob_seeds(I, 1.5, 0.05)
    want = np.zeros(shape, bool)
    want[:, 14, 20] = True
    assert np.array_equal(m, want)
    assert np.all(tr[:, 14, 20] < 0) and doh.max() > 0


def test_dark_blob_and_saddle_give_no_seed():
    shape = (2, 27, 27)
    dark = 1.0 - tube(shape, (13, 13), 2.0, 0.8)
    m, _, tr = oracle.blob_seeds(dark, 1.5, 0.0)
    assert not m[:, 5:22, 5:22].any()         # the dark centre has trace > 0
    assert tr[0, 13, 13] > 0
    y, x = np.indices((27, 27), dtype=np.float64)
    saddle = np.broadcast_to(((x - 13) ** 2 - (y - 13) ** 2) * 1e-3, shape).copy()
    _, doh, _ = oracle.blob_seeds(saddle, 1.0, 0.0)
    assert np.all(doh[:, 4:23, 4:23] < 0)


def test_threshold_is_relative_to_the_volume_maximum():
    shape = (2, 30, 60)
    I = tube(shape, (15, 15), 2.0, 1.0) + tube(shape, (15, 45), 2.0, 0.3)
    _, doh, _ = oracle.blob_seeds(I, 1.5, 0.0)
    ratio = doh[0, 15, 45] / doh[0, 15, 15]
    lo, _, _ = oracle.blob_seeds(I, 1.5, 0.5 * ratio)
    hi, _, _ = oracle.blob_seeds(I, 1.5, 2.0 * ratio)
    assert lo[:, 15, 15].all() and lo[:, 15, 45].all() and lo.sum() == 4
    assert hi[:, 15, 15].all() and hi.sum() == 2


def test_plateau_gives_the_first_voxel_in_raster_order():
    doh = np.zeros((1, 6, 7))
    doh[0, 2:4, 3:5] = 5.0            # a 2 x 2 plateau
    doh[0, 0, 0] = 1.0
    tr = -np.ones_like(doh)
    m = oracle.seed_rule(doh, tr, 0.1)
    want = np.zeros_like(m)
    want[0, 2, 3] = True
    want[0, 0, 0] = True              # above 0.1 x 5 and a strict maximum
    assert np.array_equal(m, want)
    assert not oracle.seed_rule(doh, tr, 0.3)[0, 0, 0]


def test_init_phi_places_seeds_on_the_offset_level():
    shape = (3, 25, 29)
    I = 0.1 + tube(shape, (12, 9), 1.5, 1.0) + tube(shape, (12, 20), 1.5, 0.9)
    phi, m = oracle.init_phi(I, 1.5, 0.1, offset=2.0, rounds=2)
    assert m.sum() == 6
    assert np.all(phi[m] == 2.0) and np.all(phi[~m] < 2.0)
    assert phi[1, 12, 14] == pytest.approx(2.0 - 5.0)     # 5 voxels along x from a seed
    with pytest.raises(ValueError):
        oracle.init_phi(np.zeros(shape), 1.5, 0.1)
