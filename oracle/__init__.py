"""Plain FP64 CPU oracle of the 3D RSF level-set iteration (arXiv 2404.02813).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this package; the HIP product path
never does, and this package imports nothing from it.

The arithmetic lives in ``rsf_oracle.c`` (plain C, OpenMP over z); this module
only marshals NumPy arrays through ctypes.  ``real="f32"`` loads the same C
source compiled with a float working type; it exists to measure how far
rounding alone moves a trajectory, never as a reference.

Functions (each follows the passage named in ``rsf_oracle.c``):
    radius(sigma)                     truncation radius ceil(3 sigma)
    weights(sigma)                    sampled, unit-sum Gaussian taps (Sec. 3)
    conv3d(u, sigma)                  zero-padded separable Gaussian (Sec. 3)
    step(I, phi, params, reg)         one iteration + its fields (Eq. 1, Sec. 3)
    evolve(I, phi, params, iters)     ``iters`` iterations + sum|dphi| history
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rsf_oracle.c")
_LIBS = {"f64": os.path.join(_HERE, "liboracle_f64.so"),
         "f32": os.path.join(_HERE, "liboracle_f32.so")}
_loaded: dict = {}

# Regulariser readings of Sec. 2.1 (see rsf_oracle.c).
SINGLE_WELL = 0
DOUBLE_WELL = 1

PROBE_FIELDS = ("H", "f1", "f2", "e1", "e2", "kappa", "lap", "R", "E", "delta")


def build(force: bool = True) -> None:
    """Compile both oracle variants with gcc (plain -O2, OpenMP)."""
    for real, out in _LIBS.items():
        if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(_SRC):
            continue
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
               "-o", out + ".tmp", _SRC, "-lm"]
        if real == "f32":
            cmd.insert(1, "-DREAL=float")
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)


def _lib(real: str = "f64"):
    if real in _loaded:
        return _loaded[real]
    path = _LIBS[real]
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        build(force=False)
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_longlong
    lib.oracle_radius.argtypes = [ctypes.c_double]
    lib.oracle_radius.restype = ctypes.c_int
    lib.oracle_weights.argtypes = [ctypes.c_double, dp]
    lib.oracle_weights.restype = None
    lib.oracle_conv3d.argtypes = [dp, dp, i64, i64, i64, ctypes.c_double]
    lib.oracle_conv3d.restype = ctypes.c_int
    lib.oracle_step.argtypes = [dp, dp, dp, i64, i64, i64, dp, ctypes.c_int,
                                ctypes.POINTER(dp), dp]
    lib.oracle_step.restype = ctypes.c_int
    lib.oracle_evolve.argtypes = [dp, dp, i64, i64, i64, dp, ctypes.c_int, ctypes.c_int, dp]
    lib.oracle_evolve.restype = ctypes.c_int
    lib.oracle_fast_sweep.argtypes = [dp, i64, i64, i64, ctypes.c_int]
    lib.oracle_fast_sweep.restype = None
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_get_threads.restype = ctypes.c_int
    lib.oracle_real_type.restype = ctypes.c_char_p
    _loaded[real] = lib
    return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(n: int) -> None:
    for real in _LIBS:
        _lib(real).oracle_set_threads(int(n))


def threads() -> int:
    return int(_lib().oracle_get_threads())


def radius(sigma: float) -> int:
    return int(_lib().oracle_radius(float(sigma)))


def weights(sigma: float) -> np.ndarray:
    w = np.zeros(2 * radius(sigma) + 1, dtype=np.float64)
    _lib().oracle_weights(float(sigma), _dptr(w))
    return w


def conv3d(u, sigma: float, real: str = "f64") -> np.ndarray:
    u = _f64(u)
    nz, ny, nx = u.shape
    out = np.empty_like(u)
    rc = _lib(real).oracle_conv3d(_dptr(u), _dptr(out), nx, ny, nz, float(sigma))
    if rc != 0:
        raise ValueError(f"oracle_conv3d failed ({rc})")
    return out


FORCE_RSF = 0     # RSF fitting energies e_i with the same sigma
FORCE_PAPER = 1   # the Sec. 4.2 expansion with its own sigma2 (0 = identity)


def params_array(sigma, lambda1, lambda2, nu, mu, dt, eps, eta=1e-10, force=FORCE_RSF,
                 sigma2=0.0) -> np.ndarray:
    return np.array([sigma, lambda1, lambda2, nu, mu, dt, eps, eta, force, sigma2],
                    dtype=np.float64)


def step(I, phi, params, reg: int = DOUBLE_WELL, real: str = "f64"):
    """One iteration.  Returns (phi_next, fields dict, sum|dphi|)."""
    I = _f64(I)
    phi = _f64(phi)
    if I.shape != phi.shape or I.ndim != 3:
        raise ValueError("I and phi must be equal 3D shapes [nz][ny][nx]")
    nz, ny, nx = phi.shape
    out = np.empty_like(phi)
    fields = {k: np.empty_like(phi) for k in PROBE_FIELDS}
    probe = (ctypes.POINTER(ctypes.c_double) * len(PROBE_FIELDS))(
        *[_dptr(fields[k]) for k in PROBE_FIELDS])
    total = ctypes.c_double(0.0)
    p = _f64(params)
    rc = _lib(real).oracle_step(_dptr(I), _dptr(phi), _dptr(out), nx, ny, nz, _dptr(p),
                                int(reg), probe, ctypes.byref(total))
    if rc != 0:
        raise ValueError(f"oracle_step failed ({rc})")
    return out, fields, float(total.value)


def evolve(I, phi0, params, iters: int, reg: int = DOUBLE_WELL, real: str = "f64"):
    """``iters`` iterations of Eq. (1).  Returns (phi_iters, s_hist)."""
    I = _f64(I)
    phi = _f64(phi0).copy()
    if I.shape != phi.shape or I.ndim != 3:
        raise ValueError("I and phi must be equal 3D shapes [nz][ny][nx]")
    nz, ny, nx = phi.shape
    hist = np.zeros(max(int(iters), 1), dtype=np.float64)
    p = _f64(params)
    rc = _lib(real).oracle_evolve(_dptr(I), _dptr(phi), nx, ny, nz, _dptr(p), int(reg),
                                  int(iters), _dptr(hist))
    if rc != 0:
        raise ValueError(f"oracle_evolve failed ({rc})")
    return phi, hist[: int(iters)]


# ---------------------------------------------------------------------------
# Volume-level parallelism (Sec. 4.1): sub-volumes with curtains, evolved
# independently, merged by linear interpolation across the curtains.
# ---------------------------------------------------------------------------

def volume_cores(n: int, block: int):
    """Core boundaries along one axis: ceil(n / block) near-equal parts."""
    nb = -(-n // block)
    return [k * n // nb for k in range(nb + 1)]


def axis_weights(n: int, cuts, k: int, curtain: int) -> np.ndarray:
    """Weight of part k at each coordinate 0..n-1: one inside its core, zero
    outside its core +- curtain, and across each 2*curtain-wide overlap with
    a neighbour a linear ramp whose complement is the neighbour's weight."""
    c = np.arange(n, dtype=np.float64)
    lo, hi = cuts[k], cuts[k + 1]
    w = ((c >= lo) & (c < hi)).astype(np.float64)
    C = float(curtain)
    if k > 0:                       # overlap [lo - C, lo + C) with part k - 1
        m = (c >= lo - C) & (c < lo + C)
        w[m] = (c[m] - (lo - C) + 0.5) / (2.0 * C)
    if k + 2 < len(cuts):           # overlap [hi - C, hi + C) with part k + 1
        m = (c >= hi - C) & (c < hi + C)
        w[m] = ((hi + C) - c[m] - 0.5) / (2.0 * C)
    return w


def volume_boxes(shape, block: int, curtain: int):
    """[(slices, weight array)] of every sub-volume of a [nz][ny][nx] volume."""
    per_axis = []
    for n in shape:
        cuts = volume_cores(n, block)
        parts = []
        for k in range(len(cuts) - 1):
            lo = max(0, cuts[k] - curtain)
            hi = min(n, cuts[k + 1] + curtain)
            parts.append((slice(lo, hi), axis_weights(n, cuts, k, curtain)[lo:hi]))
        per_axis.append(parts)
    boxes = []
    for pz in per_axis[0]:
        for py in per_axis[1]:
            for px in per_axis[2]:
                w = pz[1][:, None, None] * py[1][None, :, None] * px[1][None, None, :]
                boxes.append(((pz[0], py[0], px[0]), w))
    return boxes


def merge_boxes(shape, boxes, fields) -> np.ndarray:
    """Sum of weight x field over the sub-volumes (the linear-interpolation
    merge of Sec. 4.1), in FP64."""
    out = np.zeros(shape, dtype=np.float64)
    for (sl, w), f in zip(boxes, fields):
        out[sl] += w * f
    return out


def evolve_volume(I, phi0, params, iters: int, block: int, curtain: int,
                  reg: int = DOUBLE_WELL):
    """Evolve every curtained sub-volume on its own with `evolve`, then merge."""
    I = _f64(I)
    phi0 = _f64(phi0)
    boxes = volume_boxes(phi0.shape, block, curtain)
    fields = [evolve(I[sl], phi0[sl], params, iters, reg)[0] for sl, _ in boxes]
    return merge_boxes(phi0.shape, boxes, fields)


# ---------------------------------------------------------------------------
# Initialisation (Sec. 4.3): determinant-of-Hessian seeds per z slice, then a
# distance function from the seeds by fast sweeping.
# ---------------------------------------------------------------------------

FAR = 1e30   # "no seed yet" distance


def smooth_slices(I, sigma: float, dtype=np.float64) -> np.ndarray:
    """Each z slice convolved with the sampled, truncated, unit-sum 2D
    Gaussian (separable: x then y), zero padding, in `dtype`."""
    w = weights(sigma).astype(dtype)
    R = (len(w) - 1) // 2
    u = np.asarray(I, dtype=dtype)
    nz, ny, nx = u.shape
    tmp = np.zeros_like(u)
    for k in range(-R, R + 1):             # along x: out[x] += w[k + R] * u[x + k]
        lo, hi = max(0, -k), min(nx, nx - k)
        tmp[:, :, lo:hi] += w[k + R] * u[:, :, lo + k:hi + k]
    out = np.zeros_like(u)
    for k in range(-R, R + 1):             # along y
        lo, hi = max(0, -k), min(ny, ny - k)
        out[:, lo:hi, :] += w[k + R] * tmp[:, lo + k:hi + k, :]
    return out


def slice_hessian(L):
    """In-slice second differences of L (central, reflect ghosts about the
    boundary voxel): Lxx, Lyy, Lxy."""
    p = np.pad(L, ((0, 0), (1, 1), (1, 1)), mode="reflect")
    c = p[:, 1:-1, 1:-1]
    Lxx = p[:, 1:-1, 2:] - 2 * c + p[:, 1:-1, :-2]
    Lyy = p[:, 2:, 1:-1] - 2 * c + p[:, :-2, 1:-1]
    Lxy = (p[:, 2:, 2:] - p[:, :-2, 2:] - p[:, 2:, :-2] + p[:, :-2, :-2]) / 4
    return Lxx, Lyy, Lxy


def blob_seeds(I, sigma_b: float, threshold: float, dtype=np.float64):
    """Seed mask: bright blobs (Lxx + Lyy < 0) whose determinant of the
    Hessian exceeds threshold x its largest value over the volume and is a
    local maximum in its 3x3 in-slice neighbourhood (strictly above the
    neighbours earlier in raster order, at least the later ones).  Returns
    (mask, doh, trace)."""
    L = smooth_slices(I, sigma_b, dtype)
    Lxx, Lyy, Lxy = slice_hessian(L)
    doh = (Lxx * Lyy - Lxy * Lxy).astype(dtype)
    tr = (Lxx + Lyy).astype(dtype)
    return seed_rule(doh, tr, threshold), doh, tr


def seed_rule(doh, tr, threshold: float) -> np.ndarray:
    """The selection of blob_seeds on given determinant and trace fields."""
    thr = doh.dtype.type(threshold) * doh.max()
    m = (doh > thr) & (tr < 0)
    nz, ny, nx = doh.shape
    p = np.pad(doh, ((0, 0), (1, 1), (1, 1)), mode="constant", constant_values=-np.inf)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dy == 0 and dx == 0:
                continue
            nb = p[:, 1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx]
            earlier = dy < 0 or (dy == 0 and dx < 0)
            m &= (doh > nb) if earlier else (doh >= nb)
    return m


def fast_sweep(u0, rounds: int = 1) -> np.ndarray:
    """Fast sweeping (Zhao 2005) on the unit grid, in FP64, from a field
    holding 0 at the seeds and FAR elsewhere."""
    u = _f64(u0).copy()
    nz, ny, nx = u.shape
    _lib().oracle_fast_sweep(_dptr(u), nx, ny, nz, int(rounds))
    return u


def init_phi(I, sigma_b: float, threshold: float, offset: float = 0.0, rounds: int = 1,
             dtype=np.float64):
    """phi0 = offset - distance to the nearest seed (seeds on the zero level
    for offset 0).  Returns (phi0, seed mask)."""
    m, _, _ = blob_seeds(I, sigma_b, threshold, dtype)
    if not m.any():
        raise ValueError("no seed found")
    u = np.where(m, 0.0, FAR)
    d = fast_sweep(u, rounds)
    return offset - d, m
