"""Seeded synthetic inputs for the RSF level-set path.

This module is shared by the HIP path's tests/benchmark and by the CPU
oracle's tests; it holds none of the level-set arithmetic.  It draws
microvessel-like phantoms: straight or curved tubes (quadratic Bezier
centrelines, radius 1-4 voxels) rendered into a binary mask, mapped to
intensities 0.1 (background) / 0.8 (vessel), blurred by a Gaussian of sd 1
(scipy's filter, reflect boundary, truncated at 3 sd) and given additive
Gaussian noise.  The paper's microscopy volumes (KESM, light-sheet, micro-CT)
are not available; these phantoms stand in for them with vessel radii of the
size the paper targets (3-10 um vessels at ~1 um voxels).

phi0 follows the box rule: +2 inside the centred box whose sides are half the
volume's extents, -2 elsewhere.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def tube_mask(shape, n_tubes: int, r_min: float, r_max: float,
              rng: np.random.Generator) -> np.ndarray:
    """Binary mask [nz][ny][nx] of `n_tubes` random tubes."""
    nz, ny, nx = shape
    dims = np.array([nx, ny, nz], dtype=np.float64)
    mask = np.zeros(shape, dtype=bool)
    for _ in range(int(n_tubes)):
        p0 = rng.uniform(0.0, 1.0, 3) * dims
        p2 = rng.uniform(0.0, 1.0, 3) * dims
        mid = 0.5 * (p0 + p2)
        if rng.random() < 0.5:
            p1 = mid
        else:
            p1 = mid + rng.normal(0.0, max(np.linalg.norm(p2 - p0) / 4.0, 1e-6), 3)
        r = float(rng.uniform(r_min, r_max))
        # B'(t) is linear in t, so its largest norm is at an end point.
        speed = max(2.0 * np.linalg.norm(p1 - p0), 2.0 * np.linalg.norm(p2 - p1), 1e-6)
        m = int(math.ceil(speed / 0.5)) + 1
        rc = int(math.ceil(r))
        o = np.arange(-rc, rc + 2)
        off = np.stack(np.meshgrid(o, o, o, indexing="ij"), -1).reshape(-1, 3)
        # offsets that can lie within r of a centre in [0, 1)^3 around the base voxel
        off = off[(((off - 0.5) ** 2).sum(-1)) <= (r + 0.87) ** 2].astype(np.int32)
        for s0 in range(0, m, 2048):
            t = np.arange(s0, min(m, s0 + 2048), dtype=np.float64) / max(m - 1, 1)
            t = t[:, None]
            c = ((1 - t) ** 2 * p0 + 2 * (1 - t) * t * p1 + t ** 2 * p2).astype(np.float32)
            v = np.floor(c).astype(np.int32)[:, None, :] + off[None, :, :]   # (k, K, 3)
            d2 = ((v - c[:, None, :]) ** 2).sum(-1)
            v = v[d2 <= r * r]
            ok = ((v >= 0) & (v < np.array([nx, ny, nz], dtype=np.int32))).all(-1)
            v = v[ok]
            mask[v[:, 2], v[:, 1], v[:, 0]] = True
    return mask


def vessel_phantom(shape, n_tubes: int, r_min: float, r_max: float, seed: int,
                   lo: float = 0.1, hi: float = 0.8, blur_sd: float = 1.0,
                   noise_sd: float = 0.05) -> np.ndarray:
    """Float32 phantom [nz][ny][nx]: tubes at `hi`, background `lo`, blurred,
    plus N(0, noise_sd^2) noise (no clipping)."""
    from scipy.ndimage import gaussian_filter

    rng = rng_for(seed)
    m = tube_mask(shape, n_tubes, r_min, r_max, rng)
    clean = np.where(m, np.float32(hi), np.float32(lo)).astype(np.float32)
    del m
    img = gaussian_filter(clean, sigma=blur_sd, truncate=3.0, mode="reflect")
    del clean
    img += np.float32(noise_sd) * rng.standard_normal(size=shape, dtype=np.float32)
    return np.ascontiguousarray(img, dtype=np.float32)


def u16_phantom(shape, n_tubes: int, r_min: float, r_max: float, seed: int,
                background: float = 6000.0, vessel: float = 50000.0, gain: float = 8.0,
                read_sd: float = 100.0, blur_sd: float = 1.0) -> np.ndarray:
    """uint16 phantom [nz][ny][nx] in detector numbers: the tube mask blurred by
    a Gaussian of sd `blur_sd`, mapped to background..vessel, then
    Poisson-Gaussian noise u = gain * Poisson(clean / gain) + N(0, read_sd^2),
    clipped to [0, 65535] and rounded."""
    from scipy.ndimage import gaussian_filter

    rng = rng_for(seed)
    m = tube_mask(shape, n_tubes, r_min, r_max, rng).astype(np.float32)
    mb = gaussian_filter(m, sigma=blur_sd, truncate=3.0, mode="reflect")
    del m
    clean = np.float32(background) + np.float32(vessel - background) * mb
    del mb
    u = np.float32(gain) * rng.poisson(clean / np.float32(gain)).astype(np.float32)
    del clean
    u += np.float32(read_sd) * rng.standard_normal(size=shape, dtype=np.float32)
    np.clip(u, 0.0, 65535.0, out=u)
    return np.rint(u).astype(np.uint16)


def box_phi0(shape, inside: float = 2.0, outside: float = -2.0) -> np.ndarray:
    """+inside on [n/4, 3n/4) along every axis, `outside` elsewhere."""
    phi = np.full(shape, outside, dtype=np.float32)
    sl = tuple(slice(n // 4, n // 4 + n // 2) for n in shape)
    phi[sl] = inside
    return phi


@dataclass(frozen=True)
class Workload:
    """A plain-volume workload: phantom recipe, box phi0 and RSF parameters."""
    name: str
    shape: tuple            # (nz, ny, nx)
    n_tubes: int
    r_min: float
    r_max: float
    seed: int
    iters: int
    sigma: float = 3.0
    lambda1: float = 1.0
    lambda2: float = 1.0
    nu: float = 0.001
    mu: float = 1.0
    dt: float = 0.1
    eps: float = 1.0

    def image(self) -> np.ndarray:
        return vessel_phantom(self.shape, self.n_tubes, self.r_min, self.r_max, self.seed)

    def phi0(self) -> np.ndarray:
        return box_phi0(self.shape)

    @property
    def voxels(self) -> int:
        return int(np.prod(self.shape))

    def params(self) -> dict:
        return dict(sigma=self.sigma, lambda1=self.lambda1, lambda2=self.lambda2,
                    nu=self.nu, mu=self.mu, dt=self.dt, eps=self.eps)


# 64^3, 12 tubes r 1-3, 20 iterations (small parity case).
SMALL_64 = Workload("vessel64_s3_it20", (64, 64, 64), 12, 1.0, 3.0, seed=1, iters=20)
# 512^3, 400 tubes r 1-4, 200 iterations (throughput case).
LARGE_512 = Workload("vessel512_s3_it200", (512, 512, 512), 400, 1.0, 4.0, seed=2, iters=200)


def scaled(w: Workload, n: int, iters: int | None = None, name: str | None = None) -> Workload:
    """Same recipe on an n^3 volume, tube count scaled by volume."""
    frac = (n ** 3) / float(np.prod(w.shape))
    tubes = max(4, int(round(w.n_tubes * frac ** (1.0 / 3.0) * frac ** (1.0 / 3.0))))
    return Workload(name or f"{w.name}_n{n}", (n, n, n), tubes, w.r_min, w.r_max,
                    w.seed + 1000 + n, iters if iters is not None else w.iters,
                    w.sigma, w.lambda1, w.lambda2, w.nu, w.mu, w.dt, w.eps)


def tile_phi0(shape, halo: int, inside: float = 2.0, outside: float = -2.0) -> np.ndarray:
    """phi0 of one tile: +inside on the centred box whose sides are half the
    tile's interior (extent minus the halo on both sides), `outside` elsewhere."""
    phi = np.full(shape, outside, dtype=np.float32)
    sl = []
    for n in shape:
        e = n - 2 * halo
        lo = halo + e // 4
        sl.append(slice(lo, lo + max(e // 2, 1)))
    phi[tuple(sl)] = inside
    return phi


def cut_tiles(volume: np.ndarray, n_tiles: int, edges, halo: int, seed: int):
    """`n_tiles` sub-volumes of `volume`: interior edge lengths drawn from
    `edges` independently per axis, `halo` voxels added on every side, origins
    uniform so the tile fits.  Returns [(origin_zyx, image tile, phi0 tile)]."""
    rng = rng_for(seed)
    out = []
    for _ in range(int(n_tiles)):
        ext = [int(rng.choice(edges)) + 2 * halo for _ in range(3)]
        org = [int(rng.integers(0, n - e + 1)) for n, e in zip(volume.shape, ext)]
        sl = tuple(slice(o, o + e) for o, e in zip(org, ext))
        img = np.ascontiguousarray(volume[sl])
        out.append((tuple(org), img, tile_phi0(img.shape, halo)))
    return out


@dataclass(frozen=True)
class TileWorkload:
    """A batch of sub-volume tiles with halos cut from one phantom volume,
    each evolved as an independent problem from its own box phi0."""
    name: str
    shape: tuple            # phantom (nz, ny, nx)
    n_tubes: int
    r_min: float
    r_max: float
    seed: int
    n_tiles: int
    edges: tuple            # interior edge lengths, drawn per axis
    halo: int
    iters: int
    sigma: float = 3.0
    lambda1: float = 1.0
    lambda2: float = 1.0
    nu: float = 0.001
    mu: float = 1.0
    dt: float = 0.1
    eps: float = 1.0

    def volume(self) -> np.ndarray:
        return vessel_phantom(self.shape, self.n_tubes, self.r_min, self.r_max, self.seed)

    def tiles(self, volume: np.ndarray):
        return cut_tiles(volume, self.n_tiles, self.edges, self.halo, self.seed + 100)

    def params(self) -> dict:
        return dict(sigma=self.sigma, lambda1=self.lambda1, lambda2=self.lambda2,
                    nu=self.nu, mu=self.mu, dt=self.dt, eps=self.eps)


# 64 tiles, interior edges from {96..256} per axis plus a 9-voxel (3 sigma)
# halo, cut from a 1024x1024x512 phantom of 1500 tubes r 1-4; 100 iterations.
TILES_64 = TileWorkload("tiles64_s3_it100", (512, 1024, 1024), 1500, 1.0, 4.0, seed=3,
                        n_tiles=64, edges=(96, 128, 160, 192, 256), halo=9, iters=100)


@dataclass(frozen=True)
class ServeWorkload:
    """A stream of tile requests cut from one uint16 volume: interior edge
    lengths drawn per axis from `edges`, sigma from `sigmas`, iterations
    uniform in [it_lo, it_hi], a ceil(3 sigma) halo on every side, box phi0,
    Poisson arrivals (rate set by the caller)."""
    name: str
    shape: tuple            # volume (nz, ny, nx)
    n_tubes: int
    r_min: float
    r_max: float
    seed: int
    n_requests: int
    edges: tuple
    sigmas: tuple
    it_lo: int
    it_hi: int
    storage: str = "f16"
    lambda1: float = 1.0
    lambda2: float = 1.0
    nu: float = 0.001
    mu: float = 1.0
    dt: float = 0.1
    eps: float = 1.0

    def volume(self) -> np.ndarray:
        return u16_phantom(self.shape, self.n_tubes, self.r_min, self.r_max, self.seed)

    def requests(self, n: int | None = None):
        """[(origin_zyx, extent_zyx, sigma, halo, iters)] in arrival order."""
        rng = rng_for(self.seed + 200)
        out = []
        for _ in range(int(n if n is not None else self.n_requests)):
            sigma = float(rng.choice(self.sigmas))
            halo = int(math.ceil(3.0 * sigma - 1e-9))
            ext = [int(rng.choice(self.edges)) + 2 * halo for _ in range(3)]
            org = [int(rng.integers(0, d - e + 1)) for d, e in zip(self.shape, ext)]
            iters = int(rng.integers(self.it_lo, self.it_hi + 1))
            out.append((tuple(org), tuple(ext), sigma, halo, iters))
        return out

    def params(self, sigma: float) -> dict:
        return dict(sigma=sigma, lambda1=self.lambda1, lambda2=self.lambda2, nu=self.nu,
                    mu=self.mu, dt=self.dt, eps=self.eps)


# 2000 requests cut from the 1024x1024x512 uint16 volume (1500 tubes r 1-4,
# seed 4): interior edges {64, 96, ..., 384} per axis, sigma in {2, 3, 4},
# 50-150 iterations, FP16 storage.
SERVE_2000 = ServeWorkload("serve2000_u16_f16", (512, 1024, 1024), 1500, 1.0, 4.0, seed=4,
                           n_requests=2000, edges=tuple(range(64, 385, 32)),
                           sigmas=(2.0, 3.0, 4.0), it_lo=50, it_hi=150)
