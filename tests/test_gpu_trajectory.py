"""Whole trajectories on the kernels the throughput runs use, against the FP64
oracle element by element (Sec. 2, Eq. 1 iterated; Sec. 3 final energy).

- A 32 x 512 x 512 slab of the 512^3 sigma = 3 vessel phantom, its own box
  phi0, 200 iterations: the 512^2 plane gives 512 update workgroups of
  64 x 8 columns, so every one marches the whole z extent and the update
  carries the next stage-1 z pass (the fused kernel the 512^3 throughput run
  times).  FP32, FP16 and BF16 storage against one oracle run.
- The mixed-precision recipe (uint16 detector numbers, sigma = 4, R = 12,
  150 iterations) on a 128 x 256 x 256 volume, the largest the oracle runs in
  about a minute, on the schedule the 1024 x 1024 x 512 volume runs: with
  FP16 storage the fused update (its update workgroups set to whole z
  columns, as the large plane gives them), with BF16 and FP32 storage the
  separate passes (radius 12 does not fuse there).

Each case prints max|dphi| inside and outside the band |phi_oracle| < 1, the
Dice of phi > 0 and the sign agreement.
"""
import sys
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_2404_02813_amd import inputs  # noqa: E402

PHI_TOL = 1e-3
SIGN_AGREE = 0.9999


def phi_tol(storage):
    """1e-3 for FP32 arithmetic with FP32 or FP16 storage; BF16 keeps 8
    significand bits and its bar scales by 2^-8 / 2^-11 = 8."""
    return PHI_TOL * (8.0 if storage == "bf16" else 1.0)


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rsf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2404_02813_amd import rsf as mod
    ctx = mod.Context(0)
    yield mod, ctx
    torch.cuda.synchronize()
    ctx.close()


def oracle_chunked(I, phi0, p, iters, chunk):
    """oracle.evolve in chunks (resuming is exact), reporting progress."""
    phi = phi0.astype(np.float64)
    hist = []
    t0 = time.time()
    done = 0
    while done < iters:
        k = min(chunk, iters - done)
        phi, h = oracle.evolve(I, phi, p, k)
        hist.extend(h.tolist())
        done += k
        say(f"  oracle {done}/{iters} iterations, {time.time() - t0:.0f} s")
    return phi, np.array(hist)


def report(got, want):
    d = np.abs(got - want)
    band = np.abs(want) < 1.0
    gp, wp = got > 0, want > 0
    dice = 2.0 * np.sum(gp & wp) / max(1, np.sum(gp) + np.sum(wp))
    agree = float(np.mean(gp == wp))
    r = dict(max=float(d.max()), band=float(d[band].max()) if band.any() else 0.0,
             outside=float(d[~band].max()) if (~band).any() else 0.0, dice=float(dice),
             agree=agree)
    say(f"  max|dphi| {r['max']:.3e} (band {r['band']:.3e}, outside {r['outside']:.3e}), "
        f"Dice {r['dice']:.7f}, sign agreement {r['agree']:.7f}")
    return r


SLAB = (32, 512, 512)


@pytest.fixture(scope="module")
def slab():
    w = inputs.LARGE_512
    say(f"generating {w.name}, slab {SLAB}")
    full = w.image()
    z0 = (w.shape[0] - SLAB[0]) // 2
    I = np.ascontiguousarray(full[z0:z0 + SLAB[0]])
    del full
    phi0 = inputs.box_phi0(SLAB)
    say("oracle on the slab")
    want, whist = oracle_chunked(I, phi0, oracle.params_array(**w.params(), eta=1e-10),
                                 w.iters, 50)
    return w, I, phi0, want, whist


@pytest.mark.timeout(900)
@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_fused_update_trajectory_matches_oracle(rsf, slab, storage):
    mod, ctx = rsf
    w, I, phi0, want, whist = slab
    say(f"slab {SLAB} x {w.iters} iterations, fused update, {storage} storage")
    vol = torch.from_numpy(I).cuda()
    phi = torch.from_numpy(phi0).cuda()
    ctx.set_fusion(True)
    ctx.profile(True)
    ctx.evolve_ex(vol, phi, mod.make_params(**w.params(), storage=storage), w.iters)
    ctx.profile(False)
    prof = ctx.profile_read()
    _, run, _, hist = ctx.stats(cap=w.iters)
    got = phi.cpu().numpy().astype(np.float64)
    # the fused update ran: one stage-1 z pass for the whole evolution
    assert prof["z_heaviside"][0] == 1
    assert prof["z_update"][0] == w.iters and run == w.iters
    r = report(got, want)
    assert r["max"] <= phi_tol(storage) and r["agree"] >= SIGN_AGREE
    # The history s_n = sum |phi_{n+1} - phi_n| is the GPU's own: the last
    # entry equals the FP64 sum over its own last two iterates (resumed at
    # 199, bitwise the same trajectory), up to the grouping of the sum.
    params = mod.make_params(**w.params(), storage=storage)
    p199 = torch.from_numpy(phi0).cuda()
    ctx.evolve_ex(vol, p199, params, w.iters - 1)
    p200 = p199.clone()
    ctx.evolve_ex(vol, p200, params, 1)
    _, _, last, _ = ctx.stats(cap=0)
    torch.cuda.synchronize()
    assert torch.equal(p200, phi)
    own = float(np.sum(np.abs(p200.cpu().numpy().astype(np.float64) -
                              p199.cpu().numpy().astype(np.float64))))
    assert last == pytest.approx(own, rel=1e-9)
    assert hist[-1] == pytest.approx(own, rel=1e-9)
    # Against the FP64 oracle's history the sums differ by the FP32 arithmetic
    # of phi itself: s_n adds up millions of far-field increments of a few
    # FP32 ulps of |phi| ~ 2, so their rounding shifts the sum by percents
    # while max|dphi| stays ~1e-5.  The oracle's own float build on this slab
    # differs from its FP64 run by up to 3.8 % in s_n (2.6e-5 in phi).
    rel = np.abs(np.array(hist) / whist - 1.0)
    say(f"  max relative s_n difference {rel.max():.4f} (iteration {int(rel.argmax())})")
    assert rel.max() < (0.1 if storage == "bf16" else 0.05)


MIXED = (128, 256, 256)


@pytest.fixture(scope="module")
def mixed():
    # the 1024 x 1024 x 512 recipe at this size: tube count scaled with the
    # cross-section (1500 / 16), seed of the full volume
    n_tubes = 94
    u = inputs.u16_phantom(MIXED, n_tubes, 1.0, 4.0, seed=4)
    I = u.astype(np.float64) / 65535.0
    phi0 = inputs.box_phi0(MIXED)
    p = dict(sigma=4.0, lambda1=1.0, lambda2=1.0, nu=0.001, mu=1.0, dt=0.1, eps=1.0)
    say(f"oracle on the uint16 recipe {MIXED}, sigma 4, 150 iterations")
    want, _ = oracle_chunked(I, phi0, oracle.params_array(**p, eta=1e-10), 150, 30)
    return u, phi0, p, want


@pytest.mark.timeout(900)
@pytest.mark.parametrize("storage", ["f16", "bf16", "f32"])
def test_mixed_precision_recipe_150_iterations(rsf, mixed, storage):
    mod, ctx = rsf
    u, phi0, p, want = mixed
    say(f"uint16 recipe {MIXED}, sigma 4 x 150, {storage} storage")
    vol = torch.from_numpy(u).cuda()
    phi = torch.from_numpy(phi0).cuda()
    fused = storage == "f16"
    if fused:
        ctx.set_split_targets(0, 0, 1)
    ctx.profile(True)
    ctx.evolve_ex(vol, phi, mod.make_params(**p, storage=storage), 150)
    ctx.profile(False)
    stage1 = ctx.profile_read()["z_heaviside"][0]
    ctx.set_split_targets(0, 0, 0)
    got = phi.cpu().numpy().astype(np.float64)
    assert stage1 == (1 if fused else 150)
    r = report(got, want)
    assert r["max"] <= phi_tol(storage) and r["agree"] >= SIGN_AGREE


def test_shrinking_ball_follows_the_radial_curvature_flow(rsf):
    """Curvature flow of a ball through the C ABI against the continuum
    equations directly (no oracle): constant image (F_d = 0), mu = 0, phi0 =
    r - rho.  kappa = -2/rho for any radially decreasing profile, so each
    voxel follows f' = -nu delta(f) 2/rho, stepped with the same Euler step;
    the GPU's gap to it is the grid's O(h^2) curvature error (0.0042 in the
    oracle at this size, under 2 % of the front's 0.26-voxel displacement),
    plus FP32 rounding."""
    mod, ctx = rsf
    say("shrinking ball: 32^3, eps 2, 64 iterations, against the per-voxel ODE")
    n, r, eps, dt, iters = 32, 8.0, 2.0, 0.1, 64
    c = (n - 1) / 2.0
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    rho = np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2)
    phi0 = (r - rho).astype(np.float32)
    vol = torch.full((n, n, n), 0.5, dtype=torch.float32, device="cuda")
    phi = torch.from_numpy(phi0).cuda()
    ctx.evolve_ex(vol, phi, mod.make_params(sigma=1.0, lambda1=1.0, lambda2=1.0, nu=1.0,
                                            mu=0.0, dt=dt, eps=eps), iters)
    got = phi.cpu().numpy().astype(np.float64)
    f = phi0.astype(np.float64)
    for _ in range(iters):
        f = f + dt * (eps / np.pi) / (eps * eps + f * f) * (-2.0 / rho)
    shell = np.abs(rho - r) <= 3
    moved = np.abs(f - phi0)[shell].max()
    gap = np.abs(got - f)[shell].max()
    say(f"  front moved {moved:.4f}, max gap {gap:.2e}")
    assert 0.2 < moved < 0.3
    assert gap <= 0.02 * moved
