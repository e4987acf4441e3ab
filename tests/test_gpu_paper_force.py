"""The force of Sec. 4.2 (sigma2 = 0, as in the paper's 3D runs) on the GPU,
through the C ABI, against the FP64 oracle's force = 1 path (pinned in
test_oracle_pins.py), with the same bar as the RSF force:
  - one-step fields within FP32 rounding of the value;
  - after N iterations max|dphi| <= 1e-3 (8e-3 with BF16 storage) and
    >= 99.99 % agreement of phi > 0;
and the batch and server paths bitwise equal to each tile alone.  sigma2 > 0
(K2*I and K2*I^2 precomputed with their own Gaussian) is held to the same bar.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_2404_02813_amd import inputs  # noqa: E402

PHI_TOL = 1e-3
SIGN_AGREE = 0.9999


def phi_tol(storage):
    """max|dphi| bar after N iterations: 1e-3 (FP32 arithmetic; FP32 or FP16
    storage).  BF16 storage keeps 8 significand bits: the bar scales with its
    unit roundoff over FP16's, 2^-8 / 2^-11 = 8."""
    return PHI_TOL * (8.0 if storage == "bf16" else 1.0)


FIELD_TOL = {"H": 1e-6, "f1": 2e-5, "f2": 2e-5, "Fd": 2e-5, "kappa": 2e-5, "lap": 2e-5,
             "R": 2e-5, "E": 2e-5, "phi_next": 2e-6}


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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def smooth(shape, seed, amp=3.0):
    from scipy.ndimage import gaussian_filter
    r = np.random.default_rng(seed)
    return (amp * 4.0 * gaussian_filter(r.normal(size=shape), 1.5, mode="reflect")).astype(np.float32)


P = dict(sigma=3.0, lambda1=1.0, lambda2=1.0, nu=0.001, mu=1.0, dt=0.1, eps=1.0)


def gparams(mod, storage="f32", reg=0, **kw):
    p = dict(P, **kw)
    return mod.make_params(**p, eta=1e-10, regulariser=reg, storage=storage,
                           force=mod.RSF_FORCE_PAPER, sigma2=0.0)


def oparams(**kw):
    return oracle.params_array(**dict(P, **kw), eta=1e-10, force=oracle.FORCE_PAPER, sigma2=0.0)


def parity(got, want):
    d = np.abs(got - want)
    return float(d.max()), float(np.mean((got > 0) == (want > 0)))


@pytest.mark.parametrize("shape,sigma,reg", [((35, 37, 40), 3.0, 0), ((35, 37, 40), 3.0, 1),
                                             ((21, 19, 70), 2.0, 0), ((9, 8, 7), 3.0, 0)])
def test_paper_force_probe_fields(rsf, shape, sigma, reg):
    mod, ctx = rsf
    say(f"paper force probe shape={shape} sigma={sigma} reg={reg}")
    I = inputs.vessel_phantom(shape, 6, 1.0, 3.0, seed=3)
    phi = smooth(shape, 4)
    kw = dict(sigma=sigma, lambda1=2.0, lambda2=1.5, nu=0.2)
    got = {k: host(v) for k, v in ctx.probe(dev(I), dev(phi), gparams(mod, reg=reg, **kw)).items()}
    nxt, f, _ = oracle.step(I, phi, oparams(**kw), reg=1 - reg)
    want = dict(f)
    want["Fd"] = 2.0 * f["e1"] - 1.5 * f["e2"]
    want["phi_next"] = nxt
    for k, tol in FIELD_TOL.items():
        scale = max(1.0, float(np.max(np.abs(want[k]))))
        err = float(np.max(np.abs(got[k] - want[k])))
        assert err < tol * scale, (k, err, scale)


@pytest.mark.parametrize("shape,sigma,iters", [((64, 64, 64), 3.0, 20), ((45, 71, 67), 2.0, 60),
                                               ((20, 33, 130), 5.0, 30)])
def test_paper_force_evolution(rsf, shape, sigma, iters):
    mod, ctx = rsf
    say(f"paper force evolve shape={shape} sigma={sigma} iters={iters}")
    I = inputs.vessel_phantom(shape, 8, 1.0, 3.0, seed=61)
    phi0 = inputs.box_phi0(shape)
    phi = dev(phi0)
    ctx.evolve_ex(dev(I), phi, gparams(mod, sigma=sigma), iters)
    _, run, _, hist = ctx.stats(cap=iters)
    want, whist = oracle.evolve(I, phi0, oparams(sigma=sigma), iters)
    dmax, agree = parity(host(phi), want)
    say(f"  max|dphi|={dmax:.3e} agree={agree:.7f}")
    assert run == iters
    assert dmax <= PHI_TOL and agree >= SIGN_AGREE
    assert np.max(np.abs(np.array(hist) / whist - 1.0)) < 1e-3


@pytest.mark.parametrize("storage", ["f16", "bf16", "f32"])
def test_paper_force_mixed_precision(rsf, storage):
    """uint16 image, FP16/BF16/FP32 storage of the convolved fields (the
    force itself is kept in FP32), sigma 4, 150 iterations."""
    mod, ctx = rsf
    n, iters = 96, 150
    say(f"paper force mixed precision storage={storage}")
    u = inputs.u16_phantom((n, n, n), 30, 1.0, 4.0, seed=41)
    I = u.astype(np.float64) / 65535.0
    phi0 = inputs.box_phi0((n, n, n))
    phi = dev(phi0)
    ctx.evolve_ex(torch.from_numpy(u).cuda(), phi, gparams(mod, storage=storage, sigma=4.0), iters)
    want, _ = oracle.evolve(I, phi0, oparams(sigma=4.0), iters)
    dmax, agree = parity(host(phi), want)
    say(f"  max|dphi|={dmax:.3e} agree={agree:.7f}")
    assert dmax <= phi_tol(storage) and agree >= SIGN_AGREE


def test_paper_force_batch_and_server_equal_alone(rsf):
    mod, ctx = rsf
    say("paper force: batch and server vs alone")
    shapes = [(40, 50, 60), (33, 47, 61), (27, 27, 150)]
    vols = [dev(inputs.vessel_phantom(s, 6, 1.0, 3.0, seed=70 + k)) for k, s in enumerate(shapes)]
    phis = [dev(inputs.tile_phi0(s, 9)) for s in shapes]
    p = gparams(mod)
    alone = []
    for v, q in zip(vols, phis):
        a = q.clone()
        ctx.evolve_ex(v, a, p, 13)
        alone.append(a)
    batch = [q.clone() for q in phis]
    ctx.evolve_batch(vols, batch, p, 13)
    torch.cuda.synchronize()
    for a, b in zip(alone, batch):
        assert torch.equal(a, b)
    # the server mixes them with RSF-force requests (a different group)
    rsf_p = mod.make_params(**P)
    outs = [q.clone() for q in phis] + [q.clone() for q in phis]
    torch.cuda.synchronize()
    with mod.Server(budget_bytes=4 << 30, chunk_iters=4) as srv:
        tickets = [srv.submit(v, o, p, 13) for v, o in zip(vols, outs[:3])]
        tickets += [srv.submit(v, o, rsf_p, 13) for v, o in zip(vols, outs[3:])]
        results = [srv.wait(t, 120.0) for t in tickets]
    assert all(r["status"] == 0 for r in results)
    for a, b in zip(alone, outs[:3]):
        assert torch.equal(a, b)
    for v, q, b in zip(vols, phis, outs[3:]):
        a = q.clone()
        ctx.evolve_ex(v, a, rsf_p, 13)
        torch.cuda.synchronize()
        assert torch.equal(a, b)


def g2params(mod, sigma2, storage="f32", **kw):
    p = dict(P, **kw)
    return mod.make_params(**p, eta=1e-10, storage=storage, force=mod.RSF_FORCE_PAPER,
                           sigma2=sigma2)


def o2params(sigma2, **kw):
    return oracle.params_array(**dict(P, **kw), eta=1e-10, force=oracle.FORCE_PAPER, sigma2=sigma2)


@pytest.mark.parametrize("shape,sigma,sigma2", [((35, 37, 40), 3.0, 1.0), ((21, 19, 70), 2.0, 3.0),
                                                ((18, 25, 31), 1.5, 5.0)])
def test_paper_force_sigma2_probe_fields(rsf, shape, sigma, sigma2):
    """sigma2 > 0: K2*I and K2*I^2 precomputed with their own Gaussian."""
    mod, ctx = rsf
    say(f"paper force sigma2={sigma2} probe shape={shape} sigma={sigma}")
    I = inputs.vessel_phantom(shape, 6, 1.0, 3.0, seed=5)
    phi = smooth(shape, 6)
    kw = dict(sigma=sigma, lambda1=2.0, lambda2=1.5, nu=0.2)
    got = {k: host(v) for k, v in ctx.probe(dev(I), dev(phi), g2params(mod, sigma2, **kw)).items()}
    nxt, f, _ = oracle.step(I, phi, o2params(sigma2, **kw), reg=1)
    want = dict(f)
    want["Fd"] = 2.0 * f["e1"] - 1.5 * f["e2"]
    want["phi_next"] = nxt
    for k, tol in FIELD_TOL.items():
        scale = max(1.0, float(np.max(np.abs(want[k]))))
        err = float(np.max(np.abs(got[k] - want[k])))
        assert err < tol * scale, (k, err, scale)


@pytest.mark.parametrize("storage,image,sigma2,iters", [("f32", "f32", 1.5, 20), ("f16", "u16", 2.0, 60),
                                                        ("f32", "u16", 4.0, 40)])
def test_paper_force_sigma2_evolution(rsf, storage, image, sigma2, iters):
    mod, ctx = rsf
    n = 64
    say(f"paper force sigma2={sigma2} evolve {storage}/{image} iters={iters}")
    if image == "u16":
        u = inputs.u16_phantom((n, n, n), 16, 1.0, 4.0, seed=47)
        I = u.astype(np.float64) / 65535.0
        vol = torch.from_numpy(u).cuda()
    else:
        I = inputs.vessel_phantom((n, n, n), 16, 1.0, 3.0, seed=48)
        vol = dev(I)
    phi0 = inputs.box_phi0((n, n, n))
    phi = dev(phi0)
    ctx.evolve_ex(vol, phi, g2params(mod, sigma2, storage=storage, sigma=4.0), iters)
    want, _ = oracle.evolve(I, phi0, o2params(sigma2, sigma=4.0), iters)
    dmax, agree = parity(host(phi), want)
    say(f"  max|dphi|={dmax:.3e} agree={agree:.7f}")
    assert dmax <= phi_tol(storage) and agree >= SIGN_AGREE


def test_paper_force_sigma2_server_and_workspace(rsf):
    mod, ctx = rsf
    say("paper force sigma2 > 0: workspace size, server vs alone")
    p = g2params(mod, 1.0)
    base = mod.rsf_workspace_bytes(40, 50, 60, 10, mod.RSF_F32)
    assert mod.rsf_workspace_bytes_params(40, 50, 60, 10, p) >= base + 2 * 40 * 50 * 60 * 4
    assert mod.rsf_workspace_bytes_params(40, 50, 60, 10, mod.make_params(**P)) == base
    shapes = [(40, 50, 60), (33, 47, 61)]
    vols = [dev(inputs.vessel_phantom(s, 6, 1.0, 3.0, seed=80 + k)) for k, s in enumerate(shapes)]
    phis = [dev(inputs.tile_phi0(s, 9)) for s in shapes]
    alone = []
    for v, q in zip(vols, phis):
        a = q.clone()
        ctx.evolve_ex(v, a, p, 9)
        alone.append(a)
    outs = [q.clone() for q in phis]
    torch.cuda.synchronize()
    with mod.Server(budget_bytes=2 << 30, chunk_iters=4) as srv:
        tickets = [srv.submit(v, o, p, 9) for v, o in zip(vols, outs)]
        results = [srv.wait(t, 120.0) for t in tickets]
    assert all(r["status"] == 0 for r in results)
    for a, b in zip(alone, outs):
        assert torch.equal(a, b)


def test_paper_force_sigma2_limits(rsf):
    mod, ctx = rsf
    say("paper force: sigma2 outside the built radii is refused")
    phi = dev(inputs.box_phi0((8, 8, 8)))
    before = phi.clone()
    for vol, p in [(dev(np.zeros((8, 8, 8))), g2params(mod, 6.0)),                  # R2 = 18
                   (torch.zeros((8, 8, 8), dtype=torch.uint16, device="cuda"),
                    g2params(mod, 0.5, storage="f16"))]:                            # R2 = 2
        with pytest.raises(mod.RsfError) as e:
            ctx.evolve_ex(vol, phi, p, 2)
        assert e.value.status == mod.RSF_ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert torch.equal(phi, before)


# --- the update fused with the next iteration's stage-1 z pass -------------

# Fusion needs every tile's update marched whole in z: volumes whose xy plane
# alone fills the resident update workgroups (>= 384 columns of 64 x 8), or
# tiles of at most 8 slices.
FUSE_CASES = [  # (shape zyx, image, storage, sigma, sigma2, iters, tol)
    ((40, 770, 256), "f32", "f32", 3.0, 0.0, 9, 0.0),
    ((8, 47, 29), "u16", "f16", 2.0, 0.0, 12, 0.0),
    ((30, 780, 260), "f32", "bf16", 4.0, 0.0, 5, 0.0),
    ((7, 44, 38), "f32", "f32", 2.0, 1.5, 7, 0.0),
    ((8, 34, 34), "f32", "f32", 3.0, 0.0, 80, 2e-3),
    ((6, 21, 23), "f32", "f32", 1.0, 0.0, 4, 0.0),
]


def fuse_case(mod, shape, image, seed):
    if image == "u16":
        vol = torch.from_numpy(inputs.u16_phantom(shape, 6, 1.0, 3.0, seed)).cuda()
    else:
        vol = dev(inputs.vessel_phantom(shape, 6, 1.0, 3.0, seed))
    return vol, dev(inputs.box_phi0(shape))


@pytest.mark.parametrize("shape,image,storage,sigma,sigma2,iters,tol", FUSE_CASES)
def test_fused_update_is_bitwise_the_separate_passes(rsf, shape, image, storage, sigma, sigma2,
                                                     iters, tol):
    """The fused update writes the next stage-1 pair exactly as the stage-1
    pass would: the whole evolution is bitwise the same, and the stage-1 pass
    is launched once instead of once per iteration."""
    mod, ctx = rsf
    say(f"fused update {shape} {image}/{storage} sigma={sigma} sigma2={sigma2} iters={iters}")
    vol, phi0 = fuse_case(mod, shape, image, 311)
    p = mod.make_params(sigma, 1.0, 1.0, 0.001, 1.0, 0.1, 1.0, storage=storage,
                        force=mod.RSF_FORCE_PAPER, sigma2=sigma2)
    out = {}
    for fuse in (False, True):
        ctx.set_fusion(fuse)
        phi = phi0.clone()
        ctx.profile(True)
        ctx.evolve_ex(vol, phi, p, iters, tol=tol)
        ctx.profile(False)
        prof = ctx.profile_read()
        _, run, last, _ = ctx.stats(cap=0)
        out[fuse] = (phi, run, last, prof["z_heaviside"][0])
    ctx.set_fusion(True)
    torch.cuda.synchronize()
    (a, run_a, last_a, zh_a), (b, run_b, last_b, zh_b) = out[False], out[True]
    say(f"  iterations {run_a}/{run_b}, stage-1 launches {zh_a} -> {zh_b}")
    assert torch.equal(a, b)
    assert run_a == run_b and last_a == last_b
    assert zh_a == iters and zh_b == 1   # stopped tiles exit launched passes early
    if tol > 0:
        assert run_a < iters


def test_fused_update_in_a_batch(rsf):
    """Tiles of one batch, each marched whole in z, fused together; each is
    bitwise the separate passes' result."""
    mod, ctx = rsf
    say("fused update: batch of tiles")
    shapes = [(8, 40, 50), (6, 36, 28), (8, 24, 33)]
    cases = [fuse_case(mod, sh, "f32", 320 + k) for k, sh in enumerate(shapes)]
    p = mod.make_params(3.0, 1.0, 1.0, 0.001, 1.0, 0.1, 1.0, force=mod.RSF_FORCE_PAPER)
    res = {}
    for fuse in (False, True):
        ctx.set_fusion(fuse)
        phis = [c[1].clone() for c in cases]
        ctx.profile(True)
        ctx.evolve_batch([c[0] for c in cases], phis, p, 6)
        ctx.profile(False)
        res[fuse] = (phis, ctx.profile_read()["z_heaviside"][0])
    ctx.set_fusion(True)
    torch.cuda.synchronize()
    assert res[True][1] == 1 and res[False][1] == 6
    for a, b in zip(res[False][0], res[True][0]):
        assert torch.equal(a, b)


# --- the Sec. 4.2 workload at full size (512^3, sigma 3, fused update) -------

@pytest.fixture(scope="module")
def large():
    w = inputs.LARGE_512
    say(f"generating {w.name}")
    return w, w.image(), w.phi0()


def test_full_size_two_iterations_sampled(rsf, large):
    """Two iterations as the throughput workload runs them (the second reads
    the stage-1 pair the fused first update wrote), against the oracle on
    crops whose inner faces lie beyond two iterations' reach."""
    mod, ctx = rsf
    w, I, phi0 = large
    say(f"{w.name} (Sec. 4.2 force): two iterations, sampled voxels")
    p = mod.make_params(**w.params(), force=mod.RSF_FORCE_PAPER)
    phi = dev(phi0)
    ctx.profile(True)
    ctx.evolve_ex(dev(I), phi, p, 2)
    ctx.profile(False)
    assert ctx.profile_read()["z_heaviside"][0] == 1   # the fused path ran
    got = host(phi)
    R = oracle.radius(w.sigma)
    margin = 2 * (2 * R + 3)
    po = oracle.params_array(**w.params(), eta=1e-10, force=oracle.FORCE_PAPER)
    r = np.random.default_rng(21)
    centers = [tuple(int(v) for v in r.integers(0, 512, 3)) for _ in range(4)]
    centers += [(0, 0, 0), (511, 511, 511), (256, 3, 500), (300, 200, 100)]
    for c in centers:
        sl = tuple(slice(max(0, k - margin), min(n, k + margin + 1)) for k, n in zip(c, I.shape))
        want, _ = oracle.evolve(I[sl], phi0[sl], po, 2)
        local = tuple(k - s.start for k, s in zip(c, sl))
        assert abs(got[c] - want[local]) < 4e-6, (c, got[c], want[local])


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_full_size_fused_equals_separate_passes(rsf, large, storage):
    mod, ctx = rsf
    w, I, phi0 = large
    say(f"{w.name} (Sec. 4.2 force): {w.iters} iterations fused vs separate, {storage}")
    p = mod.make_params(**w.params(), force=mod.RSF_FORCE_PAPER, storage=storage)
    vol = dev(I)
    out = []
    for fuse in (True, False):
        ctx.set_fusion(fuse)
        phi = dev(phi0)
        ctx.evolve_ex(vol, phi, p, w.iters)
        out.append(phi)
    ctx.set_fusion(True)
    torch.cuda.synchronize()
    assert torch.equal(out[0], out[1])
    assert bool(torch.isfinite(out[0]).all())
