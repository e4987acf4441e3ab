"""The volume-level driver (Sec. 4.1) on the GPU through the C ABI: curtained
sub-volumes evolved in batches and merged by linear interpolation, against
the oracle's own split/evolve/merge (pinned in test_volume_oracle.py)."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_2404_02813_amd import inputs  # noqa: E402

PHI_TOL = 1e-3
SIGN_AGREE = 0.9999
P = dict(sigma=1.0, lambda1=1.0, lambda2=1.0, nu=0.001, mu=1.0, dt=0.1, eps=1.0)


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


def case(shape=(36, 40, 44), seed=91):
    I = inputs.vessel_phantom(shape, 8, 1.0, 3.0, seed=seed)
    phi0 = inputs.box_phi0(shape)
    return I, phi0


@pytest.mark.parametrize("shape,block,curtain,iters", [((36, 40, 44), 20, 3, 8),
                                                       ((30, 50, 70), 25, 4, 12),
                                                       ((64, 20, 33), 30, 5, 6)])
def test_volume_driver_matches_oracle(rsf, shape, block, curtain, iters):
    mod, ctx = rsf
    say(f"volume driver shape={shape} block={block} curtain={curtain} iters={iters}")
    I, phi0 = case(shape)
    phi = dev(phi0)
    ctx.evolve_volume(dev(I), phi, mod.make_params(**P), iters, block, curtain)
    want = oracle.evolve_volume(I, phi0, oracle.params_array(**P, eta=1e-10), iters, block,
                                curtain)
    got = host(phi)
    d = np.abs(got - want)
    agree = float(np.mean((got > 0) == (want > 0)))
    say(f"  max|dphi|={d.max():.3e} agree={agree:.7f}")
    assert d.max() <= PHI_TOL and agree >= SIGN_AGREE


def test_volume_driver_zero_iterations_and_single_block(rsf):
    mod, ctx = rsf
    say("volume driver: iters = 0, one sub-volume")
    I, phi0 = case()
    p = mod.make_params(**P)
    phi = dev(phi0)
    ctx.evolve_volume(dev(I), phi, p, 0, 20, 3)
    assert np.max(np.abs(host(phi) - phi0)) < 1e-6        # weights sum to one in FP32
    a = dev(phi0)
    ctx.evolve_volume(dev(I), a, p, 7, 1000, 3)           # one sub-volume
    b = dev(phi0)
    ctx.evolve_ex(dev(I), b, p, 7)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_volume_driver_budget_groups_are_bitwise_equal(rsf):
    mod, ctx = rsf
    say("volume driver: budget-limited groups")
    I, phi0 = case((40, 42, 44), seed=92)
    p = mod.make_params(**P, storage="f32")
    vol = dev(I)
    a = dev(phi0)
    ctx.evolve_volume(vol, a, p, 5, 15, 3)
    b = dev(phi0)
    ctx.evolve_volume(vol, b, p, 5, 15, 3, budget_bytes=3 << 20)   # several groups
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_volume_driver_uint16_paper_force(rsf):
    mod, ctx = rsf
    say("volume driver: uint16 image, FP16 storage, Sec. 4.2 force")
    shape = (40, 48, 52)
    u = inputs.u16_phantom(shape, 10, 1.0, 3.0, seed=93)
    I = u.astype(np.float64) / 65535.0
    phi0 = inputs.box_phi0(shape)
    kw = dict(P, sigma=2.0)
    phi = dev(phi0)
    ctx.evolve_volume(torch.from_numpy(u).cuda(), phi,
                      mod.make_params(**kw, storage="f16", force=mod.RSF_FORCE_PAPER), 10, 24, 6)
    want = oracle.evolve_volume(I, phi0, oracle.params_array(**kw, eta=1e-10,
                                                             force=oracle.FORCE_PAPER), 10, 24, 6)
    got = host(phi)
    d = np.abs(got - want)
    say(f"  max|dphi|={d.max():.3e}")
    assert d.max() <= PHI_TOL and np.mean((got > 0) == (want > 0)) >= SIGN_AGREE


def test_volume_driver_rejects_bad_geometry(rsf):
    mod, ctx = rsf
    say("volume driver: invalid geometry")
    I, phi0 = case((30, 30, 30))
    p = mod.make_params(**P)
    phi = dev(phi0)
    before = phi.clone()
    with pytest.raises(mod.RsfError) as e:
        ctx.evolve_volume(dev(I), phi, p, 3, 10, 6)       # cores of 10 < 2 x 6
    assert e.value.status == mod.RSF_ERR_INVALID_ARG
    with pytest.raises(mod.RsfError) as e:
        ctx.evolve_volume(dev(I), phi, p, 3, 15, 3, budget_bytes=1 << 10)
    assert e.value.status == mod.RSF_ERR_BUDGET
    torch.cuda.synchronize()
    assert torch.equal(phi, before)


def test_volume_driver_caller_workspace_is_bitwise_the_same(rsf):
    """rsf_evolve_volume_ex with every device buffer in a caller-owned
    workspace: bitwise the result of the driver's own allocations, for one
    group and for several groups under a budget; a workspace one byte short
    is refused with phi untouched."""
    mod, ctx = rsf
    I, phi0 = case((40, 44, 50), seed=95)
    vol = dev(I)
    p = mod.make_params(**P)
    for budget in (0, 3 << 20):
        say(f"volume driver, caller workspace, budget {budget}")
        ref = dev(phi0)
        ctx.evolve_volume(vol, ref, p, 6, 18, 3, budget_bytes=budget)
        need = ctx.volume_workspace_bytes(torch.float32, I.shape, p, 6, 18, 3, budget)
        assert need > 0
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        got = dev(phi0)
        ctx.evolve_volume(vol, got, p, 6, 18, 3, budget_bytes=budget, workspace=ws)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
        short = dev(phi0)
        with pytest.raises(mod.RsfError) as e:
            ctx.evolve_volume(vol, short, p, 6, 18, 3, budget_bytes=budget, workspace=ws[:need - 1])
        assert e.value.status == mod.RSF_ERR_INVALID_ARG
        assert torch.equal(short, dev(phi0))
