"""Initialisation (Sec. 4.3) on the GPU through the C ABI against the oracle
(pinned in test_init_oracle.py).

Seeds are integer decisions taken from FP32 fields on the GPU and FP64 ones
in the oracle, so they are compared where the FP64 decision has a margin
that FP32 rounding cannot cross; the distance field is compared on the
GPU's own seed set (the sweep is then the same sequence of updates in both)."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_2404_02813_amd import inputs  # noqa: E402

MARGIN = 1e-4       # relative to max |doh| (resp. max |trace|); FP32 errors are ~1e-6 of it
# a distance D is a chain of about D rounded FP32 updates: relative error up
# to about D x 2^-24, i.e. 1e-5 for the largest distances here (~170)
DIST_RTOL, DIST_ATOL = 1e-5, 1e-5


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


def stable_decisions(I, sigma_b, threshold):
    """Oracle seeds plus a mask of voxels whose decision has margin: surely
    not a seed (below the threshold, dark, or a neighbour clearly above) or
    surely one (above the threshold, bright, clearly above every neighbour)."""
    m, doh, tr = oracle.blob_seeds(I, sigma_b, threshold)
    md = MARGIN * np.max(np.abs(doh))
    mt = MARGIN * np.max(np.abs(tr))
    thr = threshold * doh.max()
    nz, ny, nx = doh.shape
    p = np.pad(doh, ((0, 0), (1, 1), (1, 1)), mode="constant", constant_values=-np.inf)
    beaten = np.zeros(doh.shape, bool)
    clear = np.ones(doh.shape, bool)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dy or dx:
                nb = p[:, 1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx]
                beaten |= nb > doh + md
                clear &= doh > nb + md
    sure_no = (doh < thr - md) | (tr > mt) | beaten
    sure_yes = (doh > thr + md) & (tr < -mt) & clear
    return m, sure_no | sure_yes


def volume(kind, shape, seed):
    if kind == "u16":
        u = inputs.u16_phantom(shape, 8, 1.0, 3.0, seed)
        return torch.from_numpy(u).cuda(), u.astype(np.float64) / 65535.0   # as the kernels read it
    I = inputs.vessel_phantom(shape, 8, 1.0, 3.0, seed)
    return torch.from_numpy(np.ascontiguousarray(I)).cuda(), I.astype(np.float64)


CASES = [("f32", (12, 70, 90), 2.0, 0.05, 31), ("f32", (5, 37, 29), 1.0, 0.02, 32),
         ("u16", (16, 64, 80), 1.5, 0.05, 33), ("f32", (3, 130, 66), 3.0, 0.1, 34)]


@pytest.mark.parametrize("kind,shape,sigma_b,threshold,seed", CASES)
def test_seeds_match_oracle(rsf, kind, shape, sigma_b, threshold, seed):
    mod, ctx = rsf
    say(f"seeds {kind} shape={shape} sigma_b={sigma_b} threshold={threshold}")
    vol, I = volume(kind, shape, seed)
    mask, n = ctx.seeds(vol, sigma_b, threshold)
    got = mask.cpu().numpy().astype(bool)
    want, ok = stable_decisions(I, sigma_b, threshold)
    say(f"  seeds gpu={n} oracle={int(want.sum())} stable={ok.mean():.5f}")
    assert n == int(got.sum()) and n > 0
    assert ok.mean() > 0.99
    assert np.array_equal(got[ok], want[ok])


@pytest.mark.parametrize("kind,shape,sigma_b,threshold,seed", CASES)
def test_fast_sweep_matches_oracle(rsf, kind, shape, sigma_b, threshold, seed):
    mod, ctx = rsf
    say(f"fast sweep {kind} shape={shape}")
    vol, _ = volume(kind, shape, seed)
    mask, n = ctx.seeds(vol, sigma_b, threshold)
    m = mask.cpu().numpy().astype(bool)
    u0 = np.where(m, 0.0, oracle.FAR)
    for rounds in (1, 2):
        u = torch.from_numpy(u0.astype(np.float32)).cuda()
        ctx.fast_sweep(u, rounds)
        got = u.cpu().numpy().astype(np.float64)
        want = oracle.fast_sweep(u0, rounds)
        err = np.abs(got - want) - DIST_RTOL * want
        say(f"  rounds={rounds} max|dd|={np.max(np.abs(got - want)):.3e}")
        assert np.all(err <= DIST_ATOL)
        assert np.all(got[m] == 0.0)


def test_fast_sweep_single_seed_exact_on_axes(rsf):
    mod, ctx = rsf
    say("fast sweep: one seed, axis distances")
    shape = (33, 40, 47)
    s = (10, 25, 7)
    u0 = np.full(shape, oracle.FAR, dtype=np.float32)
    u0[s] = 0.0
    u = torch.from_numpy(u0).cuda()
    ctx.fast_sweep(u, 1)
    got = u.cpu().numpy()
    assert np.array_equal(got[s[0], s[1], :], np.abs(np.arange(47) - s[2]).astype(np.float32))
    assert np.array_equal(got[:, s[1], s[2]], np.abs(np.arange(33) - s[0]).astype(np.float32))
    want = oracle.fast_sweep(u0.astype(np.float64), 1)
    assert np.max(np.abs(got - want)) <= DIST_ATOL + DIST_RTOL * want.max()


@pytest.mark.parametrize("offset", [0.0, 2.5])
def test_init_phi_composes_seeds_and_sweep(rsf, offset):
    mod, ctx = rsf
    say(f"init phi offset={offset}")
    vol, _ = volume("f32", (10, 48, 56), 41)
    mask, n = ctx.seeds(vol, 2.0, 0.05)
    u = torch.where(mask.bool(), 0.0, oracle.FAR).float().contiguous()
    ctx.fast_sweep(u, 2)
    phi = torch.empty_like(u)
    k = ctx.init_phi(vol, phi, 2.0, 0.05, offset, 2)
    torch.cuda.synchronize()
    assert k == n
    assert torch.equal(phi, offset - u)


def test_init_phi_feeds_the_evolution(rsf):
    """phi0 from the seeds is a valid start: a few RSF iterations on the GPU
    agree with the oracle from the same phi0."""
    mod, ctx = rsf
    say("init phi then evolve")
    shape = (20, 40, 44)
    vol, I = volume("f32", shape, 42)
    phi = torch.empty(shape, dtype=torch.float32, device="cuda")
    ctx.init_phi(vol, phi, 2.0, 0.05, 1.5, 2)
    phi0 = phi.cpu().numpy().astype(np.float64)
    P = dict(sigma=2.0, lambda1=1.0, lambda2=1.0, nu=0.001, mu=1.0, dt=0.1, eps=1.0)
    ctx.evolve_ex(vol, phi, mod.make_params(**P), 5)
    want, _ = oracle.evolve(I, phi0, oracle.params_array(**P, eta=1e-10), 5)
    got = phi.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - want)) <= 1e-3


def test_init_rejects_bad_arguments(rsf):
    mod, ctx = rsf
    say("init: invalid arguments")
    vol, _ = volume("f32", (4, 20, 20), 43)
    phi = torch.full((4, 20, 20), 7.0, device="cuda")
    for bad in [dict(sigma_b=0.0, threshold=0.1), dict(sigma_b=6.0, threshold=0.1),
                dict(sigma_b=1.0, threshold=1.0), dict(sigma_b=1.0, threshold=-0.1)]:
        with pytest.raises(mod.RsfError) as e:
            ctx.init_phi(vol, phi, bad["sigma_b"], bad["threshold"])
        assert e.value.status == mod.RSF_ERR_INVALID_ARG
    with pytest.raises(mod.RsfError) as e:       # a constant zero image has no blob
        ctx.init_phi(torch.zeros_like(vol), phi, 1.0, 0.1)
    assert e.value.status == mod.RSF_ERR_INVALID_ARG
    with pytest.raises(mod.RsfError):
        ctx.fast_sweep(phi, 0)
    torch.cuda.synchronize()
    assert torch.all(phi == 7.0)


def test_init_phi_caller_workspace_is_bitwise_the_same(rsf):
    """rsf_init_phi_ex on a reused caller workspace (second call on a smaller
    volume, the workspace holding the first call's fields) equals
    rsf_init_phi; a workspace one byte short is refused with phi untouched."""
    mod, ctx = rsf
    say("init phi: caller workspace")
    need = mod.rsf_init_workspace_bytes((16, 52, 60))
    n = 16 * 52 * 60
    assert need >= n + 4 * 4 * n + 2 * 65536 * 4
    big = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    ws = big[:need]
    for shape, seed in [((16, 52, 60), 44), ((9, 30, 34), 45)]:
        vol, _ = volume("f32", shape, seed)
        want = torch.empty(shape, dtype=torch.float32, device="cuda")
        got = torch.full(shape, 3.0, dtype=torch.float32, device="cuda")
        k0 = ctx.init_phi(vol, want, 2.0, 0.05, 1.0, 2)
        k1 = mod.rsf_init_phi_ex(ctx.handle, vol, got, 2.0, 0.05, 1.0, 2, ws)
        torch.cuda.synchronize()
        assert k0 == k1 and k0 > 0
        assert torch.equal(got, want)
    vol, _ = volume("f32", (16, 52, 60), 46)
    phi = torch.full((16, 52, 60), 7.0, device="cuda")
    with pytest.raises(mod.RsfError) as e:
        mod.rsf_init_phi_ex(ctx.handle, vol, phi, 2.0, 0.05, 1.0, 2, ws[:need - 1])
    assert e.value.status == mod.RSF_ERR_INVALID_ARG
    with pytest.raises(mod.RsfError) as e:       # misaligned
        mod.rsf_init_phi_ex(ctx.handle, vol, phi, 2.0, 0.05, 1.0, 2, big[1:need + 1])
    assert e.value.status == mod.RSF_ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert torch.all(phi == 7.0)
    assert mod.rsf_init_workspace_bytes((0, 4, 4)) == 0


def test_seeds_caller_workspace_is_bitwise_the_same(rsf):
    """rsf_seeds_ex on a reused workspace (second call smaller) equals
    rsf_seeds; a short or misaligned workspace is refused, mask untouched."""
    mod, ctx = rsf
    say("seeds: caller workspace")
    need = mod.rsf_seeds_workspace_bytes((14, 50, 58))
    assert need == mod.rsf_init_workspace_bytes((14, 50, 58)) - ((14 * 50 * 58 + 255) // 256) * 256
    big = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    ws = big[:need]
    for shape, seed in [((14, 50, 58), 47), ((7, 33, 31), 48)]:
        vol, _ = volume("f32", shape, seed)
        want, n0 = ctx.seeds(vol, 2.0, 0.05)
        got, n1 = mod.rsf_seeds_ex(ctx.handle, vol, 2.0, 0.05, None, ws)
        torch.cuda.synchronize()
        assert n0 == n1 and n0 > 0
        assert torch.equal(got, want)
    vol, _ = volume("f32", (14, 50, 58), 49)
    mask = torch.full((14, 50, 58), 9, dtype=torch.uint8, device="cuda")
    for bad in (ws[:need - 1], big[1:need + 1]):
        with pytest.raises(mod.RsfError) as e:
            mod.rsf_seeds_ex(ctx.handle, vol, 2.0, 0.05, mask, bad)
        assert e.value.status == mod.RSF_ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert torch.all(mask == 9)
    assert mod.rsf_seeds_workspace_bytes((4, 0, 4)) == 0
