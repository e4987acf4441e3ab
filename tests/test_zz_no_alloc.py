"""rsf_evolve_noalloc through the C ABI: the same evolution as rsf_evolve_ex
on the same inputs (the same kernels, so bit for bit), on two calls in a row
with the second on a smaller volume, no device memory allocated by either
call, and a volume beyond the fixed workspace refused with phi untouched.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2404_02813_amd import inputs  # noqa: E402


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


def case(shape, seed, image="f32"):
    if image == "u16":
        I = inputs.u16_phantom(shape, 6, 1.0, 3.0, seed)
    else:
        I = inputs.vessel_phantom(shape, 6, 1.0, 3.0, seed=seed)
    return torch.from_numpy(I).cuda(), torch.from_numpy(inputs.box_phi0(shape)).cuda()


CASES = [  # (shape zyx, seed, sigma, iters, image, storage)
    ((72, 80, 88), 61, 3.0, 24, "f32", "f32"),
    ((40, 44, 50), 62, 2.0, 13, "f32", "f32"),
    ((64, 70, 66), 63, 4.0, 9, "u16", "f16"),
    ((34, 38, 36), 64, 3.0, 7, "u16", "bf16"),
]


def test_noalloc_equals_evolve_ex_twice_smaller_second(rsf):
    mod, ctx = rsf
    for pair in ((0, 1), (2, 3)):
        runs = []
        for k in pair:
            shape, seed, sigma, iters, image, storage = CASES[k]
            vol, phi0 = case(shape, seed, image)
            params = mod.make_params(sigma, 1.0, 1.0, 0.001, 1.0, 0.1, 1.0, storage=storage)
            ref = phi0.clone()
            ctx.evolve_ex(vol, ref, params, iters)
            _, run_ref, last_ref, hist_ref = ctx.stats(cap=iters)
            got = phi0.clone()
            runs.append((shape, vol, params, iters, ref, run_ref, hist_ref, got))
        # device memory is compared across the two calls alone: the checks
        # below allocate through torch's caching allocator
        torch.cuda.synchronize()
        free_before = torch.cuda.mem_get_info()[0]
        got_stats = []
        for shape, vol, params, iters, ref, run_ref, hist_ref, got in runs:
            say(f"no-alloc evolve {shape} x {iters}, storage {params.storage}")
            ctx.evolve_noalloc(vol, got, params, iters)
            _, run, last, hist = ctx.stats(cap=iters)
            got_stats.append((run, hist))
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free_before
        for (shape, vol, params, iters, ref, run_ref, hist_ref, got), (run, hist) in zip(
                runs, got_stats):
            assert run == run_ref == iters
            assert torch.equal(got, ref), shape
            np.testing.assert_allclose(hist, hist_ref, rtol=1e-12, atol=0.0)


def test_noalloc_refuses_too_large(rsf):
    mod, ctx = rsf
    say("no-alloc: a volume beyond the fixed workspace is refused")
    shape = (200, 200, 200)
    params = mod.make_params(3.0, 1.0, 1.0, 0.001, 1.0, 0.1, 1.0)
    need = mod.rsf_workspace_bytes_params(shape[2], shape[1], shape[0], 5, params)
    assert need > mod.RSF_NOALLOC_MAX_BYTES
    vol = torch.zeros(shape, dtype=torch.float32, device="cuda")
    phi = torch.full(shape, 1.5, dtype=torch.float32, device="cuda")
    with pytest.raises(mod.RsfError) as e:
        ctx.evolve_noalloc(vol, phi, params, 5)
    assert e.value.status == mod.RSF_ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert bool((phi == 1.5).all().item())
