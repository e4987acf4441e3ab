"""Error paths and stream ordering through the C ABI.

- A NaN in the image reaches phi (the fits, the force and the update carry
  it), so the FP64 sum |dphi| is not finite: rsf_get_stats returns
  RSF_ERR_NONFINITE, and so does the server's result for that request, while
  the other requests of the same mix finish normally and bitwise as alone.
- Calls on one context from two streams, each using the context's own
  workspace, are ordered on the device: the results equal those of the same
  calls run one after another on one stream.
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


P = dict(sigma=2.0, lambda1=1.0, lambda2=1.0, nu=0.001, mu=1.0, dt=0.1, eps=1.0)


def case(shape, seed):
    I = inputs.vessel_phantom(shape, 5, 1.0, 3.0, seed=seed)
    return torch.from_numpy(I).cuda(), torch.from_numpy(inputs.box_phi0(shape)).cuda()


def test_nan_image_gives_nonfinite_status(rsf):
    mod, ctx = rsf
    say("NaN in the image -> RSF_ERR_NONFINITE from rsf_get_stats")
    vol, phi = case((20, 24, 28), 31)
    vol[10, 12, 14] = float("nan")
    ctx.evolve(vol, phi, 3, **P)
    with pytest.raises(mod.RsfError) as e:
        ctx.stats(cap=3)
    assert e.value.status == mod.RSF_ERR_NONFINITE
    assert not bool(torch.isfinite(phi).all().item())
    # the context stays usable
    vol2, phi2 = case((20, 24, 28), 32)
    ctx.evolve(vol2, phi2, 3, **P)
    _, run, last, _ = ctx.stats(cap=0)
    assert run == 3 and np.isfinite(last)


def test_nan_request_in_server_mix(rsf):
    mod, ctx = rsf
    say("server: a NaN request gives RSF_ERR_NONFINITE, the others are unaffected")
    shapes = [(22, 26, 30), (24, 20, 28), (26, 30, 22)]
    cases = [case(s, 40 + k) for k, s in enumerate(shapes)]
    cases[1][0][5, 6, 7] = float("nan")
    params = mod.make_params(**P)
    outs = [c[1].clone() for c in cases]
    torch.cuda.synchronize()
    with mod.Server(budget_bytes=1 << 30, chunk_iters=2) as srv:
        tickets = [srv.submit(c[0], o, params, 5) for c, o in zip(cases, outs)]
        results = [srv.wait(t, 120.0) for t in tickets]
    assert results[1]["status"] == mod.RSF_ERR_NONFINITE
    for k in (0, 2):
        assert results[k]["status"] == 0
        ref = cases[k][1].clone()
        ctx.evolve_ex(cases[k][0], ref, params, 5)
        torch.cuda.synchronize()
        assert torch.equal(outs[k], ref), k


def test_two_streams_share_the_workspace_in_order(rsf):
    mod, ctx = rsf
    say("two streams on one context: ordered as if serial")
    a_vol, a_phi0 = case((40, 48, 56), 51)
    b_vol, b_phi0 = case((36, 44, 52), 52)
    params = mod.make_params(**P)
    ref_a, ref_b = a_phi0.clone(), b_phi0.clone()
    ctx.evolve_ex(a_vol, ref_a, params, 12)
    ctx.evolve_ex(b_vol, ref_b, params, 12)
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    got_a, got_b = a_phi0.clone(), b_phi0.clone()
    torch.cuda.synchronize()
    for _ in range(3):
        got_a.copy_(a_phi0)
        got_b.copy_(b_phi0)
        torch.cuda.synchronize()
        ctx.evolve_ex(a_vol, got_a, params, 12, stream=s1)
        ctx.evolve_ex(b_vol, got_b, params, 12, stream=s2)
        torch.cuda.synchronize()
        assert torch.equal(got_a, ref_a)
        assert torch.equal(got_b, ref_b)
    # the statistics are those of the last call (on s2)
    _, run, last, _ = ctx.stats(cap=0)
    assert run == 12 and np.isfinite(last)
