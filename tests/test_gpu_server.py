"""The request server (continuous batching) through the C ABI.

Every tile's phi from the server must be bitwise the result of evolving that
tile alone with rsf_evolve_ex (same parameters, iterations and tolerance):
tiles share launches but no arithmetic.  The FP64 convergence sums agree up
to the grouping of their partial sums.  Admission must respect
the HBM budget.  The single-tile path itself is checked against the oracle
in test_gpu_parity.py.
"""
import math
import sys
import time

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


def make_request(mod, seed, interior, sigma, iters, image="u16", storage="f16", tol=0.0):
    """A tile with a ceil(3 sigma) halo cut from its own small phantom."""
    R = math.ceil(3 * sigma - 1e-9)
    shape = tuple(e + 2 * R for e in interior)
    if image == "u16":
        vol = torch.from_numpy(inputs.u16_phantom(shape, 6, 1.0, 3.0, seed)).cuda()
    else:
        vol = torch.from_numpy(inputs.vessel_phantom(shape, 6, 1.0, 3.0, seed)).cuda()
    phi0 = torch.from_numpy(inputs.tile_phi0(shape, R)).cuda()
    p = mod.make_params(sigma, 1.0, 1.0, 0.001, 1.0, 0.1, 1.0, 1e-10, 0, storage)
    return {"vol": vol, "phi0": phi0, "params": p, "iters": iters, "tol": tol}


MIX = [  # (interior zyx, sigma, iters, image, storage)
    ((30, 36, 40), 2.0, 9, "u16", "f16"),
    ((24, 40, 33), 3.0, 14, "u16", "f16"),
    ((40, 24, 28), 4.0, 6, "u16", "f16"),
    ((20, 20, 64), 2.0, 17, "u16", "f16"),
    ((33, 29, 31), 3.0, 4, "u16", "f16"),
    ((26, 50, 22), 3.0, 11, "u16", "f16"),
    ((36, 36, 36), 4.0, 13, "u16", "f16"),
    ((28, 34, 30), 3.0, 7, "f32", "f32"),
    ((31, 27, 45), 3.0, 12, "f32", "f32"),
    ((22, 30, 26), 2.0, 3, "u16", "bf16"),
]


def requests(mod, base_seed=500):
    return [make_request(mod, base_seed + k, *m) for k, m in enumerate(MIX)]


def alone(ctx, rq):
    phi = rq["phi0"].clone()
    ctx.evolve_ex(rq["vol"], phi, rq["params"], rq["iters"], tol=rq["tol"])
    _, run, last, _ = ctx.stats(cap=0)
    return phi, run, last


def check_equal_alone(ctx, reqs, outs, results):
    for k, (rq, out, res) in enumerate(zip(reqs, outs, results)):
        ref, run, last = alone(ctx, rq)
        torch.cuda.synchronize()
        assert res["status"] == 0, (k, res)
        assert res["iters_run"] == run, (k, res["iters_run"], run)
        # the FP64 sum is grouped per update workgroup, which depends on the
        # split (a tile's share of its batch): equal up to rounding order
        assert res["last_sum_abs"] == pytest.approx(last, rel=1e-12, abs=0.0), k
        assert torch.equal(out, ref), k


def test_server_mix_equals_alone(rsf):
    mod, ctx = rsf
    say("server: mixed sigma/type requests vs alone (bitwise)")
    reqs = requests(mod)
    outs = [rq["phi0"].clone() for rq in reqs]
    torch.cuda.synchronize()
    with mod.Server(budget_bytes=8 << 30, chunk_iters=4) as srv:
        tickets = [srv.submit(rq["vol"], o, rq["params"], rq["iters"]) for rq, o in zip(reqs, outs)]
        results = [srv.wait(t, 120.0) for t in tickets]
        st = srv.stats()
    assert all(r is not None for r in results)
    assert st["completed"] == len(reqs) and st["resident"] == 0 and st["bytes_in_use"] == 0
    assert st["peak_resident"] > 1   # they did share the device
    for r in results:
        assert r["t_submit"] <= r["t_admit"] <= r["t_done"]
    check_equal_alone(ctx, reqs, outs, results)


def test_server_staggered_arrivals(rsf):
    """Requests that arrive while others run join the batch at a chunk
    boundary; results are unchanged."""
    mod, ctx = rsf
    say("server: staggered arrivals")
    reqs = requests(mod, 600)
    outs = [rq["phi0"].clone() for rq in reqs]
    torch.cuda.synchronize()
    with mod.Server(budget_bytes=8 << 30, chunk_iters=2) as srv:
        tickets = []
        for rq, o in zip(reqs, outs):
            tickets.append(srv.submit(rq["vol"], o, rq["params"], rq["iters"]))
            time.sleep(0.003)
        results = [srv.wait(t, 120.0) for t in tickets]
    check_equal_alone(ctx, reqs, outs, results)


def test_server_budget_bounds_residency(rsf):
    mod, ctx = rsf
    say("server: budget admission")
    reqs = requests(mod, 700)[:7]
    ws = [mod.rsf_workspace_bytes(*reversed(rq["phi0"].shape), rq["iters"],
                                  rq["params"].storage) for rq in reqs]
    budget = int(2.2 * max(ws))
    outs = [rq["phi0"].clone() for rq in reqs]
    torch.cuda.synchronize()
    with mod.Server(budget_bytes=budget, chunk_iters=3, segment_bytes=1 << 20) as srv:
        tickets = [srv.submit(rq["vol"], o, rq["params"], rq["iters"]) for rq, o in zip(reqs, outs)]
        results = [srv.wait(t, 120.0) for t in tickets]
        st = srv.stats()
    assert st["peak_bytes"] <= budget
    assert st["bytes_reserved"] <= budget
    assert 1 <= st["peak_resident"] < len(reqs)
    for r, w in zip(results, ws):
        assert r["workspace_bytes"] == w
    check_equal_alone(ctx, reqs, outs, results)


def test_server_tolerance_and_zero_iters(rsf):
    mod, ctx = rsf
    say("server: tolerance stop and zero iterations")
    reqs = [make_request(mod, 801, (30, 30, 30), 3.0, 60, "f32", "f32", tol=2e-3),
            make_request(mod, 802, (26, 34, 30), 2.0, 60, "u16", "f16", tol=2e-3),
            make_request(mod, 803, (30, 30, 30), 3.0, 0, "f32", "f32"),
            make_request(mod, 804, (28, 28, 28), 3.0, 5, "f32", "f32")]
    outs = [rq["phi0"].clone() for rq in reqs]
    torch.cuda.synchronize()
    with mod.Server(budget_bytes=4 << 30, chunk_iters=4) as srv:
        tickets = [srv.submit(rq["vol"], o, rq["params"], rq["iters"], rq["tol"])
                   for rq, o in zip(reqs, outs)]
        results = [srv.wait(t, 120.0) for t in tickets]
    assert results[0]["iters_run"] < 60 and results[1]["iters_run"] < 60
    assert results[2]["iters_run"] == 0 and torch.equal(outs[2], reqs[2]["phi0"])
    check_equal_alone(ctx, reqs, outs, results)


def test_server_rejects_bad_requests(rsf):
    mod, _ = rsf
    say("server: invalid requests")
    rq = make_request(mod, 900, (20, 20, 20), 3.0, 4, "f32", "f32")
    ws = mod.rsf_workspace_bytes(*reversed(rq["phi0"].shape), 4, mod.RSF_F32)
    with mod.Server(budget_bytes=ws - 1024) as srv:
        with pytest.raises(mod.RsfError) as e:
            srv.submit(rq["vol"], rq["phi0"].clone(), rq["params"], 4)
        assert e.value.status == mod.RSF_ERR_BUDGET
        bad = mod.make_params(0.0, 1.0, 1.0, 0.001, 1.0, 0.1, 1.0)
        with pytest.raises(mod.RsfError) as e:
            srv.submit(rq["vol"], rq["phi0"].clone(), bad, 4)
        assert e.value.status == mod.RSF_ERR_INVALID_ARG
        with pytest.raises(mod.RsfError) as e:
            srv.submit(rq["vol"], rq["phi0"].clone(), rq["params"], -1)
        assert e.value.status == mod.RSF_ERR_INVALID_ARG
        with pytest.raises(mod.RsfError) as e:
            srv.poll(12345)
        assert e.value.status == mod.RSF_ERR_INVALID_ARG
        assert srv.stats()["submitted"] == 0


@pytest.mark.parametrize("order", ["arrival", "shortest"])
def test_server_voxel_cap_schedules(rsf, order):
    """With a per-chunk voxel cap only some resident tiles iterate in each
    chunk (by arrival or by least remaining work); results are unchanged."""
    mod, ctx = rsf
    say(f"server: voxel cap, order {order}")
    reqs = requests(mod, 1000)
    outs = [rq["phi0"].clone() for rq in reqs]
    torch.cuda.synchronize()
    o = mod.RSF_ORDER_ARRIVAL if order == "arrival" else mod.RSF_ORDER_SHORTEST
    with mod.Server(budget_bytes=8 << 30, chunk_iters=3, batch_voxels=150_000, order=o) as srv:
        tickets = [srv.submit(rq["vol"], o_, rq["params"], rq["iters"])
                   for rq, o_ in zip(reqs, outs)]
        results = [srv.wait(t, 120.0) for t in tickets]
    if order == "shortest":
        # the least work (iterations x voxels) finishes first
        work = [rq["iters"] * rq["phi0"].numel() for rq in reqs]
        first = int(np.argmin([r["t_done"] for r in results]))
        assert work[first] == min(work)
    check_equal_alone(ctx, reqs, outs, results)
