"""Allocation failures forced from the host (rsf_set_fault) on every path
that allocates: each allocation the call attempts is made to fail in turn.
The call then returns RSF_ERR_OUT_OF_MEMORY having made exactly that many
attempts, leaves the caller's phi untouched, and the context or server stays
usable: the same call once the fault is disarmed gives bitwise the result of
a run that never failed.  No kernel sees a failed allocation: the failure is
reported before anything is launched on the buffer."""
import sys

import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2404_02813_amd import inputs  # noqa: E402


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2404_02813_amd import rsf as m
    m.rsf_set_fault(None)
    yield m
    torch.cuda.synchronize()
    m.rsf_set_fault(None)


P = dict(sigma=2.0, lambda1=1.0, lambda2=1.0, nu=0.001, mu=1.0, dt=0.1, eps=1.0)
NEVER = "alloc_fail:1000000000"     # armed only to count the attempts


def case(shape, seed):
    I = inputs.vessel_phantom(shape, 5, 1.0, 3.0, seed=seed)
    return torch.from_numpy(I).cuda(), torch.from_numpy(inputs.box_phi0(shape)).cuda()


def attempts_of(mod, run):
    """Allocation attempts one clean call makes (on a fresh context)."""
    mod.rsf_set_fault(NEVER)
    try:
        run()
        torch.cuda.synchronize()
        return mod.rsf_fault_allocations()
    finally:
        mod.rsf_set_fault(None)


def fail_each_attempt(mod, n_attempts, call, phi, phi0, want):
    """For every attempt k: a fresh context whose call fails at attempt k,
    then succeeds on the same context once disarmed."""
    for k in range(1, n_attempts + 1):
        say(f"  allocation {k} of {n_attempts} fails")
        ctx = mod.Context(0)
        try:
            phi.copy_(phi0)
            torch.cuda.synchronize()
            mod.rsf_set_fault(f"alloc_fail:{k}")
            try:
                with pytest.raises(mod.RsfError) as e:
                    call(ctx)
                torch.cuda.synchronize()
                assert e.value.status == mod.RSF_ERR_OUT_OF_MEMORY, (k, str(e.value))
                assert mod.rsf_fault_allocations() == k
            finally:
                mod.rsf_set_fault(None)
            assert torch.equal(phi, phi0), k
            call(ctx)
            torch.cuda.synchronize()
            assert torch.equal(phi, want), k
        finally:
            ctx.close()


def test_evolve_allocation_failures(mod):
    say("evolve_ex: each allocation fails in turn")
    vol, phi0 = case((24, 40, 44), 61)
    params = mod.make_params(**P)
    want = phi0.clone()
    probe = mod.Context(0)
    try:
        n = attempts_of(mod, lambda: probe.evolve_ex(vol, want, params, 6))
    finally:
        probe.close()
    assert n >= 2          # the workspace and the pinned table staging
    phi = phi0.clone()
    fail_each_attempt(mod, n, lambda c: c.evolve_ex(vol, phi, params, 6), phi, phi0, want)


def test_volume_driver_allocation_failures(mod):
    say("evolve_volume: each allocation fails in turn")
    vol, phi0 = case((30, 36, 40), 62)
    params = mod.make_params(**P)
    want = phi0.clone()
    probe = mod.Context(0)
    try:
        n = attempts_of(mod, lambda: probe.evolve_volume(vol, want, params, 4, 16, 2))
    finally:
        probe.close()
    assert n >= 4          # accumulator, copies, workspace, staging
    phi = phi0.clone()
    fail_each_attempt(mod, n, lambda c: c.evolve_volume(vol, phi, params, 4, 16, 2), phi,
                      phi0, want)


def test_init_phi_allocation_failures(mod):
    say("init_phi: each allocation fails in turn")
    I = inputs.vessel_phantom((10, 40, 48), 8, 1.0, 3.0, seed=63)
    vol = torch.from_numpy(I).cuda()
    phi0 = torch.full(I.shape, 5.0, dtype=torch.float32, device="cuda")
    want = phi0.clone()
    probe = mod.Context(0)
    try:
        n = attempts_of(mod, lambda: probe.init_phi(vol, want, 2.0, 0.05, 1.0, 2))
    finally:
        probe.close()
    assert n == 8          # mask, distance, three fields, two reductions, the maximum
    phi = phi0.clone()
    fail_each_attempt(mod, n, lambda c: c.init_phi(vol, phi, 2.0, 0.05, 1.0, 2), phi, phi0,
                      want)


def test_autotune_allocation_failures(mod):
    say("autotune: its first allocations fail in turn")
    shapes = [(20, 36, 40), (16, 30, 34)]
    cases = [case(s, 64 + k) for k, s in enumerate(shapes)]
    vols = [c[0] for c in cases]
    params = mod.make_params(**P)
    ref = [c[1].clone() for c in cases]
    ctx = mod.Context(0)
    try:
        ctx.evolve_batch(vols, ref, params, 5)
        torch.cuda.synchronize()
    finally:
        ctx.close()
    for k in (1, 2, 3):
        say(f"  allocation {k} fails")
        ctx = mod.Context(0)
        try:
            phis = [c[1].clone() for c in cases]
            torch.cuda.synchronize()
            mod.rsf_set_fault(f"alloc_fail:{k}")
            try:
                with pytest.raises(mod.RsfError) as e:
                    ctx.autotune(vols, phis, params, trial_iters=1)
                torch.cuda.synchronize()
                assert e.value.status == mod.RSF_ERR_OUT_OF_MEMORY
            finally:
                mod.rsf_set_fault(None)
            for p, c in zip(phis, cases):
                assert torch.equal(p, c[1])
            ctx.evolve_batch(vols, phis, params, 5)
            torch.cuda.synchronize()
            for p, r in zip(phis, ref):
                assert torch.equal(p, r)
        finally:
            ctx.close()


def test_server_request_fails_then_server_serves(mod):
    say("server: a request whose arena cannot grow fails; the next one runs")
    vol, phi0 = case((22, 30, 34), 66)
    params = mod.make_params(**P)
    ctx = mod.Context(0)
    want = phi0.clone()
    try:
        ctx.evolve_ex(vol, want, params, 5)
        torch.cuda.synchronize()
    finally:
        ctx.close()
    with mod.Server(budget_bytes=1 << 30, chunk_iters=2) as srv:
        a, b = phi0.clone(), phi0.clone()
        torch.cuda.synchronize()
        mod.rsf_set_fault("alloc_fail:1")
        try:
            r = srv.wait(srv.submit(vol, a, params, 5), 120.0)
            assert r["status"] == mod.RSF_ERR_OUT_OF_MEMORY
            assert mod.rsf_fault_allocations() == 1
        finally:
            mod.rsf_set_fault(None)
        assert torch.equal(a, phi0)
        r = srv.wait(srv.submit(vol, b, params, 5), 120.0)
        assert r["status"] == 0
        torch.cuda.synchronize()
        assert torch.equal(b, want)


def test_server_restarts_its_arena_after_a_failed_growth(mod):
    """A request that needs a larger segment than the arena holds, when that
    growth fails and nothing is resident: the server frees its segments and
    grows again, and the request completes."""
    say("server: failed growth, arena restarted, request completes")
    small_vol, small_phi0 = case((12, 20, 24), 67)
    vol, phi0 = case((26, 40, 44), 68)
    params = mod.make_params(**P)
    ctx = mod.Context(0)
    want = phi0.clone()
    try:
        ctx.evolve_ex(vol, want, params, 5)
        torch.cuda.synchronize()
    finally:
        ctx.close()
    with mod.Server(budget_bytes=1 << 30, chunk_iters=2, segment_bytes=1 << 18) as srv:
        s = small_phi0.clone()
        assert srv.wait(srv.submit(small_vol, s, params, 3), 120.0)["status"] == 0
        assert srv.stats()["bytes_reserved"] < mod.rsf_workspace_bytes(44, 40, 26, 5)
        b = phi0.clone()
        torch.cuda.synchronize()
        mod.rsf_set_fault("alloc_fail:1")
        try:
            r = srv.wait(srv.submit(vol, b, params, 5), 120.0)
            assert mod.rsf_fault_allocations() == 2     # the failed growth, then the new one
        finally:
            mod.rsf_set_fault(None)
        assert r["status"] == 0
        torch.cuda.synchronize()
        assert torch.equal(b, want)
