"""Iterations replayed from captured HIP graphs, and batches whose update
carries the next stage-1 z pass, through the C ABI.

Both change only how the launches are issued (a graph replays the same
kernel launches with the same arguments; the fused update writes the
stage-1 pair the separate pass would write, in the same tap order), so the
results must be bitwise those of direct, separate launches.  Each graph
replay is checked against the direct result, over several calls in a row
with other device work and synchronisations between them, alternating
shapes so that kept graphs are replaced and replayed again.
"""
import sys

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
    ctx.set_graphs(True)
    ctx.set_fusion(True)
    ctx.close()


def case(shape, seed, sigma=3.0, storage="f32"):
    I = inputs.vessel_phantom(shape, 6, 1.0, 3.0, seed=seed)
    from paper_2404_02813_amd import rsf as mod
    p = mod.make_params(sigma, 1.0, 1.0, 0.001, 1.0, 0.1, 1.0, storage=storage)
    return torch.from_numpy(I).cuda(), torch.from_numpy(inputs.box_phi0(shape)).cuda(), p


def direct(mod, ctx, vol, phi0, p, iters):
    ctx.set_graphs(False)
    out = phi0.clone()
    ctx.evolve_ex(vol, out, p, iters)
    _, run, last, hist = ctx.stats(cap=iters)
    ctx.set_graphs(True)
    torch.cuda.synchronize()
    return out, hist


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_graph_replays_equal_direct_launches(rsf, storage):
    mod, ctx = rsf
    shapes = [((40, 48, 56), 71, 37), ((36, 44, 70), 72, 21), ((40, 48, 56), 71, 37)]
    cases = [case(s, seed, storage=storage) for s, seed, _ in shapes]
    refs = [direct(mod, ctx, v, p0, p, it) for (v, p0, p), (_, _, it) in zip(cases, shapes)]
    scratch = torch.ones(1 << 20, device="cuda")
    for rep in range(3):
        for k, ((vol, phi0, p), (shape, _, iters)) in enumerate(zip(cases, shapes)):
            say(f"graph replay: rep {rep}, {shape} x {iters}, {storage} storage")
            got = phi0.clone()
            ctx.evolve_ex(vol, got, p, iters)
            # other device work and a synchronisation between the calls
            scratch.mul_(1.0001).add_(got.mean())
            _, run, _, hist = ctx.stats(cap=iters)
            torch.cuda.synchronize()
            assert run == iters
            assert torch.equal(got, refs[k][0]), (rep, k)
            assert hist == refs[k][1]


def test_batch_fused_and_graphs_equal_separate_direct(rsf):
    mod, ctx = rsf
    # planes large enough that the tiles' column tiles alone fill the
    # resident update workgroups: the batch fuses
    shapes = [(12, 260, 300), (10, 280, 270), (14, 250, 310)]
    iters = 19
    cases = [case(s, 80 + k) for k, s in enumerate(shapes)]
    vols = [c[0] for c in cases]
    p = cases[0][2]

    def run(fuse, graphs):
        ctx.set_fusion(fuse)
        ctx.set_graphs(graphs)
        phis = [c[1].clone() for c in cases]
        ctx.profile(True)
        ctx.evolve_batch(vols, phis, p, iters)
        ctx.profile(False)
        prof = ctx.profile_read()
        hists = [ctx.tile_stats(t, cap=iters)[3] for t in range(len(shapes))]
        torch.cuda.synchronize()
        return phis, hists, prof

    say("batch: separate passes, direct launches")
    ref, ref_h, prof = run(False, False)
    assert prof["z_heaviside"][0] == iters
    say("batch: fused update (per-pass events on: direct launches)")
    fused, fused_h, prof = run(True, False)
    # the fused update ran: one stage-1 pass for the whole evolution
    assert prof["z_heaviside"][0] == 1 and prof["z_update"][0] == iters
    for a, b in zip(fused, ref):
        assert torch.equal(a, b)
    # the FP64 sums are grouped per update workgroup, and a fused tile is one
    # z chunk: equal up to that grouping
    for a, b in zip(fused_h, ref_h):
        assert a == pytest.approx(b, rel=1e-12, abs=0.0)
    say("batch: fused update replayed from graphs, twice")
    for _ in range(2):
        ctx.set_fusion(True)
        ctx.set_graphs(True)
        phis = [c[1].clone() for c in cases]
        ctx.evolve_batch(vols, phis, p, iters)
        hists = [ctx.tile_stats(t, cap=iters)[3] for t in range(len(shapes))]
        torch.cuda.synchronize()
        for a, b in zip(phis, ref):
            assert torch.equal(a, b)
        assert hists == fused_h
    ctx.set_fusion(True)
    ctx.set_graphs(True)
