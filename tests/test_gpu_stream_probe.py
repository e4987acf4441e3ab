"""The streaming kernel bench.py measures the achievable bandwidth with: each
read/write mix computes out_j = j + sum_k in_k exactly (small sums of
integers), including a length that leaves a partial last span, and bad
arguments are refused."""
import sys

import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("n", [4096, 1 << 20, (1 << 20) + 1028])
@pytest.mark.parametrize("mix", [(1, 1), (2, 2), (3, 2), (4, 3), (4, 1)])
def test_stream_probe_sums(n, mix):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2404_02813_amd import rsf
    r, w = mix
    say(f"stream probe {r} reads, {w} writes, n = {n}")
    inp = torch.arange(r * n, device="cuda", dtype=torch.float32).remainder_(97)
    out = torch.full((w * n,), -1.0, device="cuda")
    rsf.rsf_stream_probe(inp, r, out, w)
    torch.cuda.synchronize()
    want = inp.view(r, n).sum(0)
    for j in range(w):
        assert torch.equal(out.view(w, n)[j], want + j)


def test_stream_probe_refuses_bad_arguments():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2404_02813_amd import rsf
    inp = torch.ones(4 * 1024, device="cuda")
    out = torch.ones(3 * 1024, device="cuda")
    L = rsf.lib()
    s = torch.cuda.current_stream().cuda_stream
    assert L.rsf_stream_probe(inp.data_ptr(), 5, out.data_ptr(), 1, 1024, s) == rsf.RSF_ERR_INVALID_ARG
    assert L.rsf_stream_probe(inp.data_ptr(), 1, out.data_ptr(), 4, 1024, s) == rsf.RSF_ERR_INVALID_ARG
    assert L.rsf_stream_probe(inp.data_ptr(), 1, out.data_ptr(), 1, 1022, s) == rsf.RSF_ERR_INVALID_ARG
    assert L.rsf_stream_probe(inp.data_ptr() + 4, 1, out.data_ptr(), 1, 1024, s) == rsf.RSF_ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert bool((out == 1).all().item())
