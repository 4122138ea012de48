"""The bandwidth references behind the measurements (chfpe_stream_copy,
chfpe_stream_mix): exact results on sizes with a ragged tail (not a
multiple of the grid's stride).  They are plain
streaming kernels, so their results are fixed by definition (a copy, a sum
of up to three arrays, zeros)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2509_25840_amd as pk
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch, pk


@pytest.mark.parametrize("n", [2, 2 * 1000 + 2, 2 * 256 * 8 * 3 + 6, 2 * 1_000_003])
def test_stream_copy_and_mix_are_exact(env, n):
    torch, pk = env
    print(f"[stream] n={n} doubles", flush=True)
    sys.stdout.flush()
    g = torch.Generator().manual_seed(n)
    srcs = [torch.randn(n, dtype=torch.float64, generator=g).cuda() for _ in range(3)]
    dst = torch.full((n,), 7.0, dtype=torch.float64, device="cuda")
    pk.stream_copy(dst, srcs[0], 8 * n)
    torch.cuda.synchronize()
    assert torch.equal(dst, srcs[0])
    for ns in range(4):
        dst.fill_(7.0)
        pk.stream_mix(dst, srcs[:ns], 8 * n)
        torch.cuda.synchronize()
        ref = np.zeros(n)
        for t in srcs[:ns]:
            ref = ref + t.cpu().numpy()  # the kernel adds the sources in this order
        assert np.array_equal(dst.cpu().numpy(), ref), ns
