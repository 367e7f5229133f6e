"""The entry point that allocates nothing (ss_filter_ascii_noalloc) against the one it mirrors
(ss_filter_ascii_async, automatic tile), through the C ABI: two calls in a row on each schedule, the
second with a smaller batch, every result word equal (and equal to the oracle's)."""
import numpy as np
import pytest

import oracle
from paper_1910_09020_amd import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_09020_amd as ss
    from paper_1910_09020_amd import runner
    ss.lib()
    return torch, ss, runner


def _device(torch, b, off=0):
    d = torch.device("cuda")
    total = int(b["reads"].size)
    rd = torch.full((total + 64,), ord("A"), dtype=torch.uint8, device=d)
    rf = torch.full((total + 64,), ord("A"), dtype=torch.uint8, device=d)
    rd[off:off + total].copy_(torch.from_numpy(b["reads"]))
    rf[off:off + total].copy_(torch.from_numpy(b["refs"]))
    return rd[off:], rf[off:]


@pytest.mark.parametrize("m,E,n1,n2,off", [
    (100, 11, 1_500_007, 60_013, 0),    # two kernels over scratch chunks (several chunks, then one)
    (100, 3, 400_000, 5_000, 0),        # fused kernel, no scratch
    (100, 8, 300_000, 4_001, 0),        # fused kernel above E = 5 (four count digits)
    (250, 4, 300_001, 20_000, 0),       # aligned 250 bp: the chunked schedule
    (100, 5, 200_000, 33, 1),           # unaligned inputs: the fused kernel
])
def test_noalloc_matches_async(rt, m, E, n1, n2, off):
    torch, ss, runner = rt
    ctx = runner.context()
    st = torch.cuda.current_stream()
    d = torch.device("cuda")
    for n in (n1, n2):
        b = gen.long_pairs(n, m, 0, 800, seed=1910090207 + n)
        rd, rf = _device(torch, b, off)
        err = torch.zeros(1, dtype=torch.int32, device=d)
        want = torch.empty(n + 8, dtype=torch.int16, device=d)
        got = torch.full((n + 8,), -1, dtype=torch.int16, device=d)
        print(f"  m={m} E={E} n={n} off={off}", flush=True)
        ss.ss_filter_ascii_async(ctx, rd, rf, n, m, E, 0, want, err, st)
        ss.ss_filter_ascii_noalloc(ctx, rd, rf, n, m, E, got, err, st)
        torch.cuda.synchronize()
        assert int(err.item()) == 0
        assert torch.equal(got[:n], want[:n]), f"m={m} E={E} n={n}"
        if n <= 100_000:
            w = oracle.batch(b["reads"], b["refs"], b["offsets"], b["lengths"], E=E, threads=8)
            acc, ed = runner.results_numpy(got, n)
            assert np.array_equal(acc, w["accept"]) and np.array_equal(ed, w["edits"])


def test_noalloc_limits(rt):
    torch, ss, runner = rt
    ctx = runner.context()
    L = ss.lib()
    d = torch.device("cuda")
    x = torch.empty(64, dtype=torch.uint8, device=d)
    out = torch.empty(64, dtype=torch.int16, device=d)
    assert L.ss_filter_ascii_noalloc(ctx, x.data_ptr(), x.data_ptr(), 1, ss.SS_MAX_LEN_FUSED + 1, 3,
                                     out.data_ptr(), None, None) == ss.SS_ELEN
    assert L.ss_filter_ascii_noalloc(ctx, x.data_ptr(), x.data_ptr(), 1, 10, ss.SS_MAX_E_SLICED + 1,
                                     out.data_ptr(), None, None) == ss.SS_ELEN
    assert L.ss_filter_ascii_noalloc(ctx, x.data_ptr(), x.data_ptr(), 0, 10, 3, out.data_ptr(), None, None) == ss.SS_OK
