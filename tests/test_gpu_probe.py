"""The random-row bandwidth probe (rs_probe_rows) touches exactly the rows
its hash names, in bounds, and rejects malformed arguments. Its row index
hash is recomputed here from the SplitMix64 finalizer."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

M64 = (1 << 64) - 1


def mix64(x):
    x ^= x >> 30
    x = (x * 0xBF58476D1CE4E5B9) & M64
    x ^= x >> 27
    x = (x * 0x94D049BB133111EB) & M64
    return x ^ (x >> 31)


def probe_row(w, s, g, n_rows):
    return mix64((w << 32) ^ (s << 8) ^ g ^ 0x9E3779B97F4A7C15) & (n_rows - 1)


@pytest.fixture(scope="module")
def lib():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2010_08423_amd as R

    return R, torch


def test_probe_reads_the_hashed_rows(lib):
    R, torch = lib
    n_rows, waves, steps = 1 << 16, 8, 3
    val = (torch.arange(n_rows, dtype=torch.int64, device="cuda") * 7919 + 11)
    rows = val.repeat_interleave(64).view(n_rows, 64).contiguous()
    out = torch.empty((waves, 64), dtype=torch.int64, device="cuda")
    R.probe_rows(rows, out, waves, steps, 0)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for w in range(waves):
        want = 0
        for s in range(steps):
            for g in range(16):
                want ^= probe_row(w, s, g, n_rows) * 7919 + 11
        assert all(int(np.uint64(x)) == want for x in got[w].view(np.uint64)), w


def test_probe_writes_the_hashed_rows(lib):
    R, torch = lib
    n_rows, waves, steps = 1 << 20, 8, 1
    rows = torch.full((n_rows, 64), -1, dtype=torch.int64, device="cuda")
    out = torch.empty((waves, 64), dtype=torch.int64, device="cuda")
    R.probe_rows(rows, out, waves, steps, 1)
    torch.cuda.synchronize()
    hits = {}
    for w in range(waves):
        for g in range(16):
            hits.setdefault(probe_row(w, 0, 64 + g, n_rows), []).append(g)
    host = rows.cpu().numpy()
    for r, gs in hits.items():
        if len(gs) == 1:  # a row written by one wave holds its value in every lane
            assert (host[r] == gs[0]).all(), r
    untouched = np.ones(n_rows, bool)
    untouched[list(hits)] = False
    assert (host[untouched] == -1).all()
    assert (out.cpu().numpy() == 0).all()


def test_probe_rejects_bad_arguments(lib):
    R, torch = lib
    rows = torch.zeros((3, 64), dtype=torch.int64, device="cuda")
    out = torch.empty((8, 64), dtype=torch.int64, device="cuda")
    with pytest.raises(R.RSError):
        R.probe_rows(rows, out, 8, 1, 0)  # 3 rows: not a power of two
    rows = torch.zeros((4, 64), dtype=torch.int64, device="cuda")
    with pytest.raises(R.RSError):
        R.probe_rows(rows, out, 6, 1, 0)  # 6 waves: not a multiple of 4
    with pytest.raises(R.RSError):
        R.probe_rows(rows, out, 8, 1, 3)  # no mode 3
