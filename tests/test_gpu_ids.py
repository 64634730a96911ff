"""GPU parity of the IDs path (host map -> staged int32/int64 ids -> device
widen -> embedding lookup), every id and every output row against the
oracle's table encode, left-padded, and its embedding lookup, for both
staging widths, sequential and pipelined, over several micro-batches with
a ragged last one."""
import numpy as np
import pytest

import oracle
import paper_2601_05531_amd as dt
import synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    return torch


def _want_ids(lut, pad_id, rows, T):
    n, L = rows.shape
    offs = np.arange(n + 1, dtype=np.int64) * L
    ids, oo = oracle.encode(oracle.LUT256, rows.reshape(-1), offs, lut=lut)
    w, _ = oracle.pad(ids, oo, T, oracle.LEFT, pad_id)
    return w.astype(np.int64)


def _rows(n, L, seed):
    data = synth.genome(synth.substream(98, seed), synth.substream(99, seed), 3, n * L)
    return data.reshape(n, L).copy()


@pytest.mark.parametrize("width", [4, 8])
@pytest.mark.parametrize("overlap", [False, True])
@pytest.mark.parametrize("kind", ["fallback_lut256", "single"])
def test_ids_path_equals_oracle(width, overlap, kind):
    torch = _torch()
    if kind == "single":
        v = dt.Vocab(dt.SINGLE)
        lut = np.full(256, 1, np.int32)
        for j, c in enumerate("ACGT"):
            lut[ord(c)] = lut[ord(c.lower())] = 5 + j
        lut[ord("N")] = lut[ord("n")] = 9
        pad_id = 0
    else:
        lut = oracle.fallback_lut()
        v = dt.Vocab(dt.LUT256, lut256=lut, pad_id=0)
        pad_id = 0
    n, L, T = 333, 500, 512
    rows = _rows(n, L, 1)
    g = torch.Generator().manual_seed(3)
    table = torch.randn((16, 128), generator=g).to(torch.bfloat16)
    d_table = table.cuda()
    # a budget of 40 rows of T' ids: 9 micro-batches, the last one ragged
    p = dt.IdsPath(v, width=width, overlap=overlap, threads=4, token_budget=40 * T + 7)
    for rep in range(2):  # the second run reuses the staging and ping-pong buffers
        d_ids = torch.full((n, T), -5, dtype=torch.int64, device="cuda")
        d_out = torch.empty((n, T, 128), dtype=torch.bfloat16, device="cuda")
        r = p.run(rows, n, L, T, d_ids=d_ids, table=d_table, d_out=d_out)
        torch.cuda.synchronize()
        assert dt.sync_status() == 0
        assert r.micro_rows == 40 and r.n_micro == 9 and r.h2d_bytes == n * T * width
        want = _want_ids(lut, pad_id, rows, T)
        assert np.array_equal(d_ids.cpu().numpy(), want)
        emb = oracle.embed(table.view(torch.int16).numpy(), want)
        assert np.array_equal(d_out.view(torch.int16).cpu().numpy(), emb)
    # embedder only (ids kept in the ping-pong buffers), T' = L
    d_out = torch.empty((n, L, 128), dtype=torch.bfloat16, device="cuda")
    p.run(rows, n, L, 0, table=d_table, d_out=d_out)
    torch.cuda.synchronize()
    assert dt.sync_status() == 0
    emb = oracle.embed(table.view(torch.int16).numpy(), _want_ids(lut, pad_id, rows, L))
    assert np.array_equal(d_out.view(torch.int16).cpu().numpy(), emb)
    p.close()
    v.close()


def test_ids_path_edge_cases():
    torch = _torch()
    lut = oracle.fallback_lut()
    v = dt.Vocab(dt.LUT256, lut256=lut)
    p = dt.IdsPath(v, width=4, overlap=True, token_budget=1)  # budget below one row: one row per micro-batch
    rows = _rows(5, 37, 2)
    d_ids = torch.empty((5, 41), dtype=torch.int64, device="cuda")
    r = p.run(rows, 5, 37, 41, d_ids=d_ids)
    assert r.micro_rows == 1 and r.n_micro == 5
    assert np.array_equal(d_ids.cpu().numpy(), _want_ids(lut, 0, rows, 41))
    # odd offsets into the caller's ids: unaligned widen stores
    d_ids = torch.empty((3, 7), dtype=torch.int64, device="cuda")
    r = p.run(_rows(3, 7, 3), 3, 7, 7, d_ids=d_ids)
    assert np.array_equal(d_ids.cpu().numpy(), _want_ids(lut, 0, _rows(3, 7, 3), 7))
    r = p.run(np.zeros(0, np.uint8), 0, 10, 10, d_ids=d_ids)
    assert r.n_micro == 0
    with pytest.raises(dt.DnatokError):
        p.run(rows, 5, 37, 36, d_ids=d_ids)  # token_len < row length
    with pytest.raises(dt.DnatokError):
        p.run(rows, 5, 37, 37)  # no output
    # ids outside the table raise the device flag
    small = torch.zeros((2, 8), dtype=torch.float32, device="cuda")
    d_out = torch.empty((5, 37, 8), dtype=torch.float32, device="cuda")
    p.run(rows, 5, 37, 37, table=small, d_out=d_out)
    assert dt.sync_status() == dt.DERR_IDS
    p.close()
    with pytest.raises(dt.DnatokError) as e:
        dt.IdsPath(dt.Vocab(dt.KMER, k=3))
    assert e.value.code == dt.EVOCAB
    v.close()


@pytest.mark.parametrize("B,T", [(4096, 512), (8192, 512), (2048, 2048)])
@pytest.mark.parametrize("width,overlap", [(4, True), (8, False)])
def test_ids_path_benchmark_shapes(B, T, width, overlap):
    """The benchmark's three shapes with the paper's token budget (1,048,576
    ids per micro-batch) and the single-nucleotide table: every id against
    the oracle, and the embedding rows of the first and last micro-batch."""
    torch = _torch()
    v = dt.Vocab(dt.SINGLE)
    lut = np.full(256, 1, np.int32)
    for j, c in enumerate("ACGT"):
        lut[ord(c)] = lut[ord(c.lower())] = 5 + j
    lut[ord("N")] = lut[ord("n")] = 9
    rows = _rows(B, T, 2)
    g = torch.Generator().manual_seed(4)
    table = torch.randn((11, 128), generator=g).to(torch.bfloat16)
    p = dt.IdsPath(v, width=width, overlap=overlap, threads=16, token_budget=0)
    d_ids = torch.full((B, T), -5, dtype=torch.int64, device="cuda")
    r = p.run(rows, B, T, T, d_ids=d_ids)
    torch.cuda.synchronize()
    assert dt.sync_status() == 0
    b = (1 << 20) // T
    assert r.micro_rows == b and r.n_micro == (B + b - 1) // b
    want = _want_ids(lut, 0, rows, T)
    assert np.array_equal(d_ids.cpu().numpy(), want)
    # the embedder over the first and the last micro-batch's rows
    for lo in (0, (r.n_micro - 1) * b):
        part = rows[lo:lo + b]
        d_out = torch.empty((len(part), T, 128), dtype=torch.bfloat16, device="cuda")
        p.run(np.ascontiguousarray(part), len(part), T, T, table=table.cuda(), d_out=d_out)
        torch.cuda.synchronize()
        assert dt.sync_status() == 0
        emb = oracle.embed(table.view(torch.int16).numpy(), want[lo:lo + b])
        assert np.array_equal(d_out.view(torch.int16).cpu().numpy(), emb)
    p.close()
    v.close()
