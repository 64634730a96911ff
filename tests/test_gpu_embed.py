"""GPU parity of the output-parallel paths: encode variants (reverse
complement, overlapping k-mers), the encode fused with the embedding lookup,
and the lookup of given ids. The HIP library (through its C-ABI) against the
CPU oracle, element by element; embedding rows are compared byte for byte."""
import numpy as np
import pytest

import oracle
import paper_2601_05531_amd as dt
import synth

pytestmark = pytest.mark.gpu

RC, OV = dt.VARIANT_REVCOMP, dt.VARIANT_OVERLAP


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    return torch


def _dev(a):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _ragged(seed, n=400, hi=3000.0):
    """Rows of a decorated order-3 genome (soft-masking, N runs, invalid
    bytes) with log-uniform lengths plus empty rows and rows of 1..16 bases."""
    lens = synth.loguniform_int(synth.substream(70, seed), n, 1, hi)
    lens[::37] = 0
    lens[5::41] = np.arange(1, len(lens[5::41]) + 1) % 17
    data = synth.genome(synth.substream(70, 1000 + seed), synth.substream(70, 2000 + seed), 3, int(lens.sum()))
    return data, synth.offsets_from_lengths(lens)


def _want(kind, data, offs, k, variant, cls, lut=None, cls_id=2, sep_id=3):
    d = oracle.revcomp(data, offs) if variant & RC else data
    if variant & OV:
        return oracle.encode_overlap(d, offs, k, add_cls_sep=cls)
    return oracle.encode(kind, d, offs, k=k, lut=lut, add_cls_sep=cls, cls_id=cls_id, sep_id=sep_id)


LUT_IDS = dict(pad_id=0, cls_id=5, sep_id=6)


def _vocab(kind, k):
    if kind == dt.LUT256:
        return dt.Vocab(dt.LUT256, lut256=oracle.fallback_lut(), **LUT_IDS)
    return dt.Vocab(kind, k=k)


def _oracle_ids(kind, data, offs, k, variant, cls):
    if kind == dt.LUT256:
        return _want(kind, data, offs, k, variant, cls, lut=oracle.fallback_lut(), cls_id=LUT_IDS["cls_id"],
                     sep_id=LUT_IDS["sep_id"])
    return _want(kind, data, offs, k, variant, cls)


# ---------------------------------------------------------------- encode variants

VARIANT_CASES = [
    (dt.SINGLE, 1, RC), (dt.LUT256, 1, RC),
    (dt.KMER, 1, RC), (dt.KMER, 3, RC), (dt.KMER, 6, RC), (dt.KMER, 8, RC), (dt.KMER, 15, RC),
    (dt.KMER, 1, OV), (dt.KMER, 2, OV), (dt.KMER, 6, OV), (dt.KMER, 15, OV),
    (dt.KMER, 6, RC | OV),
]


@pytest.mark.parametrize("kind,k,variant", VARIANT_CASES)
@pytest.mark.parametrize("cls", [False, True])
def test_variant_packed(kind, k, variant, cls):
    torch = _torch()
    data, offs = _ragged(k * 10 + variant)
    print("variant packed kind=%d k=%d variant=%d cls=%d n=%d nbytes=%d" % (kind, k, variant, cls, len(offs) - 1,
                                                                          len(data)), flush=True)
    want_ids, want_off = _oracle_ids(kind, data, offs, k, variant, cls)
    v = _vocab(kind, k)
    ids, out_off, _ = dt.encode(v, _dev(data), _dev(offs), h_offsets=offs, add_cls_sep=cls, variant=variant)
    torch.cuda.synchronize()
    assert dt.sync_status() == 0
    assert np.array_equal(out_off.cpu().numpy(), want_off)
    got = ids.cpu().numpy()
    bad = np.nonzero(got != want_ids)[0]
    assert got.shape == want_ids.shape and bad.size == 0, bad[:5]


@pytest.mark.parametrize("kind,k,variant,side,extra", [
    (dt.SINGLE, 1, RC, dt.PAD_RIGHT, 0), (dt.LUT256, 1, RC, dt.PAD_LEFT, 3),
    (dt.KMER, 4, OV, dt.PAD_RIGHT, 1500), (dt.KMER, 6, RC | OV, dt.PAD_LEFT, 0),
    (dt.KMER, 5, RC, dt.PAD_LEFT, 7),
])
def test_variant_padded(kind, k, variant, side, extra):
    torch = _torch()
    data, offs = _ragged(100 + k)
    print("variant padded kind=%d k=%d variant=%d side=%d extra=%d" % (kind, k, variant, side, extra), flush=True)
    want_ids, want_off = _oracle_ids(kind, data, offs, k, variant, True)
    W = int(np.diff(want_off).max()) + extra
    pad_id = LUT_IDS["pad_id"] if kind == dt.LUT256 else 0
    w_ids, w_mask = oracle.pad(want_ids, want_off, W, side, pad_id)
    v = _vocab(kind, k)
    ids, out_off, mask = dt.encode(v, _dev(data), _dev(offs), h_offsets=offs, add_cls_sep=True, layout=dt.PADDED,
                                   pad_side=side, pad_to=W, variant=variant)
    torch.cuda.synchronize()
    assert dt.sync_status() == 0
    assert np.array_equal(out_off.cpu().numpy(), want_off)
    assert np.array_equal(ids.cpu().numpy(), w_ids)
    assert np.array_equal(mask.cpu().numpy(), w_mask)


def test_variant_rejections():
    _torch()
    data, offs = _ragged(1, n=4)
    d, o = _dev(data), _dev(offs)
    with pytest.raises(dt.DnatokError):
        dt.encode(dt.Vocab(dt.SINGLE), d, o, h_offsets=offs, variant=OV)
    with pytest.raises(dt.DnatokError):
        dt.encode(dt.Vocab(dt.BPE, merges=np.zeros((0, 2), np.int32)), d, o, h_offsets=offs, variant=RC)
    with pytest.raises(dt.DnatokError):
        dt.encode(dt.Vocab(dt.KMER, k=3), d, o, h_offsets=offs, variant=4)


# ---------------------------------------------------------------- fused encode + embedding lookup

def _table(seed, V, D, dtype):
    """A random table and its rows as bytes (uint8 [V, row_bytes])."""
    torch = _torch()
    g = torch.Generator().manual_seed(seed)
    if dtype in (torch.int8, torch.uint8):
        t = torch.randint(-100, 100, (V, D), generator=g).to(dtype)
    else:
        t = torch.randn(V, D, generator=g).to(dtype)
    return t.to("cuda"), t.view(torch.uint8).numpy().reshape(V, -1)


def _emb_bytes(emb):
    torch = _torch()
    return emb.contiguous().view(torch.uint8).cpu().numpy().reshape(emb.shape[:-1] + (-1,))


EMBED_CASES = [
    # kind, k, variant, D, dtype name
    (dt.SINGLE, 1, 0, 128, "bfloat16"),    # 256-byte rows: 16-byte units
    (dt.KMER, 6, 0, 33, "float32"),        # 132-byte rows: 4-byte units
    (dt.KMER, 3, RC, 4, "float16"),        # 8-byte rows
    (dt.KMER, 2, OV, 1, "bfloat16"),       # 2-byte rows
    (dt.LUT256, 1, 0, 3, "int8"),          # 3-byte rows: byte units
]


@pytest.mark.parametrize("kind,k,variant,D,dtn", EMBED_CASES)
@pytest.mark.parametrize("layout,side", [(dt.PACKED, dt.PAD_RIGHT), (dt.PADDED, dt.PAD_LEFT),
                                         (dt.PADDED, dt.PAD_RIGHT)])
def test_embed_parity(kind, k, variant, D, dtn, layout, side):
    torch = _torch()
    data, offs = _ragged(200 + k + D, n=150, hi=2000.0)
    print("embed kind=%d k=%d variant=%d D=%d %s layout=%d side=%d" % (kind, k, variant, D, dtn, layout, side),
          flush=True)
    v = _vocab(kind, k)
    table, rows = _table(k * 1000 + D, v.vocab_size + 3, D, getattr(torch, dtn))
    want_ids, want_off = _oracle_ids(kind, data, offs, k, variant, True)
    emb, out_off, ids, mask = dt.embed(v, _dev(data), _dev(offs), table, h_offsets=offs, add_cls_sep=True,
                                       layout=layout, pad_side=side, variant=variant, want_ids=True)
    torch.cuda.synchronize()
    assert dt.sync_status() == 0
    assert np.array_equal(out_off.cpu().numpy(), want_off)
    if layout == dt.PADDED:
        W = int(np.diff(want_off).max())
        pad_id = LUT_IDS["pad_id"] if kind == dt.LUT256 else 0
        want_ids, w_mask = oracle.pad(want_ids, want_off, W, side, pad_id)
        assert np.array_equal(mask.cpu().numpy(), w_mask)
    assert np.array_equal(ids.cpu().numpy(), want_ids)
    got = _emb_bytes(emb)
    want = oracle.embed(rows, want_ids)
    assert got.shape == want.shape
    bad = np.nonzero((got != want).any(axis=-1).reshape(-1))[0]
    assert bad.size == 0, bad[:5]


def test_embed_misaligned_output_and_guard_rows():
    # an output view starting 2 bytes in (2-byte units), and a PACKED capacity
    # short by 5 rows: DERR_CAPACITY raised, rows past the capacity untouched
    torch = _torch()
    data, offs = _ragged(300, n=60)
    v = dt.Vocab(dt.KMER, k=4)
    table, rows = _table(7, v.vocab_size, 8, torch.bfloat16)
    want_ids, want_off = _want(dt.KMER, data, offs, 4, 0, False)
    total = int(want_off[-1])
    raw = torch.full(((total + 1) * 16 + 2,), 0xAB, dtype=torch.uint8, device="cuda")
    out = raw[2:2 + total * 16]
    out_off = torch.empty(len(offs), dtype=torch.int64, device="cuda")
    opts = dt.make_opts()
    d_data, d_offs = _dev(data), _dev(offs)  # kept alive until the launch has run
    dt.dnatok_embed(v.handle, dt._ptr(d_data), len(data), dt._ptr(d_offs), len(offs) - 1, dt._ptr(table),
                    table.shape[0], 16, dt._ptr(out), total - 5, dt._ptr(out_off), None, None, opts,
                    torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert dt.sync_status() == dt.DERR_CAPACITY
    got = out.cpu().numpy().reshape(total, 16)
    want = oracle.embed(rows, want_ids)
    assert np.array_equal(got[:total - 5], want[:total - 5])
    assert (got[total - 5:] == 0xAB).all()
    r = raw.cpu().numpy()
    assert (r[:2] == 0xAB).all() and (r[2 + total * 16:] == 0xAB).all()


def test_embed_rejections():
    torch = _torch()
    data, offs = _ragged(2, n=4)
    v = dt.Vocab(dt.KMER, k=3)
    small = torch.zeros((v.vocab_size - 1, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(dt.DnatokError):
        dt.embed(v, _dev(data), _dev(offs), small, h_offsets=offs)
    b = dt.Vocab(dt.BPE, merges=np.zeros((0, 2), np.int32))
    with pytest.raises(dt.DnatokError):
        dt.embed(b, _dev(data), _dev(offs), torch.zeros((16, 4), device="cuda"), h_offsets=offs)


# ---------------------------------------------------------------- lookup of given ids

def test_embed_ids_bpe_and_out_of_range():
    torch = _torch()
    corpus = synth.genome(synth.substream(71, 0), synth.substream(71, 1), 3, 100_000)
    merges = oracle.bpe_train(corpus, 200)
    data, offs = _ragged(400, n=120)
    v = dt.Vocab(dt.BPE, merges=merges)
    ids, out_off, _ = dt.encode(v, _dev(data), _dev(offs), h_offsets=offs, add_cls_sep=True)
    table, rows = _table(9, v.vocab_size, 64, torch.bfloat16)
    emb = dt.embed_ids(ids, table)
    torch.cuda.synchronize()
    assert dt.sync_status() == 0
    want_ids, _ = oracle.encode(oracle.BPE, data, offs, merges=merges, add_cls_sep=True)
    assert np.array_equal(_emb_bytes(emb), oracle.embed(rows, want_ids))
    # ids outside the table: zero rows and DERR_IDS
    bad = torch.tensor([0, -1, v.vocab_size, 5, 2 ** 31 - 1], dtype=torch.int32, device="cuda")
    emb = dt.embed_ids(bad, table)
    torch.cuda.synchronize()
    assert dt.sync_status() == dt.DERR_IDS
    got = _emb_bytes(emb)
    assert np.array_equal(got[0], rows[0]) and np.array_equal(got[3], rows[5])
    assert (got[[1, 2, 4]] == 0).all()


# ---------------------------------------------------------------- captured graph of variant encodes

def test_variant_encodes_in_a_graph():
    # reverse-complement and overlapping encodes captured once, replayed over
    # changing input bytes with eager work in between; every replay equals
    # the oracle on the bytes it saw
    torch = _torch()
    data, offs = _ragged(500, n=200)
    d_bytes, d_offs = _dev(data), _dev(offs)
    cases = [(dt.Vocab(dt.KMER, k=6), RC | OV, dt.PADDED), (dt.Vocab(dt.KMER, k=4), RC, dt.PACKED),
             (dt.Vocab(dt.SINGLE), RC, dt.PADDED)]
    calls, outs = [], []
    for v, variant, layout in cases:
        total, W = dt.plan(v, offs, add_cls_sep=True, variant=variant)
        cap = len(offs[:-1]) * W if layout == dt.PADDED else total
        ids = torch.empty(cap, dtype=torch.int32, device="cuda")
        oo = torch.empty(len(offs), dtype=torch.int64, device="cuda")
        mask = torch.empty(cap, dtype=torch.int8, device="cuda") if layout == dt.PADDED else None
        calls.append(dict(vocab=v, d_bytes=d_bytes, d_offsets=d_offs, d_ids=ids, d_out_offsets=oo, d_mask=mask,
                          add_cls_sep=True, layout=layout, pad_to=W if layout == dt.PADDED else 0, variant=variant))
        outs.append((ids, oo, mask, W))
    g = dt.Graph(calls)
    rng = np.random.default_rng(9)
    for rep in range(3):
        cur = data.copy()
        flip = rng.choice(len(cur), 2000, replace=False)
        cur[flip] = np.frombuffer(b"ACGTNacgtn#", np.uint8)[rng.integers(0, 11, 2000)]
        d_bytes.copy_(torch.from_numpy(cur))
        g.launch()
        torch.cuda.synchronize()
        assert dt.sync_status() == 0
        for (v, variant, layout), (ids, oo, mask, W) in zip(cases, outs):
            want_ids, want_off = _want(v.kind, cur, offs, v.k, variant, True)
            assert np.array_equal(oo.cpu().numpy(), want_off)
            if layout == dt.PADDED:
                w_ids, w_mask = oracle.pad(want_ids, want_off, W)
                assert np.array_equal(ids.cpu().numpy().reshape(-1, W), w_ids)
                assert np.array_equal(mask.cpu().numpy().reshape(-1, W), w_mask)
            else:
                assert np.array_equal(ids.cpu().numpy(), want_ids)
        _ = torch.ones(1 << 20, device="cuda").sum().item()  # eager work between replays
    g.close()


# ---------------------------------------------------------------- full-size batch, sampled rows

def test_embed_full_batch_sampled_rows():
    # the 4096 x 8192 batch, single-nucleotide ids with CLS/SEP, left-padded,
    # D = 128 bf16 (the paper's embedding width): 8.6 GB of output. Sampled
    # rows are compared with the oracle run on those rows alone.
    torch = _torch()
    data, offs = synth.workload_markov_batch()
    v = dt.Vocab(dt.SINGLE)
    table, rows = _table(11, 11, 128, torch.bfloat16)
    print("embed full batch n=%d nbytes=%d" % (len(offs) - 1, len(data)), flush=True)
    emb, out_off, _, mask = dt.embed(v, _dev(data), _dev(offs), table, h_offsets=offs, add_cls_sep=True,
                                     layout=dt.PADDED, pad_side=dt.PAD_LEFT)
    torch.cuda.synchronize()
    assert dt.sync_status() == 0
    rng = np.random.default_rng(5)
    sample = np.concatenate([[0, len(offs) - 2], rng.choice(len(offs) - 1, 10, replace=False)])
    for r in sample:
        row = data[offs[r]:offs[r + 1]]
        ids, _ = oracle.encode(oracle.SINGLE, row, np.array([0, len(row)]), add_cls_sep=True)
        assert np.array_equal(_emb_bytes(emb[r]), oracle.embed(rows, ids))
        assert (mask[r].cpu().numpy() == 1).all()
    del emb


def test_full_batch_lookups_back_to_back():
    # two lookups in a row on the full batch (33.5M cells) with 2-byte rows,
    # reverse complement and right padding in the second; every cell is
    # compared with the oracle
    torch = _torch()
    data, offs = synth.workload_markov_batch()
    d_data, d_offs = _dev(data), _dev(offs)
    table, rows = _table(13, 11, 1, torch.bfloat16)
    v = dt.Vocab(dt.SINGLE)
    for variant, side in ((0, dt.PAD_LEFT), (RC, dt.PAD_RIGHT)):
        print("full-batch lookup variant=%d side=%d" % (variant, side), flush=True)
        emb, out_off, _, mask = dt.embed(v, d_data, d_offs, table, h_offsets=offs, add_cls_sep=True,
                                         layout=dt.PADDED, pad_side=side, variant=variant)
        torch.cuda.synchronize()
        assert dt.sync_status() == 0
        want_ids, want_off = _want(dt.SINGLE, data, offs, 1, variant, True)
        w_ids, w_mask = oracle.pad(want_ids, want_off, int(np.diff(want_off).max()), side)
        assert np.array_equal(_emb_bytes(emb), oracle.embed(rows, w_ids))
        assert np.array_equal(mask.cpu().numpy(), w_mask)
        del emb


def test_overlap_full_batch_sampled_rows():
    torch = _torch()
    data, offs = synth.workload_markov_batch()
    v = dt.Vocab(dt.KMER, k=6)
    print("overlap full batch", flush=True)
    ids, out_off, mask = dt.encode(v, _dev(data), _dev(offs), h_offsets=offs, add_cls_sep=True, layout=dt.PADDED,
                                   variant=OV | RC)
    torch.cuda.synchronize()
    assert dt.sync_status() == 0
    assert ids.shape == (4096, 8192 - 6 + 1 + 2)
    rng = np.random.default_rng(6)
    for r in np.concatenate([[0, 4095], rng.choice(4096, 10, replace=False)]):
        row = data[offs[r]:offs[r + 1]]
        o = np.array([0, len(row)])
        want, _ = oracle.encode_overlap(oracle.revcomp(row, o), o, 6, add_cls_sep=True)
        assert np.array_equal(ids[r].cpu().numpy(), want)


# ---------------------------------------------------------------- edge cases

def test_empty_batches_and_empty_rows():
    torch = _torch()
    v = dt.Vocab(dt.KMER, k=5)
    table, rows = _table(3, v.vocab_size, 8, torch.float32)
    # no rows at all
    offs = np.zeros(1, np.int64)
    d = torch.zeros(16, dtype=torch.uint8, device="cuda")
    for layout in (dt.PACKED, dt.PADDED):
        emb, oo, _, _ = dt.embed(v, d[:0], _dev(offs), table, h_offsets=offs, layout=layout, pad_to=4)
        ids, oo2, _ = dt.encode(v, d[:0], _dev(offs), h_offsets=offs, layout=layout, pad_to=4, variant=RC | OV)
        torch.cuda.synchronize()
        assert dt.sync_status() == 0
        assert oo.cpu().tolist() == [0] and oo2.cpu().tolist() == [0]
    # only empty rows, with and without CLS/SEP
    offs = np.zeros(9, np.int64)
    for cls in (False, True):
        emb, oo, ids, mask = dt.embed(v, d[:0], _dev(offs), table, h_offsets=offs, add_cls_sep=cls,
                                      layout=dt.PADDED, pad_to=3, want_ids=True)
        torch.cuda.synchronize()
        assert dt.sync_status() == 0
        want = [[2, 3, 0] if cls else [0, 0, 0]] * 8
        assert ids.cpu().numpy().tolist() == want
        assert np.array_equal(_emb_bytes(emb), oracle.embed(rows, np.array(want)))


def test_bad_offsets_raise_the_flag_and_stay_in_bounds():
    # decreasing and out-of-range offsets: each row is clamped on its own as
    # the row scan clamps it (start into [0, nbytes], end into [start,
    # nbytes]), DERR_OFFSETS is raised, and nothing is written past the outputs
    torch = _torch()
    data = synth.genome(synth.substream(72, 0), synth.substream(72, 1), 3, 1000)
    nbytes = len(data)
    offs = np.array([0, 100, 50, 300, nbytes + 50, nbytes], np.int64)
    n = len(offs) - 1
    rows = []
    for i in range(n):
        o0 = min(max(int(offs[i]), 0), nbytes)
        o1 = min(max(int(offs[i + 1]), o0), nbytes)
        rows.append(data[o0:o1])
    assert [len(r) for r in rows] == [100, 0, 250, nbytes - 300, 0]
    per_row = [oracle.encode_overlap(r, np.array([0, len(r)]), 3, add_cls_sep=True)[0] for r in rows]
    want_off = np.concatenate([[0], np.cumsum([len(x) for x in per_row])])
    W = max(len(x) for x in per_row)
    v = dt.Vocab(dt.KMER, k=3)
    guard = 64
    ids = torch.full((n * W + guard,), -7, dtype=torch.int32, device="cuda")
    mask = torch.full((n * W + guard,), -7, dtype=torch.int8, device="cuda")
    oo = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    d_data, d_offs = _dev(data), _dev(offs)
    opts = dt.make_opts(True, dt.PADDED, dt.PAD_RIGHT, W, variant=OV)
    dt.dnatok_encode(v.handle, dt._ptr(d_data), nbytes, dt._ptr(d_offs), n, dt._ptr(ids), n * W, dt._ptr(oo),
                     dt._ptr(mask), opts, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert dt.sync_status() & dt.DERR_OFFSETS
    assert np.array_equal(oo.cpu().numpy(), want_off)
    got = ids.cpu().numpy()
    for i, x in enumerate(per_row):
        assert np.array_equal(got[i * W:i * W + len(x)], x)
        assert (got[i * W + len(x):(i + 1) * W] == 0).all()
    assert (got[n * W:] == -7).all() and (mask.cpu().numpy()[n * W:] == -7).all()
