"""GPU parity of encode/decode: the HIP library (through its C-ABI) against the
CPU oracle, element by element, bit-exact (integer work)."""
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


def _dev(a):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _vocab(kind, k=1, lut=None, merges=None, **kw):
    return dt.Vocab(kind, k=k, lut256=lut, merges=merges, **kw)


def _oracle(kind, data, offs, k=1, lut=None, merges=None, cls=False, cls_id=2, sep_id=3):
    return oracle.encode(kind, data, offs, k=k, lut=lut, merges=merges, add_cls_sep=cls, cls_id=cls_id,
                         sep_id=sep_id)


def check_packed(v, data, offs, cls, k=1, lut=None, merges=None, cls_id=2, sep_id=3, byte_shift=0):
    torch = _torch()
    print("packed kind=%d k=%d n=%d nbytes=%d cls=%d shift=%d" % (v.kind, k, len(offs) - 1, len(data), cls,
                                                                 byte_shift), flush=True)
    want_ids, want_off = _oracle(v.kind, data, offs, k, lut, merges, cls, cls_id, sep_id)
    buf = np.zeros(len(data) + 16, np.uint8)
    buf[byte_shift:byte_shift + len(data)] = data
    d_buf = _dev(buf)
    d_bytes = d_buf[byte_shift:byte_shift + len(data)]
    ids, out_off, _ = dt.encode(v, d_bytes, _dev(offs), h_offsets=offs, add_cls_sep=cls)
    torch.cuda.synchronize()
    assert dt.sync_status() == 0
    assert np.array_equal(out_off.cpu().numpy(), want_off)
    got = ids.cpu().numpy()
    assert got.shape == want_ids.shape
    bad = np.nonzero(got != want_ids)[0]
    assert bad.size == 0, "first mismatch at %d: got %d want %d" % (bad[0], got[bad[0]], want_ids[bad[0]])


def check_padded(v, data, offs, cls, side, k=1, lut=None, pad_extra=0, pad_id=0, cls_id=2, sep_id=3):
    torch = _torch()
    print("padded kind=%d k=%d n=%d side=%d cls=%d extra=%d" % (v.kind, k, len(offs) - 1, side, cls, pad_extra),
          flush=True)
    want_ids, want_off = _oracle(v.kind, data, offs, k, lut, None, cls, cls_id, sep_id)
    W = int(np.diff(want_off).max(initial=0)) + pad_extra
    W = max(W, 1)
    w_ids, w_mask = oracle.pad(want_ids, want_off, W, side, pad_id)
    ids, out_off, mask = dt.encode(v, _dev(data), _dev(offs), h_offsets=offs, add_cls_sep=cls, layout=dt.PADDED,
                                   pad_side=side, pad_to=W)
    torch.cuda.synchronize()
    assert dt.sync_status() == 0
    assert np.array_equal(out_off.cpu().numpy(), want_off)
    assert np.array_equal(ids.cpu().numpy(), w_ids)
    assert np.array_equal(mask.cpu().numpy(), w_mask)


# ---------------------------------------------------------------- small workload (1 Mbase)

@pytest.mark.parametrize("cls", [False, True])
def test_iid_batch_single_and_6mer(cls):
    data, offs = synth.workload_iid()
    check_packed(_vocab(dt.SINGLE), data, offs, cls)
    check_packed(_vocab(dt.KMER, 6), data, offs, cls, k=6)


# ---------------------------------------------------------------- batched k-mer workload at full size

@pytest.fixture(scope="module")
def markov_batch():
    return synth.workload_markov_batch()


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_markov_batch_padded_full_size(markov_batch, k):
    data, offs = markov_batch
    check_padded(_vocab(dt.KMER, k), data, offs, True, dt.PAD_RIGHT, k=k)


def test_markov_batch_single_packed_and_left(markov_batch):
    data, offs = markov_batch
    check_packed(_vocab(dt.SINGLE), data, offs, True)
    sub = offs[:513]
    check_padded(_vocab(dt.KMER, 5), data[:sub[-1]], sub, True, dt.PAD_LEFT, k=5, pad_extra=7)


# ---------------------------------------------------------------- boundary fuzz

def _fuzz_batch(seed, n, max_len, alphabet_mix=True):
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, max_len + 1, n)
    lens[rng.integers(0, n, max(1, n // 10))] = 0
    total = int(lens.sum())
    data = synth.uniform_bytes(seed, total)
    if alphabet_mix:  # mostly DNA with every byte value present somewhere
        dna = np.frombuffer(b"ACGTNacgtn", np.uint8)
        pick = rng.random(total) < 0.9
        data[pick] = dna[rng.integers(0, 10, int(pick.sum()))]
    offs = synth.offsets_from_lengths(lens)
    return data, offs


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 7, 8, 15])
def test_fuzz_kmer_all_shapes(k):
    data, offs = _fuzz_batch(1000 + k, 2500, 130)
    v = _vocab(dt.KMER, k)
    for shift in (0, 1, 7, 15):
        check_packed(v, data, offs, cls=bool(shift % 2), k=k, byte_shift=shift)
    check_padded(v, data, offs, True, dt.PAD_RIGHT, k=k, pad_extra=3)
    check_padded(v, data, offs, False, dt.PAD_LEFT, k=k)


@pytest.mark.parametrize("k", [1, 3, 8])
def test_wide_padding_rows_are_mostly_pads(k):
    # short rows in a wide matrix: almost every store group of a row is pads
    data, offs = _fuzz_batch(2000 + k, 700, 130)
    v = _vocab(dt.KMER, k) if k > 1 else _vocab(dt.SINGLE)
    check_padded(v, data, offs, True, dt.PAD_RIGHT, k=k, pad_extra=3001)
    check_padded(v, data, offs, False, dt.PAD_LEFT, k=k, pad_extra=2999)


def test_fuzz_single_and_lut256():
    data, offs = _fuzz_batch(77, 3000, 130)
    for shift in (0, 3, 8):
        check_packed(_vocab(dt.SINGLE), data, offs, cls=True, byte_shift=shift)
    lut = oracle.fallback_lut()
    v = _vocab(dt.LUT256, lut=lut, pad_id=0, cls_id=101, sep_id=102)
    check_packed(v, data, offs, True, lut=lut, cls_id=101, sep_id=102, byte_shift=5)
    check_padded(v, data, offs, True, dt.PAD_LEFT, lut=lut, cls_id=101, sep_id=102, pad_extra=2)
    rng = np.random.default_rng(5)
    lut2 = rng.integers(0, 1 << 30, 256).astype(np.int32)
    check_packed(_vocab(dt.LUT256, lut=lut2), data, offs, False, lut=lut2)


def test_long_rows_cross_many_tiles():
    rng = np.random.default_rng(3)
    lens = rng.integers(15000, 70000, 40)
    lens[5] = 0
    lens[6] = 1
    data = synth.genome(synth.substream(9, 1), 31337, 3, int(lens.sum()))
    offs = synth.offsets_from_lengths(lens)
    for k in (1, 3, 6):
        v = _vocab(dt.KMER, k)
        check_packed(v, data, offs, True, k=k, byte_shift=k)
        check_padded(v, data, offs, True, dt.PAD_RIGHT, k=k)


def test_selftest_strings():
    data = np.frombuffer(b"ACGTNacgtn", np.uint8).copy()
    offs = np.array([0, 10], np.int64)
    lut = oracle.fallback_lut()
    check_packed(_vocab(dt.LUT256, lut=lut), data, offs, False, lut=lut)
    check_packed(_vocab(dt.SINGLE), data, offs, False)
    all_bytes = np.arange(256, dtype=np.uint8)
    check_packed(_vocab(dt.SINGLE), all_bytes, np.array([0, 256]), True)
    check_packed(_vocab(dt.KMER, 2), all_bytes, np.array([0, 256]), True, k=2)


# ---------------------------------------------------------------- edge cases

def test_empty_batch_and_empty_rows():
    torch = _torch()
    v = _vocab(dt.KMER, 3)
    # n = 0
    ids, out_off, _ = dt.encode(v, torch.zeros(1, dtype=torch.uint8, device="cuda"),
                                torch.zeros(1, dtype=torch.int64, device="cuda"), h_offsets=np.zeros(1, np.int64))
    torch.cuda.synchronize()
    assert out_off.cpu().tolist() == [0]
    # only empty rows, with and without specials
    offs = np.zeros(9, np.int64)
    data = np.zeros(0, np.uint8)
    for cls in (False, True):
        check_packed(v, data, offs, cls, k=3)
    check_padded(v, data, offs, True, dt.PAD_LEFT, k=3, pad_extra=4)
    # rows that do not start at byte 0, unused bytes between and after rows
    data = synth.iid(5, 50000, 0.05)
    offs = np.array([100, 100, 7000, 7000, 33000, 49000], np.int64)
    check_packed(_vocab(dt.KMER, 6), data, offs, True, k=6)


def test_output_offset_base_and_repeated_calls():
    torch = _torch()
    v = _vocab(dt.KMER, 4)
    for i, n in enumerate([300, 17, 1200, 5, 800]):
        data, offs = _fuzz_batch(500 + i, n, 3000)
        want_ids, want_off = _oracle(dt.KMER, data, offs, 4)
        ids = torch.empty(len(want_ids) + 8, dtype=torch.int32, device="cuda")
        out_off = torch.empty(n + 1, dtype=torch.int64, device="cuda")
        opts = dt.make_opts(offset_base=1000 + i)
        d_bytes, d_offs = _dev(data), _dev(offs)
        # write into ids[1:] so the output start is not 16-byte aligned
        dt.dnatok_encode(v.handle, d_bytes.data_ptr(), len(data), d_offs.data_ptr(), n, ids.data_ptr() + 4,
                         len(want_ids), out_off.data_ptr(), None, opts, torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        assert dt.sync_status() == 0
        assert np.array_equal(out_off.cpu().numpy(), want_off + 1000 + i)
        assert np.array_equal(ids[1:1 + len(want_ids)].cpu().numpy(), want_ids)


def test_device_side_errors_are_flagged_and_bounded():
    torch = _torch()
    v = _vocab(dt.KMER, 3)
    data, offs = _fuzz_batch(9, 400, 200)
    want_ids, want_off = _oracle(dt.KMER, data, offs, 3)
    d_bytes, d_offs = _dev(data), _dev(offs)
    stream = torch.cuda.current_stream().cuda_stream
    # PACKED capacity too small: nothing written past it
    cap = len(want_ids) // 2
    ids = torch.full((len(want_ids) + 64,), -7, dtype=torch.int32, device="cuda")
    out_off = torch.empty(len(offs), dtype=torch.int64, device="cuda")
    dt.dnatok_encode(v.handle, d_bytes.data_ptr(), len(data), d_offs.data_ptr(), len(offs) - 1, ids.data_ptr(), cap,
                     out_off.data_ptr(), None, dt.make_opts(), stream)
    assert dt.sync_status() == dt.DERR_CAPACITY
    got = ids.cpu().numpy()
    assert np.all(got[cap:] == -7) and np.array_equal(got[:cap], want_ids[:cap])
    assert np.array_equal(out_off.cpu().numpy(), want_off)
    # decreasing offsets
    bad = offs.copy()
    bad[10] = bad[12] + 5
    dt.dnatok_encode(v.handle, d_bytes.data_ptr(), len(data), _dev(bad).data_ptr(), len(bad) - 1, ids.data_ptr(),
                     ids.numel(), out_off.data_ptr(), None, dt.make_opts(), stream)
    assert dt.sync_status() & dt.DERR_OFFSETS
    # offsets beyond nbytes
    bad = offs.copy()
    bad[-1] = len(data) + 100
    dt.dnatok_encode(v.handle, d_bytes.data_ptr(), len(data), _dev(bad).data_ptr(), len(bad) - 1, ids.data_ptr(),
                     ids.numel(), out_off.data_ptr(), None, dt.make_opts(), stream)
    assert dt.sync_status() & dt.DERR_OFFSETS
    # PADDED width below the longest row
    W = int(np.diff(want_off).max()) - 1
    n = len(offs) - 1
    pid = torch.full((n * W + 64,), -7, dtype=torch.int32, device="cuda")
    pm = torch.full((n * W + 64,), -7, dtype=torch.int8, device="cuda")
    dt.dnatok_encode(v.handle, d_bytes.data_ptr(), len(data), d_offs.data_ptr(), n, pid.data_ptr(), n * W,
                     out_off.data_ptr(), pm.data_ptr(), dt.make_opts(layout=dt.PADDED, pad_to=W), stream)
    assert dt.sync_status() == dt.DERR_ROW_WIDTH
    assert np.all(pid.cpu().numpy()[n * W:] == -7) and np.all(pm.cpu().numpy()[n * W:] == -7)
    # host-checkable errors return at once
    with pytest.raises(dt.DnatokError) as e:
        dt.dnatok_encode(v.handle, d_bytes.data_ptr(), len(data), d_offs.data_ptr(), n, pid.data_ptr(), 10,
                         out_off.data_ptr(), pm.data_ptr(), dt.make_opts(layout=dt.PADDED, pad_to=W), stream)
    assert e.value.code == dt.ETOOSMALL
    with pytest.raises(dt.DnatokError) as e:
        dt.Vocab(dt.KMER, 16)
    assert e.value.code == dt.EVOCAB


def test_two_streams_concurrently():
    torch = _torch()
    v = _vocab(dt.KMER, 6)
    jobs = [_fuzz_batch(70 + i, 2000, 4000) for i in range(2)]
    streams = [torch.cuda.Stream() for _ in jobs]
    outs = []
    for (data, offs), s in zip(jobs, streams):
        with torch.cuda.stream(s):
            d_bytes, d_offs = _dev(data), _dev(offs)
            outs.append((dt.encode(v, d_bytes, d_offs, h_offsets=offs, stream=s), d_bytes, d_offs))
    torch.cuda.synchronize()
    for (data, offs), ((ids, out_off, _), _, _), s in zip(jobs, outs, streams):
        assert dt.sync_status(s) == 0
        want_ids, want_off = _oracle(dt.KMER, data, offs, 6)
        assert np.array_equal(ids.cpu().numpy(), want_ids)
        assert np.array_equal(out_off.cpu().numpy(), want_off)


# ---------------------------------------------------------------- decode

@pytest.mark.parametrize("kind,k", [(dt.SINGLE, 1)] + [(dt.KMER, k) for k in range(1, 9)] + [(dt.KMER, 12)])
def test_decode_matches_oracle(kind, k):
    # single-nucleotide and k <= 8: the strided kernel, one instance per k;
    # k = 12: the contiguous kernel, a tile's output (4,096 x 12 bytes) over
    # the LDS stage, so tokens are written directly
    torch = _torch()
    rng = np.random.default_rng(k)
    vs = 10 if kind == dt.SINGLE else 5 + 4 ** k
    ids = rng.integers(-3, vs + 5, 50000).astype(np.int32)
    lens = rng.integers(0, 300, 400)
    offs = synth.offsets_from_lengths(lens)
    offs = offs[offs <= len(ids)]
    v = _vocab(kind, k)
    want, want_off = oracle.decode(kind, ids, offs, k=k)
    out, out_off = dt.decode(v, _dev(ids), _dev(offs))
    torch.cuda.synchronize()
    assert dt.sync_status() == 0
    assert np.array_equal(out_off.cpu().numpy(), want_off)
    assert np.array_equal(out.cpu().numpy()[:want_off[-1]], want)


@pytest.mark.parametrize("kind,k", [(dt.SINGLE, 1), (dt.KMER, 6)])
def test_decode_empty_and_tile_edges(kind, k):
    # no ids (rows all empty, or no rows), exactly one tile of 4,096 and of
    # 8,192 ids, one id past it, and rows ending on tile edges
    torch = _torch()
    v = _vocab(kind, k)
    rng = np.random.default_rng(40 + k)
    vs = 10 if kind == dt.SINGLE else 5 + 4 ** k
    cases = [(0, [0, 0, 0, 0]), (0, [0]), (4096, [0, 4096]), (8192, [0, 8192]), (8193, [0, 4096, 8192, 8193]),
             (16384, [0, 1, 4095, 4096, 8191, 8192, 12288, 16384])]
    for n_ids, offs in cases:
        offs = np.array(offs, np.int64)
        ids = rng.integers(-3, vs + 5, n_ids).astype(np.int32)
        print("decode edges kind=%d k=%d ids=%d rows=%d" % (kind, k, n_ids, len(offs) - 1), flush=True)
        want, want_off = oracle.decode(kind, ids, offs, k=k)
        d_ids = _dev(ids) if n_ids else torch.zeros(0, dtype=torch.int32, device="cuda")
        out, out_off = dt.decode(v, d_ids, _dev(offs))
        torch.cuda.synchronize()
        assert dt.sync_status() == 0
        assert np.array_equal(out_off.cpu().numpy(), want_off)
        assert np.array_equal(out.cpu().numpy()[:want_off[-1]], want)


@pytest.mark.parametrize("kind,k", [(dt.SINGLE, 1), (dt.KMER, 6), (dt.KMER, 8), (dt.KMER, 12)])
def test_decode_many_tiles_look_back(kind, k):
    """Some 3M ids (hundreds of tiles of 4,096 ids, so
    the look-back walks more than one window of 64 predecessors), specials
    and out-of-vocabulary ids mixed in, rows from empty to 20,000 ids, the
    output at several 16-byte phases: every byte and offset against the
    oracle."""
    torch = _torch()
    rng = np.random.default_rng(100 + k)
    vs = 10 if kind == dt.SINGLE else 5 + 4 ** k
    n_ids = 3_000_000 if k <= 8 else 700_000
    ids = rng.integers(5, vs, n_ids).astype(np.int32)
    sp = rng.random(n_ids) < 0.01
    ids[sp] = rng.integers(-2, 12, int(sp.sum()))
    lens = rng.integers(0, 20000, 400)
    offs = synth.offsets_from_lengths(lens)
    offs = np.concatenate([offs[offs < n_ids], [n_ids]]).astype(np.int64)
    v = _vocab(kind, k)
    want, want_off = oracle.decode(kind, ids, offs, k=k)
    d_ids, d_offs = _dev(ids), _dev(offs)
    n = len(offs) - 1
    cap = int(want_off[-1])
    for shift in (0, 3, 13):
        print("decode kind=%d k=%d shift=%d ids=%d rows=%d" % (kind, k, shift, n_ids, n), flush=True)
        buf = torch.full((cap + 64,), 7, dtype=torch.uint8, device="cuda")
        oo = torch.empty(n + 1, dtype=torch.int64, device="cuda")
        dt.dnatok_decode(v.handle, d_ids.data_ptr(), n_ids, d_offs.data_ptr(), n, buf.data_ptr() + shift, cap,
                         oo.data_ptr(), None)
        torch.cuda.synchronize()
        assert dt.sync_status() == 0
        assert np.array_equal(oo.cpu().numpy(), want_off)
        got = buf.cpu().numpy()
        assert np.all(got[:shift] == 7) and np.all(got[shift + cap:] == 7)
        bad = np.nonzero(got[shift:shift + cap] != want)[0]
        assert bad.size == 0, "first mismatch at byte %d" % bad[0]


@pytest.mark.parametrize("kind,k", [(dt.SINGLE, 1), (dt.KMER, 6)])
def test_decode_capacity_short(kind, k):
    """An output buffer 1,001 bytes short: DERR_CAPACITY is raised, the
    bytes inside the capacity are right (tiles crossing it write their
    tokens one by one), nothing is written past it, and the output offsets
    are still the full ones."""
    torch = _torch()
    rng = np.random.default_rng(300 + k)
    vs = 10 if kind == dt.SINGLE else 5 + 4 ** k
    n_ids = 400_000
    ids = rng.integers(5, vs, n_ids).astype(np.int32)
    offs = np.array([0, 1000, 150_000, n_ids], np.int64)
    v = _vocab(kind, k)
    want, want_off = oracle.decode(kind, ids, offs, k=k)
    cap = int(want_off[-1]) - 1001
    buf = torch.full((cap + 4096,), 7, dtype=torch.uint8, device="cuda")
    oo = torch.empty(len(offs), dtype=torch.int64, device="cuda")
    dt.dnatok_decode(v.handle, _dev(ids).data_ptr(), n_ids, _dev(offs).data_ptr(), len(offs) - 1, buf.data_ptr(), cap,
                     oo.data_ptr(), None)
    torch.cuda.synchronize()
    assert dt.sync_status() == dt.DERR_CAPACITY
    got = buf.cpu().numpy()
    assert np.array_equal(got[:cap], want[:cap])
    assert np.all(got[cap:] == 7)
    assert np.array_equal(oo.cpu().numpy(), want_off)


def test_encode_decode_roundtrip_acgt():
    torch = _torch()
    rng = np.random.default_rng(1)
    lens = rng.integers(0, 2000, 300) * 6
    data = np.frombuffer(b"ACGT", np.uint8)[rng.integers(0, 4, int(lens.sum()))].copy()
    offs = synth.offsets_from_lengths(lens)
    for kind, k in ((dt.SINGLE, 1), (dt.KMER, 6), (dt.KMER, 2)):
        v = _vocab(kind, k)
        ids, out_off, _ = dt.encode(v, _dev(data), _dev(offs), h_offsets=offs, add_cls_sep=True)
        out, dec_off = dt.decode(v, ids, out_off)
        torch.cuda.synchronize()
        assert np.array_equal(dec_off.cpu().numpy(), offs)
        assert np.array_equal(out.cpu().numpy()[:offs[-1]], data)


# ---------------------------------------------------------------- several k-mer vocabularies in one pass

def _check_multi(vs, ks, data, offs, cls, layout, side):
    torch = _torch()
    print("multi ks=%s n=%d layout=%d side=%d cls=%d" % (ks, len(offs) - 1, layout, side, cls), flush=True)
    res = dt.encode_multi(vs, _dev(data), _dev(offs), h_offsets=offs, add_cls_sep=cls, layout=layout, pad_side=side)
    torch.cuda.synchronize()
    assert dt.sync_status() == 0
    for k, (ids, oo, mask) in zip(ks, res):
        want_ids, want_off = _oracle(dt.KMER, data, offs, k, cls=cls)
        assert np.array_equal(oo.cpu().numpy(), want_off), k
        if layout == dt.PADDED:
            W = ids.shape[1]
            w_ids, w_mask = oracle.pad(want_ids, want_off, W, side, 0)
            assert np.array_equal(ids.cpu().numpy(), w_ids), k
            assert np.array_equal(mask.cpu().numpy(), w_mask), k
        else:
            assert np.array_equal(ids.cpu().numpy(), want_ids), k


def test_multi_vocab_fuzz_all_layouts():
    data, offs = _fuzz_batch(501, 2500, 130)
    ks = [1, 2, 3, 4, 5, 6, 7, 8]
    vs = [_vocab(dt.KMER, k) for k in ks]
    _check_multi(vs, ks, data, offs, True, dt.PACKED, dt.PAD_RIGHT)
    _check_multi(vs, ks, data, offs, True, dt.PADDED, dt.PAD_RIGHT)
    _check_multi(vs, ks, data, offs, False, dt.PADDED, dt.PAD_LEFT)


def test_multi_vocab_markov_full_size(markov_batch):
    data, offs = markov_batch
    ks = [3, 4, 5, 6]
    _check_multi([_vocab(dt.KMER, k) for k in ks], ks, data, offs, True, dt.PADDED, dt.PAD_RIGHT)


def test_multi_vocab_many_rows_unfused_scan():
    # more rows than the PADDED launch folds its row scans into
    data, offs = _fuzz_batch(502, 20000, 40)
    ks = [3, 6]
    _check_multi([_vocab(dt.KMER, k) for k in ks], ks, data, offs, True, dt.PADDED, dt.PAD_RIGHT)


@pytest.mark.parametrize("ks", [(6,), (3, 4, 5, 6)])
def test_walkers_with_several_tiles_prefetch(ks):
    # 4 KiB tiles and one tile walker per CU: every walker takes several tiles
    # (the tile count is not a multiple of the 8 XCDs) and puts the next one's
    # loads in flight while writing the current one
    data, offs = synth.workload_markov_batch(600, 5000, seed=synth.substream(95, len(ks)))
    ragged = synth.offsets_from_lengths(np.random.default_rng(96).integers(0, 12000, 250))
    ragged = ragged[ragged <= len(data)]
    vs = [_vocab(dt.KMER, k) for k in ks]
    dt.set_tuning(vs[0], tile_bytes=4096, blocks_per_cu=1)
    _check_multi(vs, list(ks), data, offs, True, dt.PADDED, dt.PAD_RIGHT)
    _check_multi(vs, list(ks), data, offs, False, dt.PACKED, dt.PAD_RIGHT)
    _check_multi(vs, list(ks), data[:ragged[-1]], ragged, True, dt.PADDED, dt.PAD_LEFT)


def test_multi_vocab_errors():
    torch = _torch()
    data, offs = _fuzz_batch(503, 10, 50)
    bpe = dt.Vocab(dt.BPE, merges=np.zeros((0, 2), np.int32))
    with pytest.raises(dt.DnatokError) as e:
        dt.encode_multi([_vocab(dt.KMER, 3), bpe], _dev(data), _dev(offs), h_offsets=offs)
    assert e.value.code == dt.EVOCAB
    vs = [_vocab(dt.KMER, 3), _vocab(dt.KMER, 4)]
    outs = [(torch.empty(1000, dtype=torch.int32, device="cuda"), torch.empty(11, dtype=torch.int64, device="cuda"),
             None) for _ in vs]
    opts = [dt.make_opts(True), dt.make_opts(False)]
    with pytest.raises(dt.DnatokError) as e:
        dt.MultiCall(vs, _dev(data), _dev(offs), outs, opts).run()
    assert e.value.code == dt.EINVAL


@pytest.mark.parametrize("k", [1, 3, 6])
def test_small_packed_batches_scan_in_the_cell_launch(k):
    # up to 512 rows PACKED: the row starts are formed inside the cell launch
    for n_rows, seed in ((1, 1), (37, 2), (512, 3)):
        data, offs = _fuzz_batch(600 + seed * 10 + k, n_rows, 3000)
        v = _vocab(dt.KMER, k) if k > 1 else _vocab(dt.SINGLE)
        kind = dt.KMER if k > 1 else dt.SINGLE
        for shift, cls in ((0, True), (3, False)):
            check_packed(v, data, offs, cls, k=k, byte_shift=shift)
