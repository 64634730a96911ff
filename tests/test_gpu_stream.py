"""GPU parity of the pinned host-to-device stream: every id and window offset
equals the oracle's encode of the same windows (oracle.windows cuts records
into windows; oracle.encode encodes them), for chunk sizes from one byte to
whole records, record ends on and across window and chunk boundaries, and
both the overlapped and the sequential (baseline) schedule."""
import numpy as np
import pytest

import oracle
import paper_2601_05531_amd as dt
import synth

pytestmark = pytest.mark.gpu


def _pinned(data):
    import torch
    t = torch.empty(len(data), dtype=torch.uint8, pin_memory=True)
    t.numpy()[:] = data
    return t


def _run(vocab, data, rec_lens, window, chunk, cls=False, overlap=True, n_slots=3):
    """Push `data` (records of rec_lens) in chunks of `chunk` bytes."""
    h = _pinned(data)
    starts = np.concatenate([[0], np.cumsum(rec_lens)])
    max_windows = int(sum(-(-int(L) // window) for L in rec_lens)) + 8
    max_tokens = int(len(data)) + 2 * max_windows + 8
    s = dt.Stream(vocab, window, chunk, max_tokens, max_windows, n_slots=n_slots, add_cls_sep=cls, overlap=overlap)
    ends_all = starts[1:]
    for c0 in range(0, max(len(data), 1), chunk):
        c1 = min(c0 + chunk, len(data))
        ends = ends_all[(ends_all > c0) & (ends_all <= c1)] - c0
        # a record that ends exactly at a chunk start is reported by the earlier chunk
        s.push(h[c0:c1], ends)
    ids, woff, r = s.flush()
    s.close()
    return ids.cpu().numpy(), woff.cpu().numpy(), r


def _want(kind, k, data, rec_lens, window, cls=False):
    woffs = oracle.windows(rec_lens, window)
    return oracle.encode(kind, data, woffs, k=k, add_cls_sep=cls)


@pytest.mark.parametrize("chunk", [1, 7, 997, 4096, 65536])
def test_stream_small_records_all_chunk_sizes(chunk):
    rng = np.random.default_rng(chunk)
    rec_lens = [int(x) for x in rng.integers(0, 3000, 12)] + [0, 1, 37, 38, 74]
    if chunk < 100:
        rec_lens = [int(x) // 10 for x in rec_lens]
    data = synth.genome(synth.substream(7, chunk), 11 + chunk, 3, int(sum(rec_lens)))
    v = dt.Vocab(dt.KMER, k=6)
    print("stream chunk=%d bytes=%d" % (chunk, len(data)), flush=True)
    ids, woff, r = _run(v, data, rec_lens, 37, chunk)
    want_ids, want_off = _want(dt.KMER, 6, data, rec_lens, 37)
    assert r.n_windows == len(want_off) - 1 and r.n_bytes == len(data)
    assert np.array_equal(woff, want_off)
    assert np.array_equal(ids, want_ids)


@pytest.mark.parametrize("overlap", [True, False])
def test_stream_chromosome_like(overlap):
    # records longer than several chunks, 6000-base windows, 6-mers
    lens = synth.chromosome_lengths(total=24_000_000, n=5, lo=1e6, hi=1e7, seed=3)
    data = synth.chromosomes(lens, seed=4)
    v = dt.Vocab(dt.KMER, k=6)
    print("stream chromosomes overlap=%d bytes=%d" % (overlap, len(data)), flush=True)
    ids, woff, r = _run(v, data, lens, 6000, 4 << 20, overlap=overlap)
    want_ids, want_off = _want(dt.KMER, 6, data, lens, 6000)
    assert np.array_equal(woff, want_off)
    assert np.array_equal(ids, want_ids)


def test_stream_single_vocab_with_specials_two_slots():
    rng = np.random.default_rng(2)
    rec_lens = [int(x) for x in rng.integers(1, 20000, 9)]
    data = synth.genome(synth.substream(8, 1), 5, 3, int(sum(rec_lens)))
    v = dt.Vocab(dt.SINGLE)
    ids, woff, r = _run(v, data, rec_lens, 1000, 3001, cls=True, n_slots=2)
    want_ids, want_off = _want(dt.SINGLE, 1, data, rec_lens, 1000, cls=True)
    assert np.array_equal(woff, want_off)
    assert np.array_equal(ids, want_ids)


def test_stream_reset_and_reuse():
    import torch
    v = dt.Vocab(dt.KMER, k=3)
    data = synth.iid(9, 50000, 0.02)
    h = _pinned(data)
    s = dt.Stream(v, 500, 8192, 60000, 200)
    outs = []
    for _ in range(2):
        for c0 in range(0, len(data), 8192):
            s.push(h[c0:c0 + 8192])
        ids, woff, r = s.flush()
        outs.append((ids.cpu().numpy(), woff.cpu().numpy()))
        s.reset()
    s.close()
    want_ids, want_off = _want(dt.KMER, 3, data, [len(data)], 500)
    for ids, woff in outs:
        assert np.array_equal(ids, want_ids) and np.array_equal(woff, want_off)
    torch.cuda.synchronize()


def test_stream_errors_leave_no_partial_output():
    import torch
    v = dt.Vocab(dt.KMER, k=6)
    data = synth.iid(10, 40000, 0.0)
    h = _pinned(data)
    # capacity: the second push would overflow max_windows -> rejected before any work
    s = dt.Stream(v, 6000, 20000, 10**6, 4)
    s.push(h[:20000])
    with pytest.raises(dt.DnatokError) as e:
        s.push(h[20000:40000])
    assert e.value.code == dt.ETOOSMALL
    with pytest.raises(dt.DnatokError) as e:  # failed stream refuses pushes
        s.push(h[20000:40000])
    assert e.value.code == dt.ESTATE
    s.reset()
    s.push(h[:20000])
    ids, woff, r = s.flush()
    assert r.n_windows == 4  # 3 full windows + the flushed tail
    want_ids, want_off = _want(dt.KMER, 6, data[:20000], [20000], 6000)
    assert np.array_equal(ids.cpu().numpy(), want_ids)
    with pytest.raises(dt.DnatokError) as e:  # flushed stream refuses pushes
        s.push(h[:10])
    assert e.value.code == dt.ESTATE
    s.reset()
    pageable = torch.from_numpy(data.copy())
    with pytest.raises(dt.DnatokError) as e:
        s.push(pageable[:100])
    assert e.value.code == dt.EINVAL
    s.reset()
    with pytest.raises(dt.DnatokError) as e:  # chunk larger than chunk_bytes
        s.push(h[:30000])
    assert e.value.code == dt.EINVAL
    s.close()
    with pytest.raises(dt.DnatokError) as e:
        dt.Stream(dt.Vocab(dt.BPE, merges=np.zeros((0, 2), np.int32)), 100, 1000, 100, 10)
    assert e.value.code == dt.EVOCAB
