"""GPU parity at the full sizes of the benchmarked workloads, every id and
offset against the CPU oracle (bit-exact), in the launch configurations the
benchmark times:

* the ragged BPE batch: 1,024 rows of 500-20,000 bases, encoded with the
  committed 4,096-merge table, at the autotuner's tiling and at the
  library's default;
* the 2 GiB host-to-device stream: 16 chromosomes cut into 6,000-base
  windows, pushed in 64 MiB chunks through 3 slots, 6-mers, overlapped and
  sequential;
* the serving trace at its full size range: requests of 100 bases to
  1 Mbase over four vocabularies (single-nucleotide, 3-mer, 6-mer,
  BPE-4096), 32 MiB / 512-request batches under a 16 GiB budget, replayed
  at the trace's arrival times, each result against the oracle's encode of
  that sequence alone;
* decode of the batched workload's PACKED ids (4096 x 8192 bases with
  CLS/SEP: 33.6M single-nucleotide ids, 5.6M 6-mer ids), as the benchmark
  decodes them.

The oracle runs with its rows split over host threads (a static partition by
bytes; the same result as one call)."""
import os
import time

import numpy as np
import pytest

import oracle
import paper_2601_05531_amd as dt
import synth

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BPE_TABLE = os.path.join(ROOT, "tests", "golden", "bpe4096_order5_64M.txt")


def _threads():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    return torch


def _first_mismatch(got, want):
    bad = np.nonzero(got != want)[0]
    return "none" if bad.size == 0 else "at %d: got %d want %d" % (bad[0], got[bad[0]], want[bad[0]])


def _merges():
    return np.loadtxt(BPE_TABLE, dtype=np.int32).reshape(-1, 2)


@pytest.mark.parametrize("tiling", ["autotuned", "default"])
def test_bpe_batch_1024_rows_4096_merges(tiling):
    torch = _torch()
    merges = _merges()
    assert merges.shape == (4096, 2)
    data, offs = synth.workload_bpe_batch()
    assert len(offs) == 1025
    t0 = time.perf_counter()
    want_ids, want_off = oracle.encode_threads(oracle.BPE, data, offs, threads=_threads(), merges=merges)
    print("bpe batch: %d rows, %d bases, oracle %.1f s, tiling %s" % (
        len(offs) - 1, len(data), time.perf_counter() - t0, tiling), flush=True)
    v = dt.Vocab(dt.BPE, merges=merges)
    d_in = torch.from_numpy(data).cuda()
    d_off = torch.from_numpy(offs).cuda()
    if tiling == "autotuned":
        best, ms = dt.autotune(v, d_in, d_off, h_offsets=offs, reps=3)
        print("autotuned %s (%.3f ms)" % (best, ms), flush=True)
    ids, out_off, _ = dt.encode(v, d_in, d_off, h_offsets=offs)
    torch.cuda.synchronize()
    assert dt.sync_status() == 0
    assert np.array_equal(out_off.cpu().numpy(), want_off)
    got = ids.cpu().numpy()
    assert got.shape == want_ids.shape
    assert np.array_equal(got, want_ids), _first_mismatch(got, want_ids)
    v.close()


STREAM_BYTES = 1 << 31
STREAM_CHUNK = 64 << 20
STREAM_WINDOW = 6000


@pytest.fixture(scope="module")
def chromosomes_2gib():
    torch = _torch()
    lens = synth.chromosome_lengths(total=STREAM_BYTES)
    h = torch.empty(STREAM_BYTES, dtype=torch.uint8, pin_memory=True)
    t0 = time.perf_counter()
    synth.chromosomes(lens, out=h.numpy(), threads=_threads())
    woffs = oracle.windows(lens, STREAM_WINDOW)
    want_ids, want_off = oracle.encode_threads(oracle.KMER, h.numpy(), woffs, threads=_threads(), k=6)
    print("stream: %d bytes in %d records, %d windows, %d tokens; generation + oracle %.1f s" % (
        STREAM_BYTES, len(lens), len(woffs) - 1, len(want_ids), time.perf_counter() - t0), flush=True)
    yield lens, h, want_ids, want_off
    del h


@pytest.mark.parametrize("overlap", [True, False])
def test_stream_2gib_64mib_chunks_6mers(chromosomes_2gib, overlap):
    torch = _torch()
    lens, h, want_ids, want_off = chromosomes_2gib
    ends_all = np.cumsum(lens)
    v = dt.Vocab(dt.KMER, k=6)
    st = dt.Stream(v, STREAM_WINDOW, STREAM_CHUNK, len(want_ids), len(want_off) - 1, n_slots=3, overlap=overlap)
    print("stream overlap=%s: pushing %d chunks" % (overlap, STREAM_BYTES // STREAM_CHUNK), flush=True)
    for c0 in range(0, STREAM_BYTES, STREAM_CHUNK):
        c1 = c0 + STREAM_CHUNK
        st.push(h[c0:c1], ends_all[(ends_all > c0) & (ends_all <= c1)] - c0)
    ids, woff, r = st.flush(copy=False)
    assert r.n_windows == len(want_off) - 1 and r.n_tokens == len(want_ids) and r.n_bytes == STREAM_BYTES
    assert np.array_equal(woff.cpu().numpy(), want_off)
    got = ids.cpu().numpy()
    assert np.array_equal(got, want_ids), _first_mismatch(got, want_ids)
    st.close()
    v.close()


def test_serving_trace_full_size_range():
    """At least 500 requests of the trace (its first 440 plus the 20 largest
    of each vocabulary), sizes up to 1 Mbase, replayed at the trace's arrival
    times with the benchmark's batch limits."""
    torch = _torch()
    merges = _merges()
    vocab_rows = [(dt.Vocab(dt.SINGLE), oracle.SINGLE, 1, None),
                  (dt.Vocab(dt.KMER, k=3), oracle.KMER, 3, None),
                  (dt.Vocab(dt.KMER, k=6), oracle.KMER, 6, None),
                  (dt.Vocab(dt.BPE, merges=merges), oracle.BPE, 1, merges)]
    arrivals, sizes, which = synth.serving_trace()
    pick = set(range(440))
    for vi in range(4):
        idx = np.nonzero(which == vi)[0]
        pick.update(idx[np.argsort(sizes[idx])[-20:]].tolist())
    pick = np.array(sorted(pick))
    assert len(pick) >= 500 and sizes[pick].max() > 900_000
    G = 64 << 20
    h = torch.empty(G, dtype=torch.uint8, pin_memory=True)
    synth.genome(synth.substream(5, 1), synth.substream(5, 2), 3, G, out=h.numpy())
    rng = np.random.default_rng(synth.substream(5, 3))
    starts_all = rng.integers(0, G - int(sizes.max()), len(sizes))
    starts, lens, vs = starts_all[pick], sizes[pick], which[pick]
    arr = arrivals[pick] - arrivals[pick[0]]
    # the picked requests keep their order; gaps longer than 5 ms are cut short
    arr = np.concatenate([[0.0], np.cumsum(np.minimum(np.diff(arr), 5e-3))])
    print("serving: %d requests, %d bases, largest %d" % (len(pick), int(lens.sum()), int(lens.max())), flush=True)

    srv = dt.Server(budget_bytes=16 << 30, n_streams=4, max_batch=512, max_batch_bytes=32 << 20)
    tickets = []
    t0 = time.perf_counter()
    for i in range(len(pick)):
        d = t0 + arr[i] - time.perf_counter()
        if d > 0:
            time.sleep(d)
        a, n = int(starts[i]), int(lens[i])
        tickets.append(srv.submit(vocab_rows[vs[i]][0], h[a:a + n], add_cls_sep=True))
    got = []
    for t in tickets:
        ids, r = srv.wait(t)
        assert r.status == dt.OK and r.dev_flags == 0
        got.append(ids.cpu().numpy())
        srv.release(t)
    done, batches, peak = srv.stats()
    srv.close()
    print("serving: %d batches, peak arena %d bytes" % (batches, peak), flush=True)
    # how many requests share a batch depends on how fast the box drains the
    # replay (a fast one serves each request before the next arrives);
    # batching itself is pinned by the back-to-back server test
    assert done == len(pick) and 1 <= batches <= len(pick)

    # the oracle, one request alone per call, requests spread over threads
    from concurrent.futures import ThreadPoolExecutor
    hn = h.numpy()

    def want(i):
        _, kind, k, m = vocab_rows[vs[i]]
        a, n = int(starts[i]), int(lens[i])
        ids, _ = oracle.encode(kind, hn[a:a + n], np.array([0, n], np.int64), k=k, merges=m, add_cls_sep=True)
        return ids

    order = np.argsort(-lens)  # longest first, so the threads finish together
    with ThreadPoolExecutor(max_workers=_threads()) as ex:
        res = dict(zip(order.tolist(), ex.map(want, order.tolist())))
    for i in range(len(pick)):
        assert np.array_equal(got[i], res[i]), "request %d (vocab %d, %d bytes): %s" % (
            int(pick[i]), int(vs[i]), int(lens[i]), _first_mismatch(got[i], res[i]) if got[i].shape == res[i].shape
            else "lengths %d vs %d" % (len(got[i]), len(res[i])))
    for row in vocab_rows:
        row[0].close()


@pytest.mark.parametrize("kind,k", [(oracle.SINGLE, 1), (oracle.KMER, 6)])
def test_decode_batched_workload(kind, k):
    torch = _torch()
    data, offs = synth.workload_markov_batch()
    ids_h, off_h = oracle.encode_threads(kind, data, offs, threads=_threads(), k=k, add_cls_sep=True)
    want, want_off = oracle.decode(kind, ids_h, off_h, k=k)
    print("decode %s: %d ids -> %d bytes" % ("single" if kind == oracle.SINGLE else "6-mer", len(ids_h), len(want)),
          flush=True)
    v = dt.Vocab(kind, k=k)
    out, out_off = dt.decode(v, torch.from_numpy(ids_h).cuda(), torch.from_numpy(off_h).cuda())
    torch.cuda.synchronize()
    assert dt.sync_status() == 0
    assert np.array_equal(out_off.cpu().numpy(), want_off)
    got = out[:len(want)].cpu().numpy()
    assert np.array_equal(got, want), _first_mismatch(got, want)
    v.close()
