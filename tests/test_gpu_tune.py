"""GPU tests of tuning, the autotuner and captured graphs: every tiling the
autotuner may pick gives the oracle's ids, and every replay of a captured
encode gives the oracle's ids for what its buffers hold at that replay."""
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


def _batch(seed, n, hi):
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, hi, n)
    data = synth.genome(synth.substream(90, seed), synth.substream(91, seed), 3, int(lens.sum()))
    return data, synth.offsets_from_lengths(lens)


@pytest.mark.parametrize("k", [1, 6])
def test_every_kmer_tiling_matches_oracle(k):
    torch = _torch()
    data, offs = _batch(1, 700, 3000)
    v = dt.Vocab(dt.KMER, k=k) if k > 1 else dt.Vocab(dt.SINGLE)
    want_ids, want_off = oracle.encode(dt.KMER if k > 1 else dt.SINGLE, data, offs, k=k, add_cls_sep=True)
    d_in, d_off = _dev(data), _dev(offs)
    for tile in (4096, 8192, 16384, 32768, 65536):
        for b in (0, 1, 2, 4):
            print("tiling k=%d tile=%d blocks=%d" % (k, tile, b), flush=True)
            dt.set_tuning(v, tile_bytes=tile, blocks_per_cu=b)
            ids, oo, _ = dt.encode(v, d_in, d_off, h_offsets=offs, add_cls_sep=True)
            torch.cuda.synchronize()
            assert np.array_equal(oo.cpu().numpy(), want_off)
            assert np.array_equal(ids.cpu().numpy(), want_ids)
    t, ms = dt.autotune(v, d_in, d_off, h_offsets=offs, add_cls_sep=True)
    assert t["tile_bytes"] in (4096, 8192, 16384, 32768, 65536) and ms > 0
    got = dt.dnatok_get_tuning(v.handle).as_dict()
    assert got == t
    ids, oo, _ = dt.encode(v, d_in, d_off, h_offsets=offs, add_cls_sep=True)
    assert np.array_equal(ids.cpu().numpy(), want_ids)


def test_ticketed_tiles_match_oracle():
    """Batches with more tiles than resident workgroups, cut with ticketed
    tiles (spread > 0): one and four vocabularies, PADDED (row scans fused
    into the launch) and PACKED, launched back to back (the ticket counter
    resets itself between launches)."""
    torch = _torch()
    data, offs = synth.workload_markov_batch(3000, 8192)
    data[::7919] = ord("x")
    d_in, d_off = _dev(data), _dev(offs)
    ks = (3, 4, 5, 6)
    vs = [dt.Vocab(dt.KMER, k=k) for k in ks]
    want = {k: oracle.encode_threads(dt.KMER, data, offs, k=k, add_cls_sep=True) for k in ks}
    for tile in (4096, 16384):
        for sp in (10, 100):
            print("ticketed tiles: tile=%d spread=%d" % (tile, sp), flush=True)
            for v in vs:
                dt.set_tuning(v, tile_bytes=tile, spread=sp)
            for rep in range(2):
                outs = dt.encode_multi(vs, d_in, d_off, h_offsets=offs, add_cls_sep=True, layout=dt.PADDED)
                torch.cuda.synchronize()
                assert dt.sync_status() == 0
                for k, (ids, oo, mask) in zip(ks, outs):
                    w_ids, w_off = want[k]
                    wp, wm = oracle.pad_threads(w_ids, w_off, int(np.diff(w_off).max()))
                    assert np.array_equal(oo.cpu().numpy(), w_off)
                    assert np.array_equal(ids.cpu().numpy(), wp) and np.array_equal(mask.cpu().numpy(), wm)
            ids, oo, _ = dt.encode(vs[1], d_in, d_off, h_offsets=offs, add_cls_sep=True)
            torch.cuda.synchronize()
            assert dt.sync_status() == 0
            assert np.array_equal(oo.cpu().numpy(), want[4][1]) and np.array_equal(ids.cpu().numpy(), want[4][0])
    single = dt.Vocab(dt.SINGLE)
    dt.set_tuning(single, tile_bytes=8192, spread=25)
    w_ids, w_off = oracle.encode_threads(dt.SINGLE, data, offs, add_cls_sep=True)
    ids, oo, _ = dt.encode(single, d_in, d_off, h_offsets=offs, add_cls_sep=True)
    torch.cuda.synchronize()
    assert dt.sync_status() == 0
    assert np.array_equal(oo.cpu().numpy(), w_off) and np.array_equal(ids.cpu().numpy(), w_ids)


def test_every_bpe_tiling_matches_oracle():
    torch = _torch()
    corpus = synth.bpe_corpus(n=1 << 20, seed=synth.substream(92, 0))
    merges = oracle.bpe_train(corpus, 500)
    v = dt.Vocab(dt.BPE, merges=merges)
    data, offs = _batch(2, 120, 12000)
    data[np.random.default_rng(3).integers(0, len(data), 40)] = ord("N")
    want_ids, want_off = oracle.encode(dt.BPE, data, offs, merges=merges, add_cls_sep=True)
    d_in, d_off = _dev(data), _dev(offs)
    for S in (1024, 2048, 8192, 65536):
        for w in (8, 4, 2, 1):
            print("bpe tiling S=%d waves=%d" % (S, w), flush=True)
            dt.set_tuning(v, bpe_item_bytes=S, bpe_max_waves=w)
            ids, oo, _ = dt.encode(v, d_in, d_off, h_offsets=offs, add_cls_sep=True)
            torch.cuda.synchronize()
            assert np.array_equal(oo.cpu().numpy(), want_off)
            assert np.array_equal(ids.cpu().numpy(), want_ids)
    t, ms = dt.autotune(v, d_in, d_off, h_offsets=offs, add_cls_sep=True, reps=1)
    assert t["bpe_item_bytes"] > 0 and t["bpe_max_waves"] in (1, 2, 4, 8)


def test_bad_tuning_is_rejected():
    v = dt.Vocab(dt.KMER, k=3)
    for kw in ({"tile_bytes": 5000}, {"tile_bytes": 1 << 20}, {"blocks_per_cu": -1}, {"bpe_item_bytes": 512},
               {"bpe_max_waves": 3}, {"spread": -1}, {"spread": 101}):
        with pytest.raises(dt.DnatokError) as e:
            dt.set_tuning(v, **kw)
        assert e.value.code == dt.EINVAL


@pytest.mark.parametrize("kind", ["single", "kmer6_padded", "bpe"])
def test_graph_replays_follow_buffer_contents(kind):
    torch = _torch()
    n, L = 64, 4099
    datas = [synth.iid(synth.substream(93, i), n * L, 0.01) for i in range(3)]
    offs = synth.offsets_from_lengths([L] * n)
    merges = None
    if kind == "single":
        v, okind, k = dt.Vocab(dt.SINGLE), dt.SINGLE, 1
    elif kind == "kmer6_padded":
        v, okind, k = dt.Vocab(dt.KMER, k=6), dt.KMER, 6
    else:
        merges = oracle.bpe_train(synth.bpe_corpus(n=1 << 19, seed=synth.substream(94, 0)), 200)
        v, okind, k = dt.Vocab(dt.BPE, merges=merges), dt.BPE, 1
    padded = kind == "kmer6_padded"
    W = -(-L // k) + 2
    cap = n * W if padded else n * (L + 2)
    d_in = _dev(datas[0])
    d_off = _dev(offs)
    ids = torch.zeros(cap, dtype=torch.int32, device="cuda")
    oo = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    mask = torch.zeros(cap, dtype=torch.int8, device="cuda") if padded else None
    g = dt.Graph([dict(vocab=v, d_bytes=d_in, d_offsets=d_off, d_ids=ids, d_out_offsets=oo, d_mask=mask,
                       add_cls_sep=True, layout=dt.PADDED if padded else dt.PACKED, pad_to=W if padded else 0)])
    other = _dev(datas[2][:L * 8])
    other_off = _dev(synth.offsets_from_lengths([L] * 8))
    for rep in range(5):
        data = datas[rep % 2]
        print("graph %s replay %d" % (kind, rep), flush=True)
        d_in.copy_(torch.from_numpy(data))
        g.launch()
        # eager work of the program between replays
        dt.encode(v, other, other_off, h_offsets=synth.offsets_from_lengths([L] * 8), add_cls_sep=True)
        torch.cuda.synchronize()
        want_ids, want_off = oracle.encode(okind, data, offs, k=k, merges=merges, add_cls_sep=True)
        assert np.array_equal(oo.cpu().numpy(), want_off)
        if padded:
            w_ids, w_mask = oracle.pad(want_ids, want_off, W)
            assert np.array_equal(ids.cpu().numpy(), w_ids.reshape(-1))
            assert np.array_equal(mask.cpu().numpy(), w_mask.reshape(-1))
        else:
            assert np.array_equal(ids.cpu().numpy()[:len(want_ids)], want_ids)
    g.close()


def test_one_graph_of_several_encodes():
    torch = _torch()
    data, offs = synth.workload_iid()
    n = len(offs) - 1
    d_in, d_off = _dev(data), _dev(offs)
    calls, wants = [], []
    for kind, k in ((dt.SINGLE, 1), (dt.KMER, 6), (dt.KMER, 3)):
        v = dt.Vocab(kind, k=k)
        want_ids, want_off = oracle.encode(kind, data, offs, k=k)
        wants.append((want_ids, want_off))
        calls.append(dict(vocab=v, d_bytes=d_in, d_offsets=d_off,
                          d_ids=torch.zeros(len(want_ids), dtype=torch.int32, device="cuda"),
                          d_out_offsets=torch.zeros(n + 1, dtype=torch.int64, device="cuda")))
    g = dt.Graph(calls)
    for rep in range(3):
        for c in calls:
            c["d_ids"].zero_()
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        for c, (want_ids, want_off) in zip(calls, wants):
            assert np.array_equal(c["d_ids"].cpu().numpy(), want_ids)
            assert np.array_equal(c["d_out_offsets"].cpu().numpy(), want_off)
    g.close()
