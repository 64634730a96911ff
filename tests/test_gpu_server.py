"""GPU tests of the serving loop: every request's ids equal the oracle's
encode of that sequence alone, whatever else shares its batch, stream or
arena (continuous batching), with pinned and pageable inputs, under a budget
small enough that admission has to wait for released results."""
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


@pytest.fixture(scope="module")
def vocabs():
    corpus = synth.genome(synth.substream(80, 0), synth.substream(80, 1), 3, 300_000)
    merges = oracle.bpe_train(corpus, 400)
    vs = [(dt.Vocab(dt.SINGLE), oracle.SINGLE, 1, None),
          (dt.Vocab(dt.KMER, k=3), oracle.KMER, 3, None),
          (dt.Vocab(dt.KMER, k=6), oracle.KMER, 6, None),
          (dt.Vocab(dt.BPE, merges=merges), oracle.BPE, 1, merges)]
    return vs


def _requests(seed, n, hi):
    rng = np.random.default_rng(seed)
    genome = synth.genome(synth.substream(81, seed), synth.substream(82, seed), 3, 4 << 20)
    sizes = np.floor(np.exp(rng.uniform(0, np.log(hi), n))).astype(np.int64)
    sizes[rng.integers(0, n, max(1, n // 50))] = 0
    starts = rng.integers(0, len(genome) - hi, n)
    which = rng.integers(0, 4, n)
    cls = rng.random(n) < 0.7
    return genome, sizes, starts, which, cls


def _want(vocab_row, data, cls):
    _, kind, k, merges = vocab_row
    ids, _ = oracle.encode(kind, data, np.array([0, len(data)], np.int64), k=k, merges=merges, add_cls_sep=cls)
    return ids


def test_mix_equals_alone(vocabs):
    torch = _torch()
    genome, sizes, starts, which, cls = _requests(1, 400, 20000)
    pinned = torch.empty(len(genome), dtype=torch.uint8, pin_memory=True)
    pinned.numpy()[:] = genome
    srv = dt.Server(budget_bytes=1 << 30, n_streams=4, max_batch=64, max_batch_bytes=1 << 20)
    print("server mix: %d requests, %d bytes" % (len(sizes), int(sizes.sum())), flush=True)
    tickets = []
    for i in range(len(sizes)):
        a, n = int(starts[i]), int(sizes[i])
        v = vocabs[which[i]][0]
        if i % 2:
            t = srv.submit(v, pinned[a:a + n], add_cls_sep=bool(cls[i]))
        else:
            t = srv.submit(v, genome[a:a + n].copy(), add_cls_sep=bool(cls[i]))
        tickets.append(t)
    for i, t in enumerate(tickets):
        ids, r = srv.wait(t)
        assert r.dev_flags == 0
        assert r.t_submit <= r.t_start <= r.t_done
        a, n = int(starts[i]), int(sizes[i])
        want = _want(vocabs[which[i]], genome[a:a + n], bool(cls[i]))
        got = ids.cpu().numpy()
        assert np.array_equal(got, want), "request %d (vocab %d, %d bytes)" % (i, which[i], n)
        srv.release(t)
    done, batches, peak = srv.stats()
    assert done == len(sizes)
    assert batches < len(sizes)  # requests were batched
    srv.close()


def test_small_budget_admission_waits_for_releases(vocabs):
    _torch()
    genome, sizes, starts, which, cls = _requests(2, 120, 30000)
    # arena of about 300 KB: a fraction of the 120 requests fits at once
    budget = 0
    for extra in range(0, 1 << 30, 64 << 10):
        try:
            s = dt.Server(budget_bytes=extra, n_streams=2, max_batch=8, max_batch_bytes=64 << 10)
        except dt.DnatokError as e:
            assert e.code == dt.EINVAL
            continue
        s.close()
        budget = extra + (256 << 10)
        break
    srv = dt.Server(budget_bytes=budget, n_streams=2, max_batch=8, max_batch_bytes=64 << 10)
    print("server small budget: %d bytes" % budget, flush=True)
    with pytest.raises(dt.DnatokError) as e:
        srv.submit(vocabs[0][0], np.zeros(65 << 10, np.uint8))
    assert e.value.code == dt.EBUDGET
    sizes = np.minimum(sizes, 60 << 10)
    tickets = [srv.submit(vocabs[which[i]][0], genome[int(starts[i]):int(starts[i]) + int(sizes[i])].copy(),
                          add_cls_sep=bool(cls[i])) for i in range(len(sizes))]
    # results are released as they complete, in whatever order (a request
    # may wait for memory that later requests of another vocabulary hold)
    import time
    left = dict(enumerate(tickets))
    t_end = time.time() + 60
    while left and time.time() < t_end:
        for i, t in list(left.items()):
            r = dt.dnatok_server_poll(srv.handle, t)
            if r is None:
                continue
            assert r.status == dt.OK
            ids = dt.device_view(r.d_ids, r.n_tokens, "<i4")
            a, n = int(starts[i]), int(sizes[i])
            assert np.array_equal(ids.cpu().numpy(), _want(vocabs[which[i]], genome[a:a + n], bool(cls[i])))
            srv.release(t)
            del left[i]
    assert not left, "%d requests never completed" % len(left)
    done, batches, peak = srv.stats()
    assert done == len(sizes) and peak <= budget
    srv.close()
