"""GPU parity of ranked-merge BPE: the HIP library (through its C-ABI) against
the CPU oracle, id by id and offset by offset (bit-exact), on exhaustive
short strings, barrier-rich fuzz, rows longer than the on-chip symbol buffer,
trained tables of 4096 and 8192 merges, PACKED and PADDED layouts, and decode
of the resulting ids."""
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


def _packed(v, merges, data, offs, cls):
    torch = _torch()
    print("bpe packed R=%d n=%d nbytes=%d cls=%d" % (len(merges), len(offs) - 1, len(data), cls), flush=True)
    want_ids, want_off = oracle.encode(oracle.BPE, data, offs, merges=merges, add_cls_sep=cls)
    ids, out_off, _ = dt.encode(v, _dev(data), _dev(offs), h_offsets=offs, add_cls_sep=cls)
    torch.cuda.synchronize()
    assert dt.sync_status() == 0
    assert np.array_equal(out_off.cpu().numpy(), want_off)
    got = ids.cpu().numpy()
    assert got.shape == want_ids.shape
    bad = np.nonzero(got != want_ids)[0]
    assert bad.size == 0, "first mismatch at %d: got %d want %d" % (bad[0], got[bad[0]], want_ids[bad[0]])
    return want_ids, want_off


def _padded(v, merges, data, offs, cls, side, extra=0):
    torch = _torch()
    print("bpe padded R=%d n=%d side=%d cls=%d" % (len(merges), len(offs) - 1, side, cls), flush=True)
    want_ids, want_off = oracle.encode(oracle.BPE, data, offs, merges=merges, add_cls_sep=cls)
    W = max(1, int(np.diff(want_off).max(initial=0)) + extra)
    w_ids, w_mask = oracle.pad(want_ids, want_off, W, side, 0)
    ids, out_off, mask = dt.encode(v, _dev(data), _dev(offs), h_offsets=offs, add_cls_sep=cls, layout=dt.PADDED,
                                   pad_side=side, pad_to=W)
    torch.cuda.synchronize()
    assert dt.sync_status() == 0
    assert np.array_equal(out_off.cpu().numpy(), want_off)
    assert np.array_equal(ids.cpu().numpy(), w_ids)
    assert np.array_equal(mask.cpu().numpy(), w_mask)


def _random_table(seed, R, p_chain=0.2):
    """A well-formed table drawn at random: operands are bases or earlier
    merges, pairs distinct, some (X, X) pairs to exercise chains."""
    rng = np.random.default_rng(seed)
    m, seen = [], set()

    def pick():
        x = int(rng.integers(0, 4 + len(m)))
        return 5 + x if x < 4 else 10 + (x - 4)

    while len(m) < R:
        a = pick()
        b = a if rng.random() < p_chain else pick()
        if (a, b) not in seen:
            seen.add((a, b))
            m.append((a, b))
    return np.array(m, np.int32).reshape(-1, 2)


@pytest.fixture(scope="module")
def trained_small():
    corpus = synth.genome(synth.substream(60, 0), synth.substream(60, 1), 3, 200_000)
    return oracle.bpe_train(corpus, 300)


def test_exhaustive_short_strings(trained_small):
    # every ACGT string of length <= 7 as its own row (21844 rows), three tables
    parts, lens = [], []
    for L in range(8):
        idx = np.arange(4 ** L)
        digits = (idx[:, None] >> (2 * np.arange(L - 1, -1, -1))) & 3
        parts.append(np.frombuffer(b"ACGT", np.uint8)[digits].reshape(-1))
        lens += [L] * (4 ** L)
    data = np.concatenate(parts)
    offs = synth.offsets_from_lengths(lens)
    for merges in (trained_small, _random_table(1, 60, 0.3), _random_table(2, 200, 0.1)):
        v = dt.Vocab(dt.BPE, merges=merges)
        _packed(v, merges, data, offs, cls=False)


def test_random_tables_runs_and_repeats():
    # rounds that merge many ranks at once: random tables rich in (X, X)
    # pairs and shared operands, on rows of base runs, short tandem repeats
    # and uniform bases, up to 6000 bases (many occurrences per round)
    rng = np.random.default_rng(23)
    acgt = np.frombuffer(b"ACGT", np.uint8)
    for t in range(24):
        merges = _random_table(100 + t, int(rng.integers(1, 400)), float(rng.choice([0.05, 0.3, 0.6])))
        lens = rng.integers(0, 6000 if t % 3 == 0 else 300, 48)
        rows = []
        for L in lens:
            kind = int(rng.integers(0, 3))
            if kind == 0:  # runs of one base
                runs = rng.integers(1, 12, size=L + 1)
                row = np.repeat(acgt[rng.integers(0, 4, size=L + 1)], runs)[:L]
            elif kind == 1:  # a short motif repeated
                motif = acgt[rng.integers(0, 4, size=int(rng.integers(1, 5)))]
                row = np.tile(motif, L // len(motif) + 1)[:L]
            else:
                row = acgt[rng.integers(0, 4, size=L)]
            rows.append(row)
        data = np.concatenate(rows) if rows else np.zeros(0, np.uint8)
        offs = synth.offsets_from_lengths(lens)
        v = dt.Vocab(dt.BPE, merges=merges)
        _packed(v, merges, data, offs, cls=False)


def test_fuzz_barriers_and_case(trained_small):
    rng = np.random.default_rng(11)
    n = 3000
    lens = rng.integers(0, 400, n)
    lens[rng.integers(0, n, 300)] = 0
    total = int(lens.sum())
    data = synth.uniform_bytes(12, total)
    dna = np.frombuffer(b"ACGTacgtNn", np.uint8)
    pick = rng.random(total) < 0.97
    data[pick] = dna[rng.integers(0, 10, int(pick.sum()))]
    offs = synth.offsets_from_lengths(lens)
    for merges in (trained_small, _random_table(3, 120, 0.25)):
        v = dt.Vocab(dt.BPE, merges=merges)
        _packed(v, merges, data, offs, cls=False)
        _packed(v, merges, data, offs, cls=True)
        _padded(v, merges, data, offs, True, dt.PAD_RIGHT, extra=3)
        _padded(v, merges, data, offs, False, dt.PAD_LEFT)


def test_zero_merges_equals_single():
    data, offs = synth.workload_iid(n_seqs=16, seq_len=5000)
    merges = np.zeros((0, 2), np.int32)
    ids, off = _packed(dt.Vocab(dt.BPE, merges=merges), merges, data, offs, cls=True)
    s_ids, s_off = oracle.encode(oracle.SINGLE, data, offs, add_cls_sep=True)
    assert np.array_equal(ids, s_ids) and np.array_equal(off, s_off)


def test_long_runs_and_item_boundaries(trained_small):
    # barrier-free runs far longer than one item (8192 bytes) and than the
    # on-chip symbol buffer, barriers placed on and around item boundaries
    rng = np.random.default_rng(5)
    lens = [0, 1, 8191, 8192, 8193, 16384, 30000, 70001, 100, 24000]
    data = synth.markov(synth.substream(61, 0), synth.substream(61, 1), 5, int(sum(lens)))
    offs = synth.offsets_from_lengths(lens)
    for p in (8191, 8192, 8193, 16383, 16384 + 8192, 80000, 80001, 120000):
        if p < len(data):
            data[p] = ord("N")
    data[rng.integers(0, len(data), 20)] = ord("x")
    merges = _random_table(7, 400, 0.2)
    for m in (trained_small, merges):
        v = dt.Vocab(dt.BPE, merges=m)
        _packed(v, m, data, offs, cls=True)
        _padded(v, m, data, offs, True, dt.PAD_LEFT, extra=1)


def test_trained_tables_4096_and_8192():
    corpus = synth.bpe_corpus(n=1 << 21, seed=synth.substream(62, 0))
    data, offs = synth.workload_bpe_batch(n_seqs=96, seed=synth.substream(62, 1))
    # barriers in half the rows
    rng = np.random.default_rng(3)
    for i in range(0, 96, 2):
        a, b = int(offs[i]), int(offs[i + 1])
        if b > a:
            data[rng.integers(a, b, max(1, (b - a) // 700))] = ord("N")
    for R in (4096, 8192):
        merges = oracle.bpe_train(corpus, R)
        assert len(merges) == R
        v = dt.Vocab(dt.BPE, merges=merges)
        _packed(v, merges, data, offs, cls=True)


def test_decode_matches_oracle(trained_small):
    torch = _torch()
    rng = np.random.default_rng(9)
    lens = rng.integers(0, 3000, 200)
    total = int(lens.sum())
    data = np.frombuffer(b"ACGTacgtNn", np.uint8)[rng.integers(0, 10, total)].copy()
    data[rng.integers(0, total, 50)] = ord("#")
    offs = synth.offsets_from_lengths(lens)
    merges = trained_small
    v = dt.Vocab(dt.BPE, merges=merges)
    ids, out_off, _ = dt.encode(v, _dev(data), _dev(offs), h_offsets=offs, add_cls_sep=True)
    out, out_off2 = dt.decode(v, ids, out_off)
    torch.cuda.synchronize()
    want_ids, want_off = oracle.encode(oracle.BPE, data, offs, merges=merges, add_cls_sep=True)
    w_bytes, w_off = oracle.decode(oracle.BPE, want_ids, want_off, merges=merges)
    assert np.array_equal(out_off2.cpu().numpy(), w_off)
    assert np.array_equal(out.cpu().numpy()[:len(w_bytes)], w_bytes)


def test_decode_long_tokens_tiles_over_the_stage(trained_small):
    """Ids of the longest merges, densely: a 4,096-id tile's output is far
    over the 32 KiB LDS stage, so tiles write their tokens directly; mixed
    with short ids and specials so staged and direct tiles alternate, and
    rows start inside tiles. Every byte and offset against the oracle."""
    torch = _torch()
    merges = trained_small
    R = len(merges)
    lens = np.ones(10 + R, np.int64)
    for r, (a, b) in enumerate(merges):
        lens[10 + r] = lens[a] + lens[b]
    longest = 10 + np.argsort(-lens[10:])[:16]
    assert lens[longest[0]] >= 9
    rng = np.random.default_rng(77)
    n_ids = 200_000
    ids = rng.integers(5, 10 + R, n_ids).astype(np.int32)
    # stretches of long tokens, about half of the tiles
    for t0 in range(0, n_ids, 8192):
        ids[t0:t0 + 4096] = longest[rng.integers(0, len(longest), min(4096, n_ids - t0))]
    sp = rng.random(n_ids) < 0.01
    ids[sp] = rng.integers(0, 5, int(sp.sum()))
    offs = np.concatenate([[0], np.sort(rng.choice(np.arange(1, n_ids), 300, replace=False)), [n_ids]]).astype(np.int64)
    v = dt.Vocab(dt.BPE, merges=merges)
    want, want_off = oracle.decode(oracle.BPE, ids, offs, merges=merges)
    out, out_off = dt.decode(v, _dev(ids), _dev(offs))
    torch.cuda.synchronize()
    assert dt.sync_status() == 0
    assert np.array_equal(out_off.cpu().numpy(), want_off)
    assert np.array_equal(out.cpu().numpy()[:len(want)], want)


def test_empty_batch_and_bad_tables():
    torch = _torch()
    merges = _random_table(4, 50)
    v = dt.Vocab(dt.BPE, merges=merges)
    data = np.zeros(0, np.uint8)
    offs = np.zeros(1, np.int64)
    ids, out_off, _ = dt.encode(v, _dev(np.zeros(1, np.uint8))[:0], _dev(offs), h_offsets=offs)
    torch.cuda.synchronize()
    assert out_off.cpu().numpy().tolist() == [0] and ids.numel() == 0
    offs = np.array([0, 0, 0], np.int64)
    _packed(v, merges, data, offs, cls=True)
    for bad in ([(5, 6), (5, 6)], [(5, 11)], [(9, 5)]):
        with pytest.raises(dt.DnatokError) as e:
            dt.Vocab(dt.BPE, merges=np.array(bad, np.int32))
        assert e.value.code == dt.EVOCAB
    with pytest.raises(dt.DnatokError) as e:
        dt.Vocab(dt.BPE, merges=_random_table(5, 8193, 0.0))
    assert e.value.code == dt.EVOCAB
