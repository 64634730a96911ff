"""Pins of the CPU oracle against what the paper and arithmetic fix (no GPU).

Each pin is chosen so that a plausible slip in ``oracle.c`` (digit order, most-
vs least-significant base first, N vs UNK, a dropped tail token, a wrong pad
side, a BPE round that merges the wrong occurrences) fails at least one test.
"""
import itertools
import math
import os
import sys

import numpy as np
import pytest

import oracle
from oracle import brute
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(strings):
    data = np.frombuffer("".join(strings).encode("latin-1"), dtype=np.uint8).copy()
    offs = np.zeros(len(strings) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(s) for s in strings])
    return data, offs


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append(line.rstrip("\n").split("\t"))
    return rows


# ---------------------------------------------------------------- LUT256 / SINGLE

def test_fallback_lut_selftest_golden():
    (text, expected), = _golden("fallback_lut_selftest.txt")
    data, offs = _rows([text])
    ids, out_off = oracle.encode(oracle.LUT256, data, offs, lut=oracle.fallback_lut())
    assert ids.tolist() == [int(x) for x in expected.split()]
    assert out_off.tolist() == [0, 10]


def test_fallback_lut_other_bytes_zero():
    data = np.arange(256, dtype=np.uint8)
    ids, _ = oracle.encode(oracle.LUT256, data, np.array([0, 256]), lut=oracle.fallback_lut())
    dna = {ord(c): v for c, v in zip("ACGTNacgtn", [1, 2, 3, 4, 0] * 2)}
    assert ids.tolist() == [dna.get(b, 0) for b in range(256)]


def test_single_selftest_and_all_bytes():
    data, offs = _rows(["ACGTNacgtn"])
    ids, _ = oracle.encode(oracle.SINGLE, data, offs)
    assert ids.tolist() == [5, 6, 7, 8, 9, 5, 6, 7, 8, 9]
    all_bytes = np.arange(256, dtype=np.uint8)
    ids, _ = oracle.encode(oracle.SINGLE, all_bytes, np.array([0, 256]))
    want = {ord(c): 5 + i for i, c in enumerate("ACGT")}
    want.update({ord(c): 5 + i for i, c in enumerate("acgt")})
    want[ord("N")] = want[ord("n")] = 9
    assert ids.tolist() == [want.get(b, 1) for b in range(256)]


def test_single_specials_and_lengths():
    data, offs = _rows(["", "A", "acgtn#"])
    ids, out_off = oracle.encode(oracle.SINGLE, data, offs, add_cls_sep=True)
    assert ids.tolist() == [2, 3, 2, 5, 3, 2, 5, 6, 7, 8, 9, 1, 3]
    assert out_off.tolist() == [0, 2, 5, 13]
    ids, out_off = oracle.encode(oracle.SINGLE, data, offs, add_cls_sep=False)
    assert out_off.tolist() == [0, 0, 1, 7]


def test_lut256_specials_use_given_ids():
    data, offs = _rows(["AC"])
    ids, _ = oracle.encode(oracle.LUT256, data, offs, lut=oracle.fallback_lut(), add_cls_sep=True,
                           cls_id=101, sep_id=102)
    assert ids.tolist() == [101, 1, 2, 102]


# ---------------------------------------------------------------- KMER

def test_kmer_closed_forms_golden():
    for k, text, expected in _golden("kmer_closed_forms.txt"):
        data, offs = _rows([text])
        ids, _ = oracle.encode(oracle.KMER, data, offs, k=int(k))
        assert ids.tolist() == [int(x) for x in expected.split()], (k, text)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_kmer_every_kmer_against_base4(k):
    strings = ["".join(p) for p in itertools.product("ACGT", repeat=k)]
    data, offs = _rows(strings)
    ids, out_off = oracle.encode(oracle.KMER, data, offs, k=k)
    assert np.all(np.diff(out_off) == 1)
    assert ids.tolist() == [brute.kmer_id(s) for s in strings]
    # ids are a bijection onto [5, 5 + 4^k)
    assert sorted(ids.tolist()) == list(range(5, 5 + 4 ** k))
    lower = [s.lower() for s in strings]
    ids_l, _ = oracle.encode(oracle.KMER, *_rows(lower), k=k)
    assert np.array_equal(ids, ids_l)


def test_kmer_long_k_extremes():
    for k in (7, 11, 15):
        for ch, val in (("A", 0), ("T", 4 ** k - 1)):
            ids, _ = oracle.encode(oracle.KMER, *_rows([ch * k]), k=k)
            assert ids.tolist() == [5 + val]
        s = ("ACGT" * 4)[:k]
        ids, _ = oracle.encode(oracle.KMER, *_rows([s]), k=k)
        assert ids.tolist() == [brute.kmer_id(s)]


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 7, 8])
def test_kmer_lengths_closed_form(k):
    rng = np.random.default_rng(k)
    lens = list(range(0, 70)) + [int(x) for x in rng.integers(0, 5000, 20)]
    strings = ["".join(rng.choice(list("ACGTN"), size=L)) for L in lens]
    data, offs = _rows(strings)
    for cls in (False, True):
        ids, out_off = oracle.encode(oracle.KMER, data, offs, k=k, add_cls_sep=cls)
        want = [math.ceil(L / k) + 2 * cls for L in lens]
        assert np.diff(out_off).tolist() == want
        for i, L in enumerate(lens):
            row = ids[out_off[i]:out_off[i + 1]]
            if cls:
                assert row[0] == 2 and row[-1] == 3
                row = row[1:-1]
            if L % k:
                assert row[-1] == 1  # short final frame


def test_kmer_benchmark_shapes():
    # 8,192-base rows with CLS/SEP: k = 3, 4, 5, 6 -> 2733, 2050, 1641, 1368 tokens
    for k, want in ((3, 2733), (4, 2050), (5, 1641), (6, 1368)):
        _, out_off = oracle.encode(oracle.KMER, np.full(8192, ord("A"), np.uint8), np.array([0, 8192]),
                                   k=k, add_cls_sep=True)
        assert out_off[1] == want
    # 16,384-base row, 6-mers: 2,731 tokens, the last a short frame -> UNK
    ids, out_off = oracle.encode(oracle.KMER, np.full(16384, ord("C"), np.uint8), np.array([0, 16384]), k=6)
    assert out_off[1] == 2731 and ids[-1] == 1 and ids[0] == brute.kmer_id("CCCCCC")


def test_kmer_frames_not_reset_by_n():
    ids, _ = oracle.encode(oracle.KMER, *_rows(["ACGNACGTACGT"]), k=6)
    assert ids.tolist() == [1, brute.kmer_id("GTACGT")]


def test_kmer_matches_bruteforce_on_random_rows():
    rng = np.random.default_rng(7)
    alphabet = list("ACGTacgtNn#x")
    for k in (2, 3, 5, 6):
        strings = ["".join(rng.choice(alphabet, size=int(L), p=[.11] * 8 + [.04, .04, .02, .02]))
                   for L in rng.integers(0, 200, 40)]
        ids, out_off = oracle.encode(oracle.KMER, *_rows(strings), k=k)
        for i, s in enumerate(strings):
            want = []
            for j in range(0, len(s), k):
                fr = s[j:j + k]
                ok = len(fr) == k and all(c in "ACGTacgt" for c in fr)
                want.append(brute.kmer_id(fr) if ok else 1)
            assert ids[out_off[i]:out_off[i + 1]].tolist() == want


# ---------------------------------------------------------------- padding

def test_padding_invariants_and_sides():
    rng = np.random.default_rng(3)
    strings = ["".join(rng.choice(list("ACGTN"), size=int(L))) for L in rng.integers(0, 60, 30)]
    data, offs = _rows(strings)
    ids, out_off = oracle.encode(oracle.KMER, data, offs, k=3, add_cls_sep=True)
    lens = np.diff(out_off)
    W = int(lens.max()) + 5
    r_ids, r_mask = oracle.pad(ids, out_off, W, oracle.RIGHT)
    l_ids, l_mask = oracle.pad(ids, out_off, W, oracle.LEFT)
    assert r_mask.sum() == lens.sum() == l_mask.sum()
    assert np.all(r_ids[r_mask == 0] == 0) and np.all(l_ids[l_mask == 0] == 0)
    for i, L in enumerate(lens):
        assert r_mask[i].tolist() == [1] * L + [0] * (W - L)
        assert np.array_equal(np.roll(r_ids[i], W - L), l_ids[i])
        assert r_ids[i, :L].tolist() == ids[out_off[i]:out_off[i + 1]].tolist()
    with pytest.raises(ValueError):
        oracle.pad(ids, out_off, int(lens.max()) - 1)


# ---------------------------------------------------------------- decode

def test_decode_roundtrip_single_kmer():
    rng = np.random.default_rng(11)
    strings = ["".join(rng.choice(list("ACGT"), size=int(L))) for L in rng.integers(0, 90, 25)]
    data, offs = _rows(strings)
    ids, out_off = oracle.encode(oracle.SINGLE, data, offs, add_cls_sep=True)
    dec, dec_off = oracle.decode(oracle.SINGLE, ids, out_off)
    assert np.array_equal(dec, data) and np.array_equal(dec_off, offs)
    for k in (2, 3, 6):
        strings_k = [s[:len(s) - len(s) % k] for s in strings]
        data_k, offs_k = _rows(strings_k)
        ids, out_off = oracle.encode(oracle.KMER, data_k, offs_k, k=k, add_cls_sep=True)
        dec, dec_off = oracle.decode(oracle.KMER, ids, out_off, k=k)
        assert np.array_equal(dec, data_k) and np.array_equal(dec_off, offs_k)


def test_decode_unk_width_and_specials():
    ids = np.array([2, 1, 9, 3, 0, 4, 999], dtype=np.int32)
    dec, _ = oracle.decode(oracle.SINGLE, ids, np.array([0, 7]))
    assert bytes(dec) == b"NNN"
    dec, _ = oracle.decode(oracle.KMER, np.array([1, 5, 4100], np.int32), np.array([0, 3]), k=6)
    assert bytes(dec) == b"NNNNNN" + b"AAAAAA" + b"TTTTTT"


# ---------------------------------------------------------------- BPE

COUNTER_EXAMPLE = [(5, 6), (10, 7), (7, 8)]  # (A,C)->AC, (AC,G)->ACG, (G,T)->GT


def _tables():
    rng = np.random.default_rng(5)
    corp1 = "".join(rng.choice(list("ACGT"), size=3000, p=[.4, .1, .1, .4]))
    corp2 = "".join(rng.choice(list("ACGT"), size=3000))
    t1, _ = brute.bpe_train_recount(corp1, 40)
    t2, _ = brute.bpe_train_recount(corp2, 25)
    return [COUNTER_EXAMPLE, [(5, 5), (10, 10), (10, 5), (11, 11)], t1, t2]


def test_bpe_counterexample():
    ids, _ = oracle.encode(oracle.BPE, *_rows(["ACGT"]), merges=COUNTER_EXAMPLE)
    assert ids.tolist() == [11, 8]  # [ACG, T], not [AC, GT]
    assert brute.bpe_encode_text("ACGT", COUNTER_EXAMPLE) == [11, 8]


@pytest.mark.parametrize("ti", range(4))
def test_bpe_exhaustive_short_strings(ti):
    table = _tables()[ti]
    assert oracle.bpe_check(table) == 0
    strings = ["".join(p) for L in range(1, 8) for p in itertools.product("ACGT", repeat=L)]
    ids, out_off = oracle.encode(oracle.BPE, *_rows(strings), merges=table)
    for i, s in enumerate(strings):
        assert ids[out_off[i]:out_off[i + 1]].tolist() == brute.bpe_encode_text(s, table), s


def test_bpe_random_rows_with_barriers():
    rng = np.random.default_rng(9)
    tables = _tables()
    strings = ["".join(rng.choice(list("ACGTacgtNn#"), size=int(L), p=[.12] * 8 + [.02, .02, .0]
                                  if L % 2 else [.115] * 8 + [.03, .03, .02]))
               for L in rng.integers(0, 300, 60)]
    for table in tables:
        ids, out_off = oracle.encode(oracle.BPE, *_rows(strings), merges=table, add_cls_sep=True)
        for i, s in enumerate(strings):
            assert ids[out_off[i]:out_off[i + 1]].tolist() == [2] + brute.bpe_encode_text(s, table) + [3]


def test_bpe_zero_merges_is_single():
    rng = np.random.default_rng(2)
    data = rng.integers(0, 256, 5000).astype(np.uint8)
    data[::3] = np.frombuffer(b"ACGTNacgtn", np.uint8)[rng.integers(0, 10, data[::3].size)]
    offs = np.array([0, 1000, 1000, 4000, 5000])
    a, ao = oracle.encode(oracle.BPE, data, offs, merges=np.zeros((0, 2), np.int32), add_cls_sep=True)
    b, bo = oracle.encode(oracle.SINGLE, data, offs, add_cls_sep=True)
    assert np.array_equal(a, b) and np.array_equal(ao, bo)


def test_bpe_decode_concatenates_to_input():
    rng = np.random.default_rng(4)
    table = _tables()[2]
    strings = ["".join(rng.choice(list("ACGT"), size=int(L))) for L in rng.integers(1, 400, 30)]
    data, offs = _rows(strings)
    ids, out_off = oracle.encode(oracle.BPE, data, offs, merges=table)
    dec, dec_off = oracle.decode(oracle.BPE, ids, out_off, merges=table)
    assert np.array_equal(dec, data) and np.array_equal(dec_off, offs)
    for i, s in enumerate(strings):
        toks = ids[out_off[i]:out_off[i + 1]].tolist()
        assert "".join(brute.expand(t, table) for t in toks) == s


# ---------------------------------------------------------------- trainer

@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_trainer_matches_recount(seed):
    rng = np.random.default_rng(100 + seed)
    probs = rng.dirichlet([1, 1, 1, 1])
    text = "".join(rng.choice(list("ACGT"), size=1500, p=probs))
    if seed % 2:  # barriers and soft-masking
        t = list(text)
        for p in rng.integers(0, len(t), 20):
            t[p] = "N"
        for p in rng.integers(0, len(t), 200):
            t[p] = t[p].lower()
        text = "".join(t)
    want, runs = brute.bpe_train_recount(text, 60)
    got = oracle.bpe_train(np.frombuffer(text.encode(), np.uint8), 60)
    assert [tuple(x) for x in got.tolist()] == want
    assert oracle.bpe_check(got) == 0
    # encoding the corpus with the learned table reproduces the trainer's segmentation
    ids, _ = oracle.encode(oracle.BPE, np.frombuffer(text.encode(), np.uint8), np.array([0, len(text)]),
                           merges=got)
    assert [t for t in ids.tolist() if t >= 5 and t != 9] == [t for run in runs for t in run]


def test_trainer_first_merge_of_a_dominated_corpus():
    got = oracle.bpe_train(np.frombuffer(b"AAAAAAAAAAAAAAAAAAAAAC", np.uint8), 1)
    assert got.tolist() == [[5, 5]]
    # counts below 2 stop the trainer
    assert oracle.bpe_train(np.frombuffer(b"ACGT", np.uint8), 5).shape == (0, 2)


def test_trainer_deterministic_and_well_formed():
    import synth
    corpus = synth.bpe_corpus(n=200_000, seed=123)
    a = oracle.bpe_train(corpus, 300)
    b = oracle.bpe_train(corpus, 300)
    assert a.shape == (300, 2) and np.array_equal(a, b)
    assert oracle.bpe_check(a) == 0


def test_bpe_check_rejects_bad_tables():
    assert oracle.bpe_check([(5, 6), (5, 6)]) == 2       # duplicate pair
    assert oracle.bpe_check([(5, 11)]) == 1             # refers to a later merge
    assert oracle.bpe_check([(9, 5)]) == 1              # N is never merged
    assert oracle.bpe_check([(5, 6), (10, 7)]) == 0


# ---------------------------------------------------------------- windows

def test_windows_closed_form():
    lens = [0, 1, 5999, 6000, 6001, 12000, 25_000]
    offs = oracle.windows(lens, 6000)
    assert len(offs) - 1 == sum(math.ceil(L / 6000) for L in lens)
    assert offs[-1] == sum(lens)
    assert np.all(np.diff(offs) <= 6000) and np.all(np.diff(offs) > 0)


def test_bpe4096_table_is_the_trainers_output():
    # the stored table of the batched BPE workload is exactly what the oracle
    # trainer writes for the seeded 64 Mbase order-5 corpus (about 30 s)
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
    import make_bpe4096
    stored = make_bpe4096.load()
    assert stored.shape == (4096, 2)
    assert oracle.bpe_check(stored) == 0
    assert np.array_equal(make_bpe4096.make(), stored)


# ---------------------------------------------------------------- reverse complement

def test_revcomp_golden():
    for row in _golden("revcomp_overlap.txt"):
        if row[0] != "rc":
            continue
        data, offs = _rows([row[1]])
        assert bytes(oracle.revcomp(data, offs)).decode("latin-1") == row[2]


def test_revcomp_involution_and_bruteforce():
    rng = np.random.default_rng(11)
    strings = ["".join(chr(int(b)) for b in rng.integers(0, 256, int(L))) for L in rng.integers(0, 60, 30)]
    strings += ["ACGTNacgtn", "", "A"]
    data, offs = _rows(strings)
    rc = oracle.revcomp(data, offs)
    assert np.array_equal(oracle.revcomp(rc, offs), data)
    for i, s in enumerate(strings):
        assert bytes(rc[offs[i]:offs[i + 1]]).decode("latin-1") == brute.revcomp_text(s)


@pytest.mark.parametrize("k", [1, 3, 6])
def test_revcomp_kmer_closed_form(k):
    # On ACGT rows with L a multiple of k, token j of the reverse complement
    # is token nb-1-j of the row with its digits complemented (3 - d) and
    # read in reverse order.
    rng = np.random.default_rng(k)
    strings = ["".join(rng.choice(list("ACGTacgt"), size=k * int(m))) for m in rng.integers(0, 20, 12)]
    data, offs = _rows(strings)
    fwd, foff = oracle.encode(oracle.KMER, data, offs, k=k)
    rev, roff = oracle.encode(oracle.KMER, oracle.revcomp(data, offs), offs, k=k)
    assert np.array_equal(foff, roff)
    for i in range(len(strings)):
        f = fwd[foff[i]:foff[i + 1]]
        r = rev[roff[i]:roff[i + 1]]
        for j in range(len(f)):
            v = int(f[len(f) - 1 - j]) - 5
            digits = [(v >> (2 * (k - 1 - t))) & 3 for t in range(k)]
            want = 5 + sum((3 - d) * 4 ** t for t, d in enumerate(digits))
            assert int(r[j]) == want


# ---------------------------------------------------------------- overlapping k-mers

def test_overlap_golden():
    for row in _golden("revcomp_overlap.txt"):
        if row[0] != "ov":
            continue
        ids, out_off = oracle.encode_overlap(*_rows([row[2]]), k=int(row[1]))
        assert ids.tolist() == [int(x) for x in row[3].split()]


@pytest.mark.parametrize("k", [1, 2, 4, 6, 8])
def test_overlap_lengths_and_bruteforce(k):
    rng = np.random.default_rng(20 + k)
    alphabet = list("ACGTacgtNn#")
    strings = ["".join(rng.choice(alphabet, size=int(L), p=[.115] * 8 + [.04, .04, .0]))
               for L in rng.integers(0, 40, 40)] + ["", "A" * (k - 1), "C" * k]
    for cls in (False, True):
        ids, out_off = oracle.encode_overlap(*_rows(strings), k=k, add_cls_sep=cls)
        for i, s in enumerate(strings):
            L = len(s)
            nb = L - k + 1 if L >= k else (1 if L else 0)
            assert out_off[i + 1] - out_off[i] == nb + 2 * cls
            want = brute.overlap_body_text(s, k)
            if cls:
                want = [2] + want + [3]
            assert ids[out_off[i]:out_off[i + 1]].tolist() == want


@pytest.mark.parametrize("k", [2, 3, 6])
def test_overlap_contains_the_frames_and_rolls(k):
    # Every non-overlapping frame is the overlapping window at s = j*k, and
    # consecutive valid windows satisfy id' - 5 = ((id - 5) * 4 + d) mod 4^k.
    rng = np.random.default_rng(30 + k)
    strings = ["".join(rng.choice(list("ACGTN"), size=int(L), p=[.24] * 4 + [.04])) for L in rng.integers(k, 90, 25)]
    data, offs = _rows(strings)
    ov, ooff = oracle.encode_overlap(data, offs, k=k)
    fr, foff = oracle.encode(oracle.KMER, data, offs, k=k)
    for i, s in enumerate(strings):
        o = ov[ooff[i]:ooff[i + 1]]
        f = fr[foff[i]:foff[i + 1]]
        for j in range(len(s) // k):
            assert o[j * k] == f[j]
        for t in range(len(o) - 1):
            if o[t] != 1 and o[t + 1] != 1:
                d = "ACGT".index(s[t + k])
                assert int(o[t + 1]) - 5 == ((int(o[t]) - 5) * 4 + d) % 4 ** k


# ---------------------------------------------------------------- embedding lookup

def test_embed_matches_torch_embedding():
    import torch
    rng = np.random.default_rng(5)
    strings = ["".join(rng.choice(list("ACGTNacgt#"), size=int(L))) for L in rng.integers(0, 50, 20)]
    data, offs = _rows(strings)
    for kind, k, V in ((oracle.SINGLE, 1, 11), (oracle.KMER, 3, 69)):
        ids, out_off = oracle.encode(kind, data, offs, k=k, add_cls_sep=True)
        W = int(np.diff(out_off).max())
        pids, _ = oracle.pad(ids, out_off, W, oracle.LEFT)
        table = rng.standard_normal((V, 16)).astype(np.float32)
        got = oracle.embed(table, pids)
        want = torch.nn.functional.embedding(torch.from_numpy(pids.astype(np.int64)), torch.from_numpy(table))
        assert got.shape == (len(strings), W, 16)
        assert np.array_equal(got, want.numpy())
        rows = brute.embed_rows([list(r) for r in table], ids.tolist())
        assert np.array_equal(oracle.embed(table, ids), np.array(rows, dtype=np.float32).reshape(-1, 16))


def test_embed_identity_table_recovers_ids_and_rejects_range():
    data, offs = _rows(["ACGTNacgtn#", "GATTACA"])
    ids, _ = oracle.encode(oracle.SINGLE, data, offs, add_cls_sep=True)
    table = np.repeat(np.arange(10, dtype=np.int32)[:, None], 3, axis=1)
    out = oracle.embed(table, ids)
    assert np.array_equal(out[:, 0], ids) and np.array_equal(out[:, 2], ids)
    with pytest.raises(ValueError):
        oracle.embed(table, np.array([10]))
    with pytest.raises(ValueError):
        oracle.embed(table, np.array([-1]))


def test_threaded_oracle_equals_single_thread():
    """encode_threads / pad_threads split rows by bytes over threads; their
    result must be exactly the single call's (empty rows and batches too)."""
    data, offs = synth.workload_markov_batch(300, 1000)
    offs = offs.copy()
    offs[5:9] = offs[5]  # a run of empty rows
    for threads in (1, 2, 7, 64):
        for kind, k in ((oracle.SINGLE, 1), (oracle.KMER, 5)):
            a = oracle.encode(kind, data, offs, k=k, add_cls_sep=True)
            b = oracle.encode_threads(kind, data, offs, threads=threads, k=k, add_cls_sep=True)
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
            W = int(np.diff(a[1]).max()) + 3
            for side in (oracle.RIGHT, oracle.LEFT):
                p = oracle.pad(a[0], a[1], W, side)
                q = oracle.pad_threads(a[0], a[1], W, side, threads=threads)
                assert np.array_equal(p[0], q[0]) and np.array_equal(p[1], q[1])
    cuts = oracle.split_rows(offs, 7)
    assert cuts[0] == 0 and cuts[-1] == len(offs) - 1 and all(x < y for x, y in zip(cuts, cuts[1:]))
    e = oracle.encode_threads(oracle.SINGLE, data[:0], np.zeros(1, np.int64), threads=4)
    assert e[0].size == 0 and np.array_equal(e[1], [0])
