"""The benchmark's count of ranks a BPE row applies (read from the output
alone, through the merge trees of its final tokens) against a plain serial
merge that records every rank it applies, on a trained table."""
import numpy as np

import bench
import oracle
import synth


def _applied_ranks(row, merges):
    """Merge the lowest-ranked pair everywhere (leftmost first) until none is
    in the table; the set of ranks merged."""
    table = {(int(a), int(b)): r for r, (a, b) in enumerate(merges)}
    s = [{65: 5, 67: 6, 71: 7, 84: 8}[int(c)] for c in row]
    used = set()
    while True:
        ranks = [table.get((s[i], s[i + 1])) for i in range(len(s) - 1)]
        present = [r for r in ranks if r is not None]
        if not present:
            return used
        r = min(present)
        used.add(r)
        out, i = [], 0
        while i < len(s):
            if i + 1 < len(s) and ranks[i] == r:
                out.append(10 + r)
                i += 2
            else:
                out.append(s[i])
                i += 1
        s = out


def test_ranks_per_row_equal_a_recording_merge():
    corpus = synth.genome(synth.substream(61, 0), synth.substream(61, 1), 3, 100_000)
    merges = oracle.bpe_train(corpus, 200)
    rng = np.random.default_rng(5)
    lens = rng.integers(0, 400, 40)
    data = np.frombuffer(b"ACGT", np.uint8)[rng.integers(0, 4, int(lens.sum()))]
    offs = synth.offsets_from_lengths(lens)
    ids, out_off = oracle.encode(oracle.BPE, data, offs, merges=merges)
    got = bench._bpe_ranks(ids, out_off, merges)
    want = [len(_applied_ranks(data[offs[i]:offs[i + 1]], merges)) for i in range(len(lens))]
    assert got.tolist() == want
    assert max(want) > 20  # rows long enough to apply many ranks
