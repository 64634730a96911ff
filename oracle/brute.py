"""Pure-Python brute force for tiny inputs (TEST INFRASTRUCTURE ONLY).

These functions are deliberately written differently from ``oracle.c`` so that
the two pin each other:

* k-mer ids go through Python's own base conversion (``int(s, 4)``);
* BPE applies ONE merge per step, the leftmost occurrence of the lowest-rank
  pair (the per-occurrence form of ranked-merge BPE), where ``oracle.c``
  replaces every occurrence of the lowest-rank pair per round (Sennrich et
  al.'s form). For well-formed merge tables both give one segmentation;
* the BPE trainer recounts all pairs from scratch every step;
* the reverse complement goes through ``str.translate`` and slicing, the
  overlapping k-mers through string slices, the embedding lookup through a
  loop over rows.
"""
from __future__ import annotations

from collections import Counter

_DIGIT = str.maketrans("ACGTacgt", "01230123")
_BASE = {"A": 5, "C": 6, "G": 7, "T": 8}


def kmer_id(s: str) -> int:
    """Id of a full ACGT k-mer: 5 + its value as a base-4 numeral, A=0 .. T=3."""
    return 5 + int(s.translate(_DIGIT), 4)


def bpe_leftmost(symbols, merges):
    """Ranked-merge BPE on one ACGT run, one merge at a time.

    ``symbols``: list of ids. ``merges``: list of (left, right) by rank.
    Each step merges the leftmost occurrence of the lowest-ranked adjacent pair.
    """
    rank = {(int(a), int(b)): r for r, (a, b) in enumerate(merges)}
    sym = list(symbols)
    while True:
        best = None
        for p in range(len(sym) - 1):
            r = rank.get((sym[p], sym[p + 1]))
            if r is not None and (best is None or r < best[0]):
                best = (r, p)
        if best is None:
            return sym
        r, p = best
        sym[p:p + 2] = [10 + r]


def bpe_encode_text(text: str, merges):
    """BPE body of one row: runs of ACGT segmented, N -> 9, other -> UNK (1)."""
    out, run = [], []
    for ch in text:
        u = ch.upper()
        if u in _BASE:
            run.append(_BASE[u])
            continue
        if run:
            out += bpe_leftmost(run, merges)
            run = []
        out.append(9 if u == "N" else 1)
    if run:
        out += bpe_leftmost(run, merges)
    return out


def bpe_train_recount(corpus: str, n_merges: int):
    """Greedy BPE learner recounting every pair each step (tiny corpora only).

    Pairs never cross a non-ACGT byte; ties go to the smallest (left, right);
    stops when the best count is below 2; each step replaces every
    non-overlapping occurrence left to right.
    """
    runs, cur = [], []
    for ch in corpus:
        u = ch.upper()
        if u in _BASE:
            cur.append(_BASE[u])
        else:
            if cur:
                runs.append(cur)
            cur = []
    if cur:
        runs.append(cur)
    merges = []
    for r in range(n_merges):
        counts = Counter()
        for run in runs:
            for p in range(len(run) - 1):
                counts[(run[p], run[p + 1])] += 1
        if not counts:
            break
        best = min(counts.items(), key=lambda kv: (-kv[1], kv[0]))
        if best[1] < 2:
            break
        a, b = best[0]
        merges.append((a, b))
        new_runs = []
        for run in runs:
            out, p = [], 0
            while p < len(run):
                if p + 1 < len(run) and run[p] == a and run[p + 1] == b:
                    out.append(10 + r)
                    p += 2
                else:
                    out.append(run[p])
                    p += 1
            new_runs.append(out)
        runs = new_runs
    return merges, runs


def expand(tok: int, merges) -> str:
    """Uppercase string a BPE / SINGLE id stands for."""
    if 5 <= tok <= 8:
        return "ACGT"[tok - 5]
    if tok == 9:
        return "N"
    if tok >= 10:
        a, b = merges[tok - 10]
        return expand(int(a), merges) + expand(int(b), merges)
    raise ValueError(tok)


_COMP = str.maketrans("ACGTacgt", "TGCAtgca")


def revcomp_text(text: str) -> str:
    """Reverse complement of one row (A<->T, C<->G, case kept, others kept)."""
    return text.translate(_COMP)[::-1]


def kmer_body_text(text: str, k: int):
    """Non-overlapping k-mer body of one row (frames from base 0, stride k)."""
    out = []
    for s in range(0, len(text), k):
        w = text[s:s + k]
        ok = len(w) == k and all(ch in "ACGTacgt" for ch in w)
        out.append(kmer_id(w) if ok else 1)
    return out


def overlap_body_text(text: str, k: int):
    """Overlapping k-mer body of one row: one window per start s <= L - k;
    a non-empty row shorter than k is one UNK."""
    if 0 < len(text) < k:
        return [1]
    out = []
    for s in range(len(text) - k + 1):
        w = text[s:s + k]
        out.append(kmer_id(w) if all(ch in "ACGTacgt" for ch in w) else 1)
    return out


def embed_rows(table_rows, ids):
    """List of table rows picked by ids, one by one."""
    return [table_rows[i] for i in ids]
