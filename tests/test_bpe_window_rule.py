"""The rule the BPE wave kernel uses to merge several ranks in one round,
modelled on the CPU and checked against the oracle's one-rank-at-a-time
merge: the ranks present in a window above the lowest one are applied
together up to the first step where occurrences of two steps share a symbol
or a pair formed before the last step ranks at or below a later step's rank;
a list cap narrows the window, and a single rank over the cap is taken in
chunks of the sequence, each from the state the previous chunk left.
Random well-formed tables rich in (X, X) pairs, on run- and repeat-rich rows."""
import bisect

import numpy as np

import oracle

NO = 1 << 30
ACGT = np.frombuffer(b"ACGT", np.uint8)


def _occurrences(rk, r, chain):
    out, last = [], -10
    for i, x in enumerate(rk):
        if x == r and not (chain and i == last + 1):
            out.append(i)
            last = i
    return out


def _apply(s, merges_at, ranks):
    out, i = [], 0
    while i < len(s):
        if i in merges_at:
            out.append(10 + ranks[merges_at[i]])
            i += 2
        else:
            out.append(s[i])
            i += 1
    return out


def _windowed(sym, table, merges, width, cap, chunk):
    s = list(sym)
    rank = lambda a, b: table.get((a, b), NO)
    while True:
        rk = [rank(s[i], s[i + 1]) for i in range(len(s) - 1)]
        if not rk or min(rk) >= NO:
            return s
        rs = min(rk)
        d = width
        while d > 1 and sum(1 for x in rk if rs <= x < rs + d) > cap:
            d = max(1, d // 4)
        if sum(1 for x in rk if x == rs) > cap:
            # one rank in chunks: each chunk's occurrences from the current state
            start = 0
            while True:
                rk = [rank(s[i], s[i + 1]) for i in range(len(s) - 1)]
                occ = [i for i in _occurrences(rk, rs, merges[rs][0] == merges[rs][1]) if i >= start]
                if not occ:
                    break
                take = occ[:chunk]
                end = take[-1] + 1
                s = _apply(s, {i: 0 for i in take}, [rs])
                start = end - len(take)  # positions shift left by one per merge
            continue
        ranks = sorted(set(x for x in rk if rs <= x < rs + d))
        at = {}
        for st, r in enumerate(ranks):
            for i in _occurrences(rk, r, merges[r][0] == merges[r][1]):
                at[i] = st
        cut, held = len(ranks), {}
        for i, st in sorted(at.items()):
            for x in (i, i + 1):
                if x in held and held[x] != st:
                    cut = min(cut, max(st, held[x]))
                held[x] = st
        bound = lambda st, r: max(st + 1, bisect.bisect_left(ranks, r))
        for i, st in at.items():
            new = 10 + ranks[st]
            if i >= 1 and (i - 1) not in at:
                if (i - 2) in at:
                    sj = at[i - 2]
                    if sj > st:
                        cut = min(cut, bound(st, rank(s[i - 1], new)))
                    cut = min(cut, bound(max(st, sj), rank(10 + ranks[sj], new)))
                else:
                    cut = min(cut, bound(st, rank(s[i - 1], new)))
            if i + 2 < len(s):
                if (i + 2) not in at:
                    cut = min(cut, bound(st, rank(new, s[i + 2])))
                elif at[i + 2] > st:
                    cut = min(cut, bound(st, rank(new, s[i + 2])))
        cut = max(cut, 1)
        s = _apply(s, {i: st for i, st in at.items() if st < cut}, ranks)


def _table(rng, R, p_chain):
    syms, merges, table = [5, 6, 7, 8], [], {}
    tries = 0
    while len(merges) < R and tries < 50 * R:
        tries += 1
        a = syms[int(rng.integers(len(syms)))]
        b = a if rng.random() < p_chain else syms[int(rng.integers(len(syms)))]
        if (a, b) not in table:
            table[(a, b)] = len(merges)
            merges.append((a, b))
            syms.append(10 + len(merges) - 1)
    return merges, table


def test_window_rule_equals_the_oracle():
    rng = np.random.default_rng(7)
    for case in range(300):
        merges, table = _table(rng, int(rng.integers(1, 80)), float(rng.choice([0.05, 0.3, 0.6])))
        n = int(rng.integers(0, 160))
        if case % 3 == 0:
            row = np.repeat(rng.integers(0, 4, n + 1), rng.integers(1, 9, n + 1))[:n]
        elif case % 3 == 1:
            motif = rng.integers(0, 4, int(rng.integers(1, 5)))
            row = np.tile(motif, n // len(motif) + 1)[:n]
        else:
            row = rng.integers(0, 4, n)
        data = ACGT[row].astype(np.uint8)
        want, _ = oracle.encode(oracle.BPE, data, np.array([0, n], np.int64),
                                merges=np.array(merges, np.int32).reshape(-1, 2))
        width, cap, chunk = (int(rng.choice([1, 2, 8, 64])), int(rng.choice([1, 3, 16, 256])),
                             int(rng.choice([1, 2, 5])))
        got = _windowed([5 + int(x) for x in row], table, merges, width, cap, chunk)
        assert got == want.tolist(), (case, width, cap, chunk)
