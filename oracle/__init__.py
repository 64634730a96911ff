"""CPU oracle for the DNA byte->identifier tokenizer.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. The GPU library
(``paper_2601_05531_amd``) never imports, links or calls it, and the two share
no code: the oracle's rules are written out in ``oracle.c`` and
``bpe_train.c`` (plain C loops) and in ``brute.py`` (pure-Python brute force
for tiny inputs).

Every function here is a ctypes wrapper around the C oracle; see the header
comment of ``oracle.c`` for the rules and the paper passages they follow.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

SINGLE, LUT256, KMER, BPE = 0, 1, 2, 3
PACKED, PADDED = 0, 1
RIGHT, LEFT = 0, 1
PAD, UNK, CLS, SEP, MASK = 0, 1, 2, 3, 4

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "bpe_train.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle (gcc -O2, no vector intrinsics)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp] + _SRCS)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        vp = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        lib.oracle_encode.restype = i64
        lib.oracle_encode.argtypes = [ctypes.c_int, ctypes.c_int, vp, i32, i32, vp, i32,
                                      vp, vp, i32, ctypes.c_int, vp, i64, vp]
        lib.oracle_revcomp.restype = ctypes.c_int
        lib.oracle_revcomp.argtypes = [vp, vp, i32, vp]
        lib.oracle_encode_overlap.restype = i64
        lib.oracle_encode_overlap.argtypes = [ctypes.c_int, vp, vp, i32, ctypes.c_int, vp, i64, vp]
        lib.oracle_pad.restype = ctypes.c_int
        lib.oracle_pad.argtypes = [vp, vp, i32, i64, ctypes.c_int, i32, vp, vp]
        lib.oracle_decode.restype = i64
        lib.oracle_decode.argtypes = [ctypes.c_int, ctypes.c_int, vp, i32, vp, vp, i32, vp, i64, vp]
        lib.oracle_bpe_check.restype = i32
        lib.oracle_bpe_check.argtypes = [vp, i32]
        lib.oracle_bpe_train.restype = i32
        lib.oracle_bpe_train.argtypes = [vp, i64, i32, vp]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


def encode(kind: int, data, offsets, k: int = 1, lut=None, merges=None, add_cls_sep: bool = False,
           cls_id: int = CLS, sep_id: int = SEP):
    """PACKED encode. Returns (ids int32[total], out_offsets int64[n+1])."""
    data = _c(data, np.uint8)
    offsets = _c(offsets, np.int64)
    lut = _c(lut, np.int32)
    merges = _c(merges, np.int32) if merges is not None else np.zeros((0, 2), np.int32)
    n = len(offsets) - 1
    cap = int(offsets[-1] - offsets[0]) + 2 * n + 1 if n > 0 else 1
    ids = np.empty(cap, dtype=np.int32)
    out_off = np.empty(n + 1, dtype=np.int64)
    total = _load().oracle_encode(kind, k, _ptr(lut), cls_id, sep_id, _ptr(merges), len(merges),
                                  _ptr(data), _ptr(offsets), n, int(add_cls_sep), _ptr(ids), cap, _ptr(out_off))
    if total < 0:
        raise ValueError("oracle_encode failed (%d)" % total)
    return ids[:total].copy(), out_off


def split_rows(offsets, parts: int):
    """Cut rows [0, n) into at most ``parts`` contiguous ranges of about equal
    bytes (a static partition of the sequences by bytes). Returns the range
    bounds as a list of row indices [r0 = 0, r1, ..., n]."""
    offsets = np.asarray(offsets, dtype=np.int64)
    n = len(offsets) - 1
    if n <= 0 or parts <= 1:
        return [0, max(n, 0)]
    span = int(offsets[-1] - offsets[0])
    cuts = [0]
    for p in range(1, parts):
        r = int(np.searchsorted(offsets, offsets[0] + span * p // parts, side="left"))
        r = min(max(r, cuts[-1]), n)
        if r > cuts[-1]:
            cuts.append(r)
    if cuts[-1] != n:
        cuts.append(n)
    return cuts


def encode_threads(kind: int, data, offsets, threads: int | None = None, **kw):
    """``encode`` with rows split into contiguous ranges of about equal bytes,
    one range per thread (the C oracle runs unchanged in each; ctypes releases
    the interpreter lock during the call). Same result as ``encode``."""
    from concurrent.futures import ThreadPoolExecutor
    data = _c(data, np.uint8)
    offsets = _c(offsets, np.int64)
    threads = threads or os.cpu_count() or 1
    cuts = split_rows(offsets, threads)
    if len(cuts) <= 2:
        return encode(kind, data, offsets, **kw)
    with ThreadPoolExecutor(max_workers=len(cuts) - 1) as ex:
        parts = list(ex.map(lambda j: encode(kind, data, offsets[cuts[j]:cuts[j + 1] + 1], **kw),
                            range(len(cuts) - 1)))
    ids = np.concatenate([p[0] for p in parts])
    out_off = np.empty(len(offsets), dtype=np.int64)
    base = 0
    for j, (pi, po) in enumerate(parts):
        out_off[cuts[j]:cuts[j + 1] + 1] = po + base
        base += int(po[-1])
    return ids, out_off


def pad_threads(ids, out_offsets, width: int, side: int = RIGHT, pad_id: int = PAD, threads: int | None = None):
    """``pad`` with rows split into contiguous ranges, one per thread."""
    from concurrent.futures import ThreadPoolExecutor
    out_offsets = _c(out_offsets, np.int64)
    threads = threads or os.cpu_count() or 1
    cuts = split_rows(out_offsets, threads)
    if len(cuts) <= 2:
        return pad(ids, out_offsets, width, side, pad_id)

    def one(j):
        o = out_offsets[cuts[j]:cuts[j + 1] + 1]
        return pad(ids[o[0]:o[-1]], o - o[0], width, side, pad_id)

    with ThreadPoolExecutor(max_workers=len(cuts) - 1) as ex:
        parts = list(ex.map(one, range(len(cuts) - 1)))
    return np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts])


def revcomp(data, offsets):
    """Reverse complement of every row (A<->T, C<->G, case kept, other bytes
    unchanged; rows stay at their offsets). Returns uint8[len(data)]."""
    data = _c(data, np.uint8)
    offsets = _c(offsets, np.int64)
    out = data.copy()
    if _load().oracle_revcomp(_ptr(data), _ptr(offsets), len(offsets) - 1, _ptr(out)) != 0:
        raise ValueError("offsets decrease")
    return out


def encode_overlap(data, offsets, k: int, add_cls_sep: bool = False):
    """PACKED encode with overlapping k-mers (stride 1). Returns (ids, out_offsets)."""
    data = _c(data, np.uint8)
    offsets = _c(offsets, np.int64)
    n = len(offsets) - 1
    cap = int(offsets[-1] - offsets[0]) + 2 * n + 1 if n > 0 else 1
    ids = np.empty(cap, dtype=np.int32)
    out_off = np.empty(n + 1, dtype=np.int64)
    total = _load().oracle_encode_overlap(k, _ptr(data), _ptr(offsets), n, int(add_cls_sep), _ptr(ids), cap,
                                          _ptr(out_off))
    if total < 0:
        raise ValueError("oracle_encode_overlap failed (%d)" % total)
    return ids[:total].copy(), out_off


def embed(table, ids):
    """Embedding lookup, the paper's embed_tokens applied to identifiers (Design,
    the embedder mapping B x T identifiers to B x T x D activations): row r
    of the result is row ids[r] of ``table`` (any dtype, copied bit for bit).
    ``ids`` may have any shape; the result has shape ids.shape + (D,)."""
    table = np.asarray(table)
    ids = np.asarray(ids, dtype=np.int64)
    if ids.size and (ids.min() < 0 or ids.max() >= table.shape[0]):
        raise ValueError("id outside the table")
    return table[ids]


def pad(ids, out_offsets, width: int, side: int = RIGHT, pad_id: int = PAD):
    """PACKED -> PADDED. Returns (ids int32[n, W], mask int8[n, W])."""
    ids = _c(ids, np.int32)
    out_offsets = _c(out_offsets, np.int64)
    n = len(out_offsets) - 1
    out = np.empty((n, width), dtype=np.int32)
    mask = np.empty((n, width), dtype=np.int8)
    rc = _load().oracle_pad(_ptr(ids), _ptr(out_offsets), n, width, side, pad_id, _ptr(out), _ptr(mask))
    if rc != 0:
        raise ValueError("a row is longer than the pad width")
    return out, mask


def decode(kind: int, ids, offsets, k: int = 1, merges=None):
    """Decode PACKED rows. Returns (bytes uint8[total], out_offsets int64[n+1])."""
    ids = _c(ids, np.int32)
    offsets = _c(offsets, np.int64)
    merges = _c(merges, np.int32) if merges is not None else np.zeros((0, 2), np.int32)
    n = len(offsets) - 1
    widest = max(k, 1)
    if kind == BPE and len(merges):
        widest = max(widest, max_merge_len(merges))
    cap = max(1, int(offsets[-1] - offsets[0]) * widest)
    out = np.empty(cap, dtype=np.uint8)
    out_off = np.empty(n + 1, dtype=np.int64)
    total = _load().oracle_decode(kind, k, _ptr(merges), len(merges), _ptr(ids), _ptr(offsets), n,
                                  _ptr(out), cap, _ptr(out_off))
    if total < 0:
        raise ValueError("oracle_decode failed (%d)" % total)
    return out[:total].copy(), out_off


def max_merge_len(merges) -> int:
    merges = np.asarray(merges, dtype=np.int64)
    lens = np.ones(10 + len(merges), dtype=np.int64)
    for r, (a, b) in enumerate(merges):
        lens[10 + r] = lens[a] + lens[b]
    return int(lens.max()) if len(lens) else 1


def bpe_check(merges) -> int:
    merges = _c(merges, np.int32).reshape(-1, 2)
    return int(_load().oracle_bpe_check(_ptr(merges), len(merges)))


def bpe_train(corpus, n_merges: int) -> np.ndarray:
    """Learn up to ``n_merges`` ranked merges (int32[R', 2]) from one DNA string."""
    corpus = _c(corpus, np.uint8)
    out = np.zeros((max(n_merges, 1), 2), dtype=np.int32)
    got = _load().oracle_bpe_train(_ptr(corpus), corpus.size, n_merges, _ptr(out))
    if got < 0:
        raise ValueError("oracle_bpe_train failed (%d)" % got)
    return out[:got].copy()


def fallback_lut() -> np.ndarray:
    """The discovery algorithm's fixed-DNA fallback table: A/a->1, C/c->2,
    G/g->3, T/t->4, N/n->0, every other byte->0 (paper, Design, discovery
    algorithm, the branch taken when no tokenizer is present)."""
    lut = np.zeros(256, dtype=np.int32)
    for ch, v in (("A", 1), ("C", 2), ("G", 3), ("T", 4), ("N", 0)):
        lut[ord(ch)] = v
        lut[ord(ch.lower())] = v
    return lut


def windows(record_lengths, window: int) -> np.ndarray:
    """Offsets of the windows a stream of records is cut into: each record is
    split into pieces of ``window`` bases from its own start, the last piece
    of a record being shorter."""
    offs = [0]
    pos = 0
    for L in record_lengths:
        L = int(L)
        start = 0
        while start < L:
            step = min(window, L - start)
            pos += step
            start += step
            offs.append(pos)
    return np.asarray(offs, dtype=np.int64)
