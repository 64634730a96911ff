"""Seeded synthetic DNA inputs shared by the oracle side and the GPU side.

This package only generates bytes, offsets, lengths and request traces. It
contains none of the tokenizer's arithmetic (no byte classes, no ids), so the
oracle and the HIP path can both consume its output without sharing any
method code.

The byte-level generators live in ``synth.c`` (a Markov chain walk cannot be
vectorised); length draws and Poisson traces use NumPy's PCG64 seeded per
purpose. Every generator is a pure function of its seed.

Workload recipes follow the paper's synthetic microbenchmarks (Results,
Experimental Setup: equal-length synthetic strings over a fixed nucleotide
alphabet, seed 42 per the system-configuration table) widened to ragged,
soft-masked, N-containing genomes as described in the module docstring of
``synth.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

BASE_SEED = 42
_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``synth.c`` into ``libsynth.so`` (plain gcc, -O2)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        u64, i64, dbl = ctypes.c_uint64, ctypes.c_int64, ctypes.c_double
        lib.synth_substream.restype = u64
        lib.synth_substream.argtypes = [u64, u64, u64]
        lib.synth_iid.argtypes = [u64, u8p, i64, dbl]
        lib.synth_markov.argtypes = [u64, u64, ctypes.c_int, u8p, i64, ctypes.POINTER(dbl)]
        lib.synth_softmask.argtypes = [u64, u8p, i64, dbl, dbl]
        lib.synth_nruns.argtypes = [u64, u8p, i64, dbl, dbl]
        lib.synth_invalid.argtypes = [u64, u8p, i64, dbl]
        lib.synth_bytes.argtypes = [u64, u8p, i64]
        lib.synth_raw.argtypes = [u64, ctypes.POINTER(u64), i64]
        _lib = lib
    return _lib


def _u8p(a: np.ndarray):
    assert a.dtype == np.uint8 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def substream(*keys: int, base: int = BASE_SEED) -> int:
    """Deterministic 64-bit seed for a (config, purpose, index) key path."""
    lib = _load()
    s = base & 0xFFFFFFFFFFFFFFFF
    for k in keys:
        s = lib.synth_substream(s, k & 0xFFFFFFFFFFFFFFFF, 0x5EED)
    return int(s)


def raw_u64(seed: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    _load().synth_raw(seed, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), n)
    return out


def iid(seed: int, n: int, p_n: float = 0.01, out: np.ndarray | None = None) -> np.ndarray:
    out = np.empty(n, dtype=np.uint8) if out is None else out
    _load().synth_iid(seed, _u8p(out), n, p_n)
    return out


def uniform_bytes(seed: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint8)
    _load().synth_bytes(seed, _u8p(out), n)
    return out


def markov(table_seed: int, seq_seed: int, order: int, n: int, out: np.ndarray | None = None) -> np.ndarray:
    out = np.empty(n, dtype=np.uint8) if out is None else out
    cum = np.empty(4 * (4 ** order), dtype=np.float64)
    _load().synth_markov(table_seed, seq_seed, order, _u8p(out), n,
                         cum.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def decorate(seed: int, buf: np.ndarray, mask_mean: float = 300.0, open_mean: float = 450.0,
             n_run_mean: float = 50.0, n_gap_mean: float = 2450.0, p_invalid: float = 1e-4) -> np.ndarray:
    """Soft-mask, N runs and invalid bytes applied in place (in that order)."""
    lib = _load()
    n = buf.size
    if mask_mean > 0:
        lib.synth_softmask(substream(seed, 1), _u8p(buf), n, mask_mean, open_mean)
    if n_run_mean > 0:
        lib.synth_nruns(substream(seed, 2), _u8p(buf), n, n_run_mean, n_gap_mean)
    if p_invalid > 0:
        lib.synth_invalid(substream(seed, 3), _u8p(buf), n, p_invalid)
    return buf


def genome(table_seed: int, seq_seed: int, order: int, n: int, decorated: bool = True,
           out: np.ndarray | None = None) -> np.ndarray:
    g = markov(table_seed, seq_seed, order, n, out=out)
    if decorated:
        decorate(seq_seed, g)
    return g


def loguniform_int(seed: int, n: int, lo: float, hi: float) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi), size=n))).astype(np.int64)


def offsets_from_lengths(lengths) -> np.ndarray:
    off = np.zeros(len(lengths) + 1, dtype=np.int64)
    np.cumsum(np.asarray(lengths, dtype=np.int64), out=off[1:])
    return off


# ----------------------------------------------------------------------------
# Workloads (sizes and distributions of the five benchmark configurations)
# ----------------------------------------------------------------------------

def workload_iid(n_seqs: int = 64, seq_len: int = 16384, p_n: float = 0.01, seed: int | None = None):
    """Equal-length i.i.d. sequences (small case: 64 x 16,384, 1% N)."""
    seed = substream(1, 0) if seed is None else seed
    data = iid(seed, n_seqs * seq_len, p_n)
    return data, offsets_from_lengths([seq_len] * n_seqs)


def workload_markov_batch(n_seqs: int = 4096, seq_len: int = 8192, seed: int | None = None):
    """Equal-length windows cut from one order-3 Markov genome with soft-masking
    (mean 300, 40% of bases), N runs (mean 50, 2%) and 1e-4 invalid bytes."""
    seed = substream(2, 0) if seed is None else seed
    g = genome(substream(2, 1), seed, 3, n_seqs * seq_len)
    return g, offsets_from_lengths([seq_len] * n_seqs)


def chromosome_lengths(total: int = 1 << 31, n: int = 16, lo: float = 1e7, hi: float = 2.5e8,
                       seed: int | None = None) -> np.ndarray:
    """Log-uniform draws on [lo, hi], rescaled to sum to exactly ``total``.

    Sixteen log-uniform draws on [1e7, 2.5e8] sum to about 1.2e9 on average,
    short of 2 GiB; the draws keep their proportions and are scaled up, the
    rounding remainder going to the longest one."""
    seed = substream(3, 0) if seed is None else seed
    raw = np.exp(np.random.default_rng(seed).uniform(np.log(lo), np.log(hi), size=n))
    lens = np.floor(raw / raw.sum() * total).astype(np.int64)
    lens[np.argmax(lens)] += total - int(lens.sum())
    return lens


def chromosomes(lengths, out: np.ndarray | None = None, threads: int = 16, seed: int | None = None) -> np.ndarray:
    """Concatenated chromosomes (order-3 Markov + decorations), generated in parallel."""
    seed = substream(3, 1) if seed is None else seed
    lengths = np.asarray(lengths, dtype=np.int64)
    total = int(lengths.sum())
    out = np.empty(total, dtype=np.uint8) if out is None else out
    starts = np.concatenate([[0], np.cumsum(lengths)])
    table = substream(2, 1)  # same genome model as the batched workload

    def one(i):
        seg = out[starts[i]:starts[i + 1]]
        genome(table, substream(seed, i), 3, int(lengths[i]), out=seg)

    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        list(ex.map(one, range(len(lengths))))
    return out


def bpe_corpus(n: int = 1 << 26, seed: int | None = None) -> np.ndarray:
    """Order-5 Markov genome, uppercase ACGT only (BPE trainer corpus)."""
    seed = substream(4, 0) if seed is None else seed
    return markov(substream(4, 1), seed, 5, n)


def workload_bpe_batch(n_seqs: int = 1024, lo: int = 500, hi: int = 20000, seed: int | None = None):
    """Ragged sequences with log-uniform lengths, fresh walk of the trainer's chain."""
    seed = substream(4, 2) if seed is None else seed
    lens = loguniform_int(substream(seed, 0), n_seqs, lo, hi)
    data = markov(substream(4, 1), substream(seed, 1), 5, int(lens.sum()))
    return data, offsets_from_lengths(lens)


def serving_trace(n_requests: int = 20000, rate: float = 2000.0, lo: float = 100, hi: float = 1e6,
                  n_vocabs: int = 4, seed: int | None = None):
    """Poisson arrivals (exponential gaps at ``rate``), log-uniform sizes, uniform vocab index."""
    seed = substream(5, 0) if seed is None else seed
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n_requests))
    sizes = np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi), size=n_requests))).astype(np.int64)
    vocab = rng.integers(0, n_vocabs, size=n_requests)
    return arrivals, sizes, vocab
