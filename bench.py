"""Benchmark of the MI355X DNA byte->identifier tokenizer.

Prints ONE JSON line. The timed step is the device encode of the batched
k-mer workload: 4,096 sequences x 8,192 bases of a seeded order-3 Markov
genome (40% soft-masked, 2% N runs, 1e-4 invalid bytes), encoded as
non-overlapping k-mers for k = 3, 4, 5, 6 in one pass over the bytes (one
launch), CLS/SEP added, right-padded to the longest row, int32 ids plus int8
attention mask. Inputs are resident in HBM before timing starts; every step
reads a different input copy (24 copies, 768 MiB) and writes to one of 8
output sets (1.3 GB), so the 256 MB last-level cache cannot serve a repeat.
The same step as four single-vocabulary launches is reported beside it.

Extra objects on the same line:
  roofline      the encode kernel's algorithmic bytes per launch / its mean
                launch time (HIP events around each launch, on the launch
                stream) against 8 TB/s HBM;
  cpu_baseline  the CPU oracle (single thread, as written) on a bounded
                sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "tokens/s device encode + end-to-end H2D stream, % HBM/H2D peak; p50/p99 req latency"
HBM_PEAK_GBS = 8000.0
KS = (3, 4, 5, 6)
N_SEQS, SEQ_LEN = 4096, 8192
SETS = 8       # output sets
IN_SETS = 24   # input copies: 768 MiB of inputs, far beyond the 256 MB last-level cache


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def encode_leg(steps: int, warmup: int, tuning=None, per_vocab: bool = True):
    import torch
    import paper_2601_05531_amd as dt
    import synth

    data, offs = synth.workload_markov_batch(N_SEQS, SEQ_LEN)
    n = len(offs) - 1
    vocabs = {k: dt.Vocab(dt.KMER, k=k) for k in KS}
    plans = {k: dt.plan(vocabs[k], offs, add_cls_sep=True) for k in KS}  # (total, max_len)
    d_offs = torch.from_numpy(offs).cuda()
    d_in = [torch.from_numpy(data).cuda() for _ in range(IN_SETS)]
    outs = []
    for s in range(SETS):
        o = {}
        for k in KS:
            W = plans[k][1]
            o[k] = (torch.empty(n * W, dtype=torch.int32, device="cuda"),
                    torch.empty(n + 1, dtype=torch.int64, device="cuda"),
                    torch.empty(n * W, dtype=torch.int8, device="cuda"))
        outs.append(o)
    opts = {k: dt.make_opts(add_cls_sep=True, layout=dt.PADDED, pad_side=dt.PAD_RIGHT, pad_to=plans[k][1])
            for k in KS}
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    nbytes = data.size
    tokens_per_step = sum(plans[k][0] for k in KS)

    # The step: the batch for k = 3, 4, 5, 6 in one pass over its bytes (one
    # launch); step s reads input copy s % 24 and writes output set s % 8.
    vlist = [vocabs[k] for k in KS]
    calls = [dt.MultiCall(vlist, d_in[s], d_offs, [outs[s % SETS][k] for k in KS], [opts[k] for k in KS])
             for s in range(IN_SETS)]
    if tuning is None:
        tune_multi, tune_ms = calls[0].autotune(reps=3)
        log("autotuned (one pass, k=3..6): %s %.4f ms" % (tune_multi, tune_ms))
    else:
        dt.set_tuning(vocabs[KS[0]], tile_bytes=tuning[0], blocks_per_cu=tuning[1],
                      bands=tuning[2] if len(tuning) > 2 else 0)
        tune_multi = dt.dnatok_get_tuning(vocabs[KS[0]].handle).as_dict()
        log("tiling set: %s" % tune_multi)
    for s in range(warmup):
        calls[s % IN_SETS].run(stream)
    torch.cuda.synchronize()
    assert dt.sync_status() == 0
    # HIP events on the launch stream bracket the K back-to-back launches:
    # their span / K is the average launch duration (an event pair around
    # each launch would add its own release and timestamp to every launch)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for s in range(steps):
        calls[s % IN_SETS].run(stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    flags = dt.sync_status()
    if flags:
        raise RuntimeError("device error flags %d during the timed region" % flags)
    elapsed = t1 - t0
    launch_ms = ev0.elapsed_time(ev1) / steps
    # algorithmic bytes of one launch: the input once, its offsets once, and
    # per vocabulary the ids + mask of every cell and the output offsets
    bytes_launch = nbytes + 8 * (n + 1) + sum(8 * (n + 1) + 5 * n * plans[k][1] for k in KS)
    achieved = bytes_launch / (launch_ms * 1e-3) / 1e9
    for k in KS:  # oracle-free invariant on the last output set: sum(mask) == tokens
        assert int(outs[(steps - 1) % SETS][k][2].sum().item()) == plans[k][0]

    res = {
        "tokens_per_step": tokens_per_step,
        "ms_per_step": elapsed / steps * 1e3,
        "value": tokens_per_step * steps / elapsed,
        "launch_ms": launch_ms,
        "bytes_per_launch": bytes_launch,
        "bytes_written_per_launch": sum(8 * (n + 1) + 5 * n * plans[k][1] for k in KS),
        "tuning": tune_multi,
        "per_vocab": None,
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(kernel_family(tune_multi)),
            "kernel": {"k_bands": "k_bands<KMER> (row bands, %d-byte stage)" % tune_multi["tile_bytes"],
                       "k_bands_loop": "k_bands_loop<KMER> (row bands, resident workgroups, %d-byte stage)"
                                       % tune_multi["tile_bytes"],
                       "k_cells": "k_cells<KMER> (tiles)"}[kernel_family(tune_multi)] +
                      " writing k = 3, 4, 5, 6 in one pass",
            "per_launch_bytes": "1 B per input byte (read once) + 16 B per row of offsets + per vocabulary "
                                "5 B per cell (4 B id + 1 B mask over n x pad_to) = %d B" % bytes_launch,
        },
        "data": data,
        "offs": offs,
    }
    log("encode (one pass, k=3..6): %.3e tokens/s, %.4f ms/step (launch %.4f ms, %.0f GB/s)" % (
        res["value"], res["ms_per_step"], launch_ms, achieved))
    if not per_vocab:
        return res

    # Reference: the same step as four single-vocabulary launches, each tiled
    # by the autotuner for its own k.
    tuning = {}
    for k in KS:
        t, ms = dt.autotune(vocabs[k], d_in[0], d_offs, h_offsets=offs, add_cls_sep=True, layout=dt.PADDED,
                            pad_to=plans[k][1], reps=3)
        tuning[k] = {"tile_bytes": t["tile_bytes"], "blocks_per_cu": t["blocks_per_cu"], "median_ms": round(ms, 4)}

    def launch(step, j, k):
        x = d_in[(4 * step + j) % IN_SETS]
        ids, oo, mk = outs[step % SETS][k]
        dt.dnatok_encode(vocabs[k].handle, x.data_ptr(), nbytes, d_offs.data_ptr(), n, ids.data_ptr(), ids.numel(),
                         oo.data_ptr(), mk.data_ptr(), opts[k], sp)

    for s in range(warmup):
        for j, k in enumerate(KS):
            launch(s, j, k)
    torch.cuda.synchronize()
    ev4 = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in KS]
           for _ in range(steps)]
    torch.cuda.synchronize()
    u0 = time.perf_counter()
    for s in range(steps):
        for j, k in enumerate(KS):
            a, b = ev4[s][j]
            a.record(stream)
            launch(s, j, k)
            b.record(stream)
    torch.cuda.synchronize()
    u1 = time.perf_counter()
    assert dt.sync_status() == 0
    per_k_ms = {k: float(np.mean([ev4[s][j][0].elapsed_time(ev4[s][j][1]) for s in range(steps)]))
                for j, k in enumerate(KS)}
    bytes_k = {k: nbytes + 16 * (n + 1) + 5 * n * plans[k][1] for k in KS}
    achieved_k = sum(bytes_k.values()) / (sum(per_k_ms.values()) * 1e-3) / 1e9
    res["per_vocab"] = {
        "value": tokens_per_step * steps / (u1 - u0),
        "ms_per_step": (u1 - u0) / steps * 1e3,
        "per_k_launch_ms": per_k_ms,
        "autotuned": tuning,
        "achieved_GBps": round(achieved_k, 1),
    }
    log("encode (four launches): %.3e tokens/s, per-launch ms %s" % (res["per_vocab"]["value"], per_k_ms))
    return res


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "encode_multi_k_batch_traffic.md")


def kernel_family(tune) -> str:
    """The kernel a tiling of the batched workload runs: row bands (1),
    resident row bands (3; a stage over 8 KiB holds two 8,192-byte rows,
    more than the resident form stages, and runs as row bands), else tiles."""
    b, tile = tune.get("bands", 0), tune.get("tile_bytes", 0)
    if b == 3 and tile <= 8192:
        return "k_bands_loop"
    return "k_bands" if b in (1, 3) else "k_cells"


def measured_traffic(family: str):
    """HBM bytes per launch of the one-pass encode from the committed counter
    summary (FETCH_SIZE / WRITE_SIZE calibrated by a copy of known size), or
    None when the summary is missing, was taken on another kernel than the
    one this run's tiling selects (tiles, row bands, resident row bands), or
    the kernel source changed since."""
    import hashlib
    try:
        text = open(TRAFFIC_SUMMARY).read()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if ":" in line and line.startswith("    "):
            key, val = line.strip().split(":", 1)
            fields[key.strip()] = val.strip()
    try:
        if fields["kernel"].split("<")[0] != family:
            return None
        src = os.path.join(ROOT, fields["kernel_source"])
        if hashlib.sha256(open(src, "rb").read()).hexdigest() != fields["kernel_source_sha256"]:
            return None
        return int(fields["traffic_bytes_per_launch"])
    except (KeyError, OSError, ValueError):
        return None


def copy_leg(sizes=(45 << 20, 1 << 30), reps: int = 20, encode_bytes: int = 0, fill_bytes: int = 0):
    """Plain device-to-device copies (torch's copy kernel), timed like the
    encode (events around back-to-back launches): the practical HBM rate at the encode's
    traffic size (45 MiB copy = 90 MiB moved, about one k=3 launch; a copy
    moving the bytes of one multi-k encode launch) and in steady state
    (1 GiB), and the reference that calibrates the FETCH_SIZE / WRITE_SIZE
    counters (2 * size bytes per copy). Also a write-only fill of as many
    bytes as the multi-k encode writes. Buffers rotate over four copies so
    no launch finds its data in the 256 MB last-level cache."""
    import torch
    out = {}
    if fill_bytes:
        bufs = [torch.empty(fill_bytes, dtype=torch.uint8, device="cuda") for _ in range(4)]
        for i in range(3):
            bufs[i].fill_(1)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for i in range(reps):
            bufs[i % 4].fill_(i & 127)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        out["fill_%d_B" % fill_bytes] = {"ms": round(ms, 5), "GBps": round(fill_bytes / (ms * 1e-3) / 1e9, 1)}
        del bufs
    if encode_bytes:
        sizes = (sizes[0], encode_bytes // 2) + tuple(sizes[1:])
    for nbytes in sizes:
        srcs = [torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(7) for _ in range(4)]
        dsts = [torch.empty(nbytes, dtype=torch.uint8, device="cuda") for _ in range(4)]
        for i in range(3):
            dsts[i % 4].copy_(srcs[i % 4])
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for i in range(reps):
            dsts[i % 4].copy_(srcs[(i + 1) % 4])
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        key = "%d_MiB" % (nbytes >> 20) if nbytes % (1 << 20) == 0 else "%d_B" % nbytes
        out[key] = {"ms": round(ms, 5), "GBps": round(2 * nbytes / (ms * 1e-3) / 1e9, 1)}
        del srcs, dsts
    return out


STREAM_BYTES = 1 << 31
STREAM_CHUNK = 64 << 20
STREAM_WINDOW = 6000
STREAM_K = 6


def _h2d_passes(h, passes: int):
    """Pinned host -> device copy rate (copy engine): 64 MiB copies of the
    whole buffer back to back into a 3-slot device ring, one rate per pass."""
    import torch
    ring = [torch.empty(STREAM_CHUNK, dtype=torch.uint8, device="cuda") for _ in range(3)]
    rates = []
    for p in range(passes):
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for i, c0 in enumerate(range(0, STREAM_BYTES, STREAM_CHUNK)):
            ring[i % 3].copy_(h[c0:c0 + STREAM_CHUNK], non_blocking=True)
        b.record()
        torch.cuda.synchronize()
        rates.append(STREAM_BYTES / (a.elapsed_time(b) * 1e-3) / 1e9)
    del ring
    return rates


def stream_leg(passes: int = 5):
    """End-to-end pinned host -> device stream: 2 GiB of synthetic chromosomes
    (16 records, log-uniform lengths scaled to 2 GiB, same genome model as
    the batched workload) pushed in 64 MiB chunks, cut into 6000-base windows
    and encoded as 6-mers on the device, overlapped and sequential. Both the
    stream and the plain pinned H2D rate of the same buffer take the best of
    ``passes`` passes; the H2D passes run before and after the stream, and
    the denominator is the best of all of them. Returns (summary, the host
    buffer and record lengths, the overlapped stream's ids on the host)."""
    import torch
    import paper_2601_05531_amd as dt
    import synth

    lens = synth.chromosome_lengths(total=STREAM_BYTES)
    t0 = time.perf_counter()
    h = torch.empty(STREAM_BYTES, dtype=torch.uint8, pin_memory=True)
    synth.chromosomes(lens, out=h.numpy())
    log("stream: generated %d bytes of chromosomes in %.1f s" % (STREAM_BYTES, time.perf_counter() - t0))
    starts = np.concatenate([[0], np.cumsum(lens)])
    n_windows = int(sum(-(-int(L) // STREAM_WINDOW) for L in lens))
    n_tokens = 0
    for L in lens:
        full, rem = divmod(int(L), STREAM_WINDOW)
        n_tokens += full * (-(-STREAM_WINDOW // STREAM_K)) + (-(-rem // STREAM_K))

    before = _h2d_passes(h, passes)
    v = dt.Vocab(dt.KMER, k=STREAM_K)
    out = {"bytes": STREAM_BYTES, "windows": n_windows, "tokens": n_tokens, "chunk_bytes": STREAM_CHUNK,
           "slots": 3, "passes": passes}
    sample_ok = None
    got_ids = None
    runs = {}
    for mode, overlap in (("overlap", True), ("baseline", False)):
        st = dt.Stream(v, STREAM_WINDOW, STREAM_CHUNK, n_tokens, n_windows, n_slots=3, overlap=overlap)
        times = []
        for rep in range(passes):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for c0 in range(0, STREAM_BYTES, STREAM_CHUNK):
                c1 = c0 + STREAM_CHUNK
                ends = starts[1:][(starts[1:] > c0) & (starts[1:] <= c1)] - c0
                st.push(h[c0:c1], ends)
            ids, woff, r = st.flush(copy=False)
            times.append(time.perf_counter() - t0)
            assert r.n_tokens == n_tokens and r.n_windows == n_windows
            if sample_ok is None:
                sample_ok = _stream_window_check(lens, woff, n_windows)
            if overlap and rep == passes - 1:
                got_ids = ids.cpu().numpy()
            if rep < passes - 1:
                st.reset()
        st.close()
        runs[mode] = times
    after = _h2d_passes(h, passes)
    h2d = max(before + after)
    out["h2d"] = {"best_GBps": round(h2d, 2), "median_GBps": round(float(np.median(before + after)), 2),
                  "before_GBps": [round(x, 2) for x in before], "after_GBps": [round(x, 2) for x in after]}
    for mode, times in runs.items():
        t = min(times)
        out[mode] = {"s": round(t, 4), "tokens_per_s": n_tokens / t, "GBps": round(STREAM_BYTES / t / 1e9, 2),
                     "median_GBps": round(STREAM_BYTES / float(np.median(times)) / 1e9, 2),
                     "frac_of_h2d": round(STREAM_BYTES / t / 1e9 / h2d, 4)}
        log("stream %s: %.3e tokens/s, %.1f GB/s (%.0f%% of the best pinned H2D pass, %.1f GB/s)" % (
            mode, n_tokens / t, STREAM_BYTES / t / 1e9, 100 * STREAM_BYTES / t / 1e9 / h2d, h2d))
    out["window_offsets_check"] = sample_ok
    v.close()
    return out, (h, lens), got_ids


IDS_CONFIGS = ((4096, 512), (8192, 512), (2048, 2048))


def ids_leg(reps: int = 5, warmup: int = 2):
    """The paper's IDs path and its ablation (staging width x overlap) on its
    three microbenchmark shapes (B x T equal-length strings): host map
    through the single-nucleotide table into pinned staging, H2D per
    micro-batch (token budget 1,048,576), on-device widen for int32
    staging, and the embedding lookup (11 x 128 bf16 table, the paper's
    vocabulary size and width). Per arm: end-to-end tokens/s (wall clock from
    the host map to the last row written; best and median of ``reps``), the
    host map alone, and the H2D rate (staged bytes / the copies' event
    time)."""
    import torch
    import paper_2601_05531_amd as dt
    import synth

    v = dt.Vocab(dt.SINGLE)
    g = torch.Generator().manual_seed(42)
    table = torch.randn((11, 128), generator=g).to(torch.bfloat16).cuda()
    threads = _host_threads()
    out = {"workload": "B x T equal-length synthetic strings (order-3 Markov genome, soft-masked, N runs), "
                       "single-nucleotide table, embedding 11 x 128 bf16, token budget 1,048,576 per micro-batch, "
                       "%d host threads" % threads}
    for B, T in IDS_CONFIGS:
        rows = synth.genome(synth.substream(6, B), synth.substream(6, T), 3, B * T)
        h = torch.empty(B * T, dtype=torch.uint8, pin_memory=True)
        h.numpy()[:] = rows
        d_out = torch.empty((B, T, 128), dtype=torch.bfloat16, device="cuda")
        cfg = {}
        for width in (8, 4):
            for overlap in (False, True):
                p = dt.IdsPath(v, width=width, overlap=overlap, threads=threads)
                res = []
                for r in range(warmup + reps):
                    x = p.run(h, B, T, T, table=table, d_out=d_out)
                    if r >= warmup:
                        res.append(x)
                assert dt.sync_status() == 0
                p.close()
                tot = sorted(x.total_s for x in res)
                name = "%s_%s" % ("int32" if width == 4 else "int64", "pipelined" if overlap else "sequential")
                cfg[name] = {
                    "tokens_per_s": B * T / tot[0],
                    "median_tokens_per_s": B * T / float(np.median(tot)),
                    "host_map_tokens_per_s": B * T / min(x.map_s for x in res),
                    "h2d_GBps": round(max(x.h2d_bytes / x.h2d_s for x in res) / 1e9, 2),
                    "micro_batches": int(res[0].n_micro),
                }
        base = cfg["int64_sequential"]["tokens_per_s"]
        cfg["ablation_vs_baseline"] = {
            "baseline": 1.0,
            "int32_only": round(cfg["int32_sequential"]["tokens_per_s"] / base, 3),
            "overlap_only": round(cfg["int64_pipelined"]["tokens_per_s"] / base, 3),
            "both": round(cfg["int32_pipelined"]["tokens_per_s"] / base, 3),
        }
        out["B%d_T%d" % (B, T)] = cfg
        log("ids path B=%d T=%d: %s" % (B, T, {k: "%.3e" % v["tokens_per_s"] for k, v in cfg.items()
                                                if "tokens_per_s" in v}))
        del d_out, h
    v.close()
    return out


def _stream_window_check(lens, woff, n_windows):
    """Oracle-free invariant: every window's token count equals the closed
    form ceil(window bases / k), so the offsets equal their running sum."""
    want = np.empty(n_windows + 1, dtype=np.int64)
    want[0] = 0
    i = 1
    for L in lens:
        full, rem = divmod(int(L), STREAM_WINDOW)
        per = np.full(full + (1 if rem else 0), -(-STREAM_WINDOW // STREAM_K), dtype=np.int64)
        if rem:
            per[-1] = -(-rem // STREAM_K)
        want[i:i + len(per)] = per
        i += len(per)
    np.cumsum(want[1:], out=want[1:])
    return bool(np.array_equal(woff.cpu().numpy(), want))


def small_leg(reps: int = 200):
    """The small batch (64 x 16,384 i.i.d. bases, 1% N), PACKED ids for the
    single-nucleotide and 6-mer vocabularies: one step = both encodes. Launch
    bound (about a microsecond of HBM time each), so it is timed back to back
    eagerly, as replays of one captured HIP graph of both encodes over the
    same buffers, and as replays of one graph holding 8 such steps (per step:
    replay time / 8). The host time of issuing the replays is reported too:
    a replay costs the host more than the two launches it replaces."""
    import torch
    import paper_2601_05531_amd as dt
    import synth

    data, offs = synth.workload_iid()
    n = len(offs) - 1
    d_in = torch.from_numpy(data).cuda()
    d_off = torch.from_numpy(offs).cuda()
    vs = [dt.Vocab(dt.SINGLE), dt.Vocab(dt.KMER, k=6)]
    outs = []
    tokens = 0
    for v in vs:
        total, _ = dt.plan(v, offs)
        tokens += total
        outs.append((torch.empty(total, dtype=torch.int32, device="cuda"),
                     torch.empty(n + 1, dtype=torch.int64, device="cuda")))
    opts = dt.make_opts()
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream

    def eager():
        for v, (ids, oo) in zip(vs, outs):
            dt.dnatok_encode(v.handle, d_in.data_ptr(), data.size, d_off.data_ptr(), n, ids.data_ptr(), ids.numel(),
                             oo.data_ptr(), None, opts, sp)

    graph = dt.Graph([dict(vocab=v, d_bytes=d_in, d_offsets=d_off, d_ids=ids, d_out_offsets=oo)
                      for v, (ids, oo) in zip(vs, outs)])

    def replay():
        graph.launch(stream)

    graph8 = dt.Graph([dict(vocab=v, d_bytes=d_in, d_offsets=d_off, d_ids=ids, d_out_offsets=oo)
                       for _ in range(8) for v, (ids, oo) in zip(vs, outs)])

    def replay8():
        graph8.launch(stream)

    res = {}
    for name, fn, steps in (("eager", eager, 1), ("graph", replay, 1), ("graph_8_steps", replay8, 8)):
        for _ in range(10):
            fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        h0 = time.perf_counter()
        for _ in range(reps // steps):
            fn()
        host_us = (time.perf_counter() - h0) * 1e6 / (reps // steps)
        b.record(stream)
        torch.cuda.synchronize()
        us = a.elapsed_time(b) * 1e3 / ((reps // steps) * steps)
        res[name] = {"us_per_step": round(us, 2), "tokens_per_s": tokens / (us * 1e-6),
                     "host_us_per_call": round(host_us, 2)}
    graph.close()
    graph8.close()
    log("small batch: eager %.1f us/step, graph %.1f us/step, 8-step graph %.1f us/step (host per call: %.1f, %.1f, "
        "%.1f us)" % (res["eager"]["us_per_step"], res["graph"]["us_per_step"], res["graph_8_steps"]["us_per_step"],
                      res["eager"]["host_us_per_call"], res["graph"]["host_us_per_call"],
                      res["graph_8_steps"]["host_us_per_call"]))
    return {"workload": "64 x 16384 i.i.d. bases (1%% N), single-nucleotide + 6-mer PACKED, %d tokens per step"
                        % tokens, **res}


def cellwise_leg(data, offs, reps: int = 10):
    """Output-parallel paths on the batched workload (4096 x 8192 bases, CLS/SEP,
    PADDED with the int8 mask). The encode fused with the embedding lookup
    writes D = 128 bf16 rows (the paper's embedding width) per cell: the
    single-nucleotide table has 11 rows (the paper's vocabulary size), the
    6-mer table 4101; the paper left-pads, so these do too. The encode
    variants write ids: reverse-complement 6-mer frames and overlapping
    (stride 1) 6-mers of the reverse complement. Each call is a row scan plus
    one cell launch; the time per call covers both. Algorithmic bytes: input
    1 B per base plus offsets, output ids or rows plus the mask, and the table
    once."""
    import torch
    import paper_2601_05531_amd as dt

    n = len(offs) - 1
    d_in = torch.from_numpy(data).cuda()
    d_off = torch.from_numpy(offs).cuda()
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    in_bytes = data.size + 8 * (n + 1)
    cases = (("embed_single_d128_bf16", dt.SINGLE, 1, 0, 11),
             ("embed_6mer_d128_bf16", dt.KMER, 6, 0, 4101),
             ("revcomp_6mer_ids", dt.KMER, 6, dt.VARIANT_REVCOMP, 0),
             ("revcomp_overlap_6mer_ids", dt.KMER, 6, dt.VARIANT_REVCOMP | dt.VARIANT_OVERLAP, 0))
    out = {}
    for name, kind, k, variant, V in cases:
        v = dt.Vocab(kind, k=k)
        _, W = dt.plan(v, offs, add_cls_sep=True, variant=variant)
        cells = n * W
        opts = dt.make_opts(True, dt.PADDED, dt.PAD_LEFT if V else dt.PAD_RIGHT, W, variant=variant)
        oo = torch.empty(n + 1, dtype=torch.int64, device="cuda")
        mask = torch.empty(cells, dtype=torch.int8, device="cuda")
        if V:
            g = torch.Generator(device="cuda").manual_seed(42)
            table = torch.randn((V, 128), generator=g, device="cuda").to(torch.bfloat16)
            emb = torch.empty((cells, 128), dtype=torch.bfloat16, device="cuda")
            out_bytes = cells * 256 + cells + V * 256

            def call():
                dt.dnatok_embed(v.handle, d_in.data_ptr(), data.size, d_off.data_ptr(), n, table.data_ptr(), V, 256,
                                emb.data_ptr(), cells, oo.data_ptr(), None, mask.data_ptr(), opts, sp)
        else:
            ids = torch.empty(cells, dtype=torch.int32, device="cuda")
            out_bytes = cells * 5
            tuned, _ = dt.autotune(v, d_in, d_off, h_offsets=offs, add_cls_sep=True, layout=dt.PADDED, pad_to=W,
                                   variant=variant)

            def call():
                dt.dnatok_encode(v.handle, d_in.data_ptr(), data.size, d_off.data_ptr(), n, ids.data_ptr(), cells,
                                 oo.data_ptr(), mask.data_ptr(), opts, sp)
        for _ in range(3):
            call()
        torch.cuda.synchronize()
        assert dt.sync_status() == 0
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            call()
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        alg = in_bytes + out_bytes + 8 * (n + 1)
        gbps = alg / (ms * 1e-3) / 1e9
        out[name] = {"ms": round(ms, 4), "cells": cells, "cells_per_s": cells / (ms * 1e-3),
                     "algorithmic_bytes": alg, "GBps": round(gbps, 1), "frac_hbm_peak": round(gbps / HBM_PEAK_GBS, 3)}
        if not V:
            out[name]["autotuned"] = {"tile_bytes": tuned["tile_bytes"], "bands": tuned["bands"]}
        log("%s: %.3f ms, %.3e cells/s, %.0f GB/s (%.2f of peak)" % (name, ms, cells / (ms * 1e-3), gbps,
                                                                     gbps / HBM_PEAK_GBS))
        del call
        if V:
            del emb, table
        else:
            del ids
        v.close()
        torch.cuda.empty_cache()
    out["workload"] = ("4096 x 8192 bases (order-3 Markov, soft-masked, N runs, invalid bytes), CLS/SEP, PADDED "
                       "with int8 mask; embeddings D = 128 bf16 left-padded, variants right-padded")
    return out


def decode_leg(data, offs, reps: int = 10):
    """Decode (ids back to bases) of the batched workload's PACKED ids with
    CLS/SEP, for the single-nucleotide and 6-mer vocabularies: one launch per
    call. Algorithmic bytes: 4 B per id in, the decoded bases out (1 B per
    base; a 6-mer id decodes to 6), plus both offsets arrays."""
    import torch
    import paper_2601_05531_amd as dt

    n = len(offs) - 1
    d_in = torch.from_numpy(data).cuda()
    d_off = torch.from_numpy(offs).cuda()
    st = torch.cuda.current_stream()
    sp = st.cuda_stream
    out = {}
    for name, kind, k in (("single", dt.SINGLE, 1), ("6mer", dt.KMER, 6)):
        v = dt.Vocab(kind, k=k)
        ids, id_off, _ = dt.encode(v, d_in, d_off, h_offsets=offs, add_cls_sep=True)
        cap = ids.numel() * v.max_token_bytes
        dec = torch.empty(cap, dtype=torch.uint8, device="cuda")
        dec_off = torch.empty(n + 1, dtype=torch.int64, device="cuda")

        def call():
            dt.dnatok_decode(v.handle, ids.data_ptr(), ids.numel(), id_off.data_ptr(), n, dec.data_ptr(), cap,
                             dec_off.data_ptr(), sp)
        for _ in range(3):
            call()
        torch.cuda.synchronize()
        assert dt.sync_status() == 0
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        for _ in range(reps):
            call()
        b.record(st)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        out_bytes = int(dec_off[n].item())
        alg = 4 * ids.numel() + out_bytes + 16 * (n + 1)
        gbps = alg / (ms * 1e-3) / 1e9
        out[name] = {"ms": round(ms, 4), "ids": ids.numel(), "bases_out": out_bytes, "ids_per_s": ids.numel() / (ms * 1e-3),
                     "GBps": round(gbps, 1), "frac_hbm_peak": round(gbps / HBM_PEAK_GBS, 3)}
        log("decode %s: %.3f ms, %.3e ids/s, %.0f GB/s (%.2f of peak)" % (name, ms, ids.numel() / (ms * 1e-3), gbps,
                                                                        gbps / HBM_PEAK_GBS))
        v.close()
    out["workload"] = "PACKED ids (CLS/SEP) of the 4096 x 8192-base batch back to uppercase bases"
    return out


BPE_TABLE = os.path.join(ROOT, "tests", "golden", "bpe4096_order5_64M.txt")


def _bpe_ranks(ids, out_off, merges):
    """Ranks each row applies, from the output alone: every rank applied to
    a row is in the merge tree of one of its final tokens (a merged symbol
    either survives or is merged again), so they are the distinct merge ids
    over the rows' token trees. Merging one rank per round, as the
    definition reads, takes that many rounds."""
    R = len(merges)
    tree = [None] * R
    for r in range(R):
        t = {r}
        for x in merges[r]:
            if x >= 10:
                t |= tree[x - 10]
        tree[r] = frozenset(t)
    n = len(out_off) - 1
    rounds = np.zeros(n, dtype=np.int64)
    for i in range(n):
        row = np.unique(ids[out_off[i]:out_off[i + 1]])
        seen = set()
        for x in row[row >= 10]:
            seen |= tree[int(x) - 10]
        rounds[i] = len(seen)
    return rounds


def bpe_leg(reps: int = 10, tuning=None, per_seq_leg: bool = True):
    """Ragged BPE batch: 1,024 sequences, lengths log-uniform in [500, 20000]
    bases, fresh walk of the order-5 Markov chain the 4096-merge table was
    trained on; PACKED ids, no specials. The fused form encodes the whole
    batch in one call; the per-sequence form makes one call per sequence
    (the same kernels, n = 1) into the same output positions. Both are timed
    with HIP events on the launch stream and must produce identical ids."""
    import torch
    import paper_2601_05531_amd as dt
    import synth

    merges = np.loadtxt(BPE_TABLE, dtype=np.int32).reshape(-1, 2)
    v = dt.Vocab(dt.BPE, merges=merges)
    data, offs = synth.workload_bpe_batch()
    n = len(offs) - 1
    nbytes = int(data.size)
    d_in = torch.from_numpy(data).cuda()
    d_offs = torch.from_numpy(offs).cuda()
    ids = torch.empty(nbytes, dtype=torch.int32, device="cuda")
    oo = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    opts = dt.make_opts()
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream

    def fused():
        dt.dnatok_encode(v.handle, d_in.data_ptr(), nbytes, d_offs.data_ptr(), n, ids.data_ptr(), nbytes,
                         oo.data_ptr(), None, opts, sp)

    if tuning is None:
        tune, tune_ms = dt.autotune(v, d_in, d_offs, h_offsets=offs, reps=1)
        log("bpe autotuned: %s (%.3f ms)" % (tune, tune_ms))
    else:
        dt.set_tuning(v, bpe_item_bytes=tuning[0], bpe_max_waves=tuning[1])
        tune = dt.dnatok_get_tuning(v.handle).as_dict()
        log("bpe tiling set: %s" % tune)

    fused()
    torch.cuda.synchronize()
    assert dt.sync_status() == 0
    h_oo = oo.cpu().numpy()
    tokens = int(h_oo[-1])
    evs = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fused()
        b.record(stream)
        evs.append((a, b))
    torch.cuda.synchronize()
    fused_ms = float(np.median([a.elapsed_time(b) for a, b in evs]))

    rounds = _bpe_ranks(ids[:tokens].cpu().numpy(), h_oo, merges)
    out = {
        "workload": "1024 sequences, log-uniform 500-20000 bases (%d bases), order-5 Markov, BPE 4096 merges "
                    "(oracle trainer, 64 Mbase), PACKED, no specials" % nbytes,
        "tokens": tokens,
        "ranks_per_row": {
            "note": "ranks each row applies (distinct ranks in its tokens' merge trees; every row is one ACGT "
                    "run, so one item): the rounds of a one-rank-per-round merge. The kernel merges the ranks "
                    "present in a window above the lowest one in a single round where that is exact, so its "
                    "rounds are fewer; the fused call's critical path is the row with the most ranks",
            "max": int(rounds.max()), "p50": float(np.median(rounds)), "p90": float(np.percentile(rounds, 90)),
            "mean": float(rounds.mean()),
            "hist_edges": [0, 100, 200, 400, 800, 1200, 1600, 2400],
            "hist": np.histogram(rounds, bins=[0, 100, 200, 400, 800, 1200, 1600, 2400])[0].tolist(),
            "longest_row_bases": int(np.diff(offs)[int(np.argmax(rounds))]),
        },
        ("autotuned" if tuning is None else "tiling"): {"bpe_item_bytes": tune["bpe_item_bytes"],
                                                        "bpe_max_waves": tune["bpe_max_waves"]},
        "fused_ms": round(fused_ms, 4),
        "fused_tokens_per_s": tokens / (fused_ms * 1e-3),
        "fused_bases_per_s": nbytes / (fused_ms * 1e-3),
    }
    out["us_per_rank_on_critical_path"] = round(fused_ms * 1e3 / max(1, int(rounds.max())), 3)
    if not per_seq_leg:
        log("bpe: fused %.3f ms (%.3e tokens/s)" % (fused_ms, out["fused_tokens_per_s"]))
        return out, data, offs, merges

    # one call per sequence, each writing its ids where the fused call put them
    lens = np.diff(offs)
    row_offs = torch.from_numpy(np.stack([np.zeros(n, np.int64), lens], 1).copy()).cuda()
    row_oo = torch.empty(n, 2, dtype=torch.int64, device="cuda")
    ids2 = torch.empty_like(ids)
    row_opts = [dt.make_opts(offset_base=int(h_oo[i])) for i in range(n)]

    def per_seq():
        for i in range(n):
            dt.dnatok_encode(v.handle, d_in.data_ptr() + int(offs[i]), int(lens[i]), row_offs[i].data_ptr(), 1,
                             ids2.data_ptr() + 4 * int(h_oo[i]), int(lens[i]), row_oo[i].data_ptr(), None,
                             row_opts[i], sp)

    per_seq()
    torch.cuda.synchronize()
    assert dt.sync_status() == 0
    same = bool(torch.equal(ids[:tokens], ids2[:tokens])) and bool(
        torch.equal(row_oo[:, 1].cpu(), oo[1:].cpu()))
    times = []
    for _ in range(2):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        per_seq()
        b.record(stream)
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    per_ms = float(min(times))
    out.update({
        "per_sequence_ms": round(per_ms, 3),
        "per_sequence_tokens_per_s": tokens / (per_ms * 1e-3),
        "fused_speedup": round(per_ms / fused_ms, 2),
        "per_sequence_ids_identical": same,
    })
    log("bpe: fused %.3f ms (%.3e tokens/s), per-sequence %.3f ms, identical=%s" % (
        fused_ms, out["fused_tokens_per_s"], per_ms, same))
    return out, data, offs, merges


SERVE_REQUESTS = 20000
SERVE_RATE = 2000.0


def serve_leg(n_requests: int = SERVE_REQUESTS):
    """Serving trace: Poisson arrivals at 2,000 req/s, sizes log-uniform in
    [100, 1e6] bases, vocabulary uniform over {single-nt, 3-mer, 6-mer,
    BPE-4096}, CLS/SEP on, content drawn from a 64 Mbase genome of the
    batched workload's model (pinned host memory). The trace is replayed in
    real time twice: through the serving loop (16 GiB budget, 4 streams,
    continuous batching) and through the plain path (per request: one H2D
    copy, one dnatok_encode, one synchronisation, in arrival order on one
    stream). Latency = completion seen by the host - arrival."""
    import threading
    import torch
    import paper_2601_05531_amd as dt
    import synth

    merges = np.loadtxt(BPE_TABLE, dtype=np.int32).reshape(-1, 2)
    vocabs = [dt.Vocab(dt.SINGLE), dt.Vocab(dt.KMER, k=3), dt.Vocab(dt.KMER, k=6), dt.Vocab(dt.BPE, merges=merges)]
    arrivals, sizes, which = synth.serving_trace(n_requests=n_requests, rate=SERVE_RATE)
    G = 64 << 20
    h = torch.empty(G, dtype=torch.uint8, pin_memory=True)
    synth.genome(synth.substream(5, 1), synth.substream(5, 2), 3, G, out=h.numpy())
    rng = np.random.default_rng(synth.substream(5, 3))
    starts = rng.integers(0, G - int(sizes.max()), n_requests)
    total_bases = int(sizes.sum())

    def pct(x, q):
        return float(np.percentile(np.asarray(x), q)) * 1e3

    # ---- serving loop
    srv = dt.Server(budget_bytes=16 << 30, n_streams=4, max_batch=512, max_batch_bytes=32 << 20)
    warm = [srv.submit(vocabs[i % 4], h[0:100000]) for i in range(8)]
    for t in warm:
        srv.wait(t)
        srv.release(t)
    tickets = [None] * n_requests
    lat = np.zeros(n_requests)
    tokens = np.zeros(n_requests, dtype=np.int64)
    ready = threading.Semaphore(0)

    def waiter():
        for i in range(n_requests):
            ready.acquire()
            r = dt.dnatok_server_wait(srv.handle, tickets[i])
            assert r.status == dt.OK and r.dev_flags == 0
            lat[i] = r.t_done - r.t_submit
            tokens[i] = r.n_tokens
            dt.dnatok_server_release(srv.handle, tickets[i])

    th = threading.Thread(target=waiter)
    th.start()
    slip = np.zeros(n_requests)  # submission after the request's arrival time (host scheduling)
    t0 = time.perf_counter()
    for i in range(n_requests):
        d = t0 + arrivals[i] - time.perf_counter()
        if d > 0:
            time.sleep(d)
        a, n = int(starts[i]), int(sizes[i])
        slip[i] = max(0.0, time.perf_counter() - (t0 + arrivals[i]))
        tickets[i] = dt.dnatok_server_submit(srv.handle, vocabs[which[i]].handle, h.data_ptr() + a, n, 1)
        ready.release()
    th.join()
    lat += slip
    t_srv = time.perf_counter() - t0
    done, batches, peak = srv.stats()
    srv.close()
    server = {"p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "mean_ms": float(lat.mean()) * 1e3,
              "tokens_per_s": float(tokens.sum()) / t_srv, "wall_s": round(t_srv, 3), "batches": int(batches),
              "peak_arena_bytes": int(peak), "max_submit_slip_ms": float(slip.max()) * 1e3}
    log("serve (batched): p50 %.3f ms p99 %.3f ms, %.3e tokens/s, %d batches" % (
        server["p50_ms"], server["p99_ms"], server["tokens_per_s"], batches))

    # ---- plain path: one copy + one encode + one sync per request, in arrival order
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    sp = stream.cuda_stream
    cap = int(sizes.max()) + 2
    d_in = torch.empty(cap, dtype=torch.uint8, device="cuda")
    d_ids = torch.empty(cap, dtype=torch.int32, device="cuda")
    d_off = torch.empty(2, dtype=torch.int64, device="cuda")
    d_oo = torch.empty(2, dtype=torch.int64, device="cuda")
    h_off = torch.zeros(2, dtype=torch.int64, pin_memory=True)
    opts = dt.make_opts(add_cls_sep=True)
    lat2 = np.zeros(n_requests)
    tok2 = np.zeros(n_requests, dtype=np.int64)
    for i in range(4):  # warm every vocabulary
        dt.dnatok_encode(vocabs[i].handle, h.data_ptr(), 1000, d_off.data_ptr(), 0, d_ids.data_ptr(), cap,
                         d_oo.data_ptr(), None, opts, sp)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(n_requests):
        d = t0 + arrivals[i] - time.perf_counter()
        if d > 0:
            time.sleep(d)
        a, n = int(starts[i]), int(sizes[i])
        with torch.cuda.stream(stream):
            d_in[:n].copy_(h[a:a + n], non_blocking=True)
            h_off[1] = n
            d_off.copy_(h_off, non_blocking=True)
            dt.dnatok_encode(vocabs[which[i]].handle, d_in.data_ptr(), n, d_off.data_ptr(), 1, d_ids.data_ptr(),
                             cap, d_oo.data_ptr(), None, opts, sp)
        stream.synchronize()
        lat2[i] = time.perf_counter() - (t0 + arrivals[i])
        if which[i] == 3:
            tok2[i] = int(d_oo[1].item())
    t_plain = time.perf_counter() - t0
    for i in np.nonzero(which != 3)[0]:
        tok2[i] = int(dt.plan(vocabs[which[i]], np.array([0, int(sizes[i])]), True)[0])
    same_counts = bool(np.array_equal(tok2, tokens))
    tok2 = int(tok2.sum())
    plain = {"p50_ms": pct(lat2, 50), "p99_ms": pct(lat2, 99), "mean_ms": float(lat2.mean()) * 1e3,
             "tokens_per_s": tok2 / t_plain, "wall_s": round(t_plain, 3)}
    log("serve (per request): p50 %.3f ms p99 %.3f ms, %.3e tokens/s" % (
        plain["p50_ms"], plain["p99_ms"], plain["tokens_per_s"]))
    del h
    return {"workload": "%d requests, Poisson %.0f req/s, sizes log-uniform 100-1e6 bases (%d bases), vocab uniform "
                        "over single/3-mer/6-mer/BPE-4096, CLS/SEP, 16 GiB budget" % (n_requests, SERVE_RATE,
                                                                                        total_bases),
            "server": server, "per_request": plain, "token_counts_agree": same_counts,
            "p99_speedup": round(plain["p99_ms"] / server["p99_ms"], 2)}


def _host_threads():
    """Worker threads for the oracle: the CPUs this process may run on, at
    most 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(data, offs, budget_s: float = 12.0, bpe=None, stream=None):
    """The CPU oracle as written on a bounded sample: whole rows of the same
    batch, all four k, for about ``budget_s`` seconds single-threaded and the
    same again with the rows split over the host's threads (a static
    partition by bytes). Also times the oracle's BPE on the first rows of the
    BPE batch and, given the stream leg's buffer and ids, the oracle over all
    2 GiB of stream windows (threaded), checking the GPU stream's ids against
    it id for id."""
    import oracle
    threads = _host_threads()
    rows = 256
    sub = offs[:rows + 1]
    chunk = data[:sub[-1]]

    def timed(fn, budget):
        t_total, tok_total, reps = 0.0, 0, 0
        while t_total < budget:
            for k in KS:
                t0 = time.perf_counter()
                ids, oo = fn(k)
                t_total += time.perf_counter() - t0
                tok_total += int(oo[-1])
            reps += 1
        return tok_total / t_total, t_total, reps

    def one(k):
        ids, oo = oracle.encode(oracle.KMER, chunk, sub, k=k, add_cls_sep=True)
        oracle.pad(ids, oo, int(np.diff(oo).max()))
        return ids, oo

    v1, t1, r1 = timed(one, budget_s)
    big = offs[:min(len(offs), 2048 + 1)]
    big_chunk = data[:big[-1]]

    def many(k):
        ids, oo = oracle.encode_threads(oracle.KMER, big_chunk, big, threads=threads, k=k, add_cls_sep=True)
        oracle.pad_threads(ids, oo, int(np.diff(oo).max()), threads=threads)
        return ids, oo

    vt, tt, rt = timed(many, budget_s / 2)
    res = {"value": v1, "unit": "tokens/s", "cores": 1, "kind": "oracle",
           "sample": "%d reps of %d of the %d rows (%d bases), k=3,4,5,6, CLS/SEP, right-padded, "
                     "single-threaded C oracle, %.1f s" % (r1, rows, N_SEQS, int(sub[-1]), t1),
           "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
           "affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
           "threaded": {"value": vt, "unit": "tokens/s", "cores": threads,
                        "sample": "%d reps of %d rows (%d bases), k=3,4,5,6, CLS/SEP, right-padded, rows split by "
                                  "bytes over %d threads, %.1f s" % (rt, len(big) - 1, int(big[-1]), threads, tt)}}
    if bpe is not None:
        # the oracle's BPE on the first rows of the BPE batch, about 1 s
        b_data, b_offs, merges = bpe
        rows = 48
        sub = b_offs[:rows + 1]
        t0 = time.perf_counter()
        ids, oo = oracle.encode(oracle.BPE, b_data[:sub[-1]], sub, merges=merges)
        t = time.perf_counter() - t0
        res["bpe"] = {"value": int(oo[-1]) / t, "unit": "tokens/s", "cores": 1,
                      "sample": "first %d of the 1024 BPE rows (%d bases), %.1f s" % (rows, int(sub[-1]), t)}
    if stream is not None:
        (h, lens), got = stream
        woffs = oracle.windows(lens, STREAM_WINDOW)
        t0 = time.perf_counter()
        want, want_off = oracle.encode_threads(oracle.KMER, h.numpy(), woffs, threads=threads, k=STREAM_K)
        t = time.perf_counter() - t0
        res["stream"] = {"value": len(want) / t, "unit": "tokens/s", "cores": threads,
                         "sample": "all %d windows of the 2 GiB stream, 6-mers, rows split by bytes over %d "
                                   "threads, %.1f s" % (len(woffs) - 1, threads, t),
                         "gpu_stream_ids_match_oracle": bool(got is not None and np.array_equal(got, want))}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-copy", action="store_true", help="skip the device-copy reference")
    ap.add_argument("--no-stream", action="store_true", help="skip the 2 GiB host-to-device stream leg")
    ap.add_argument("--no-bpe", action="store_true", help="skip the ragged BPE batch leg")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving trace leg")
    ap.add_argument("--no-small", action="store_true", help="skip the small-batch eager/graph leg")
    ap.add_argument("--no-cellwise", action="store_true",
                    help="skip the embedding-lookup and encode-variant leg")
    ap.add_argument("--no-decode", action="store_true", help="skip the decode leg")
    ap.add_argument("--no-ids", action="store_true", help="skip the IDs path ablation leg")
    ap.add_argument("--no-per-vocab", action="store_true", help="skip the four single-vocabulary launches")
    ap.add_argument("--tuning", type=str, default=None,
                    help="TILE,BLOCKS[,BANDS]: fixed tiling of the one-pass encode instead of the autotuner's")
    ap.add_argument("--bpe-tuning", type=str, default=None,
                    help="ITEM_BYTES,WAVES: fixed BPE tiling instead of the autotuner's")
    ap.add_argument("--no-bpe-per-seq", action="store_true",
                    help="time only the fused BPE call (skip the one-call-per-sequence comparison)")
    ap.add_argument("--serve-requests", type=int, default=SERVE_REQUESTS)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the tokenizer shards by sequences with no collective on the hot path, "
              "so each GPU runs this same step on its share and there is nothing to measure across GPUs "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    import paper_2601_05531_amd as dt
    dt.lib()

    tuning = tuple(int(x) for x in args.tuning.split(",")) if args.tuning else None
    enc = encode_leg(args.steps, args.warmup, tuning=tuning, per_vocab=not args.no_per_vocab)
    copy = None
    if not args.no_copy:
        copy = copy_leg(encode_bytes=enc["bytes_per_launch"], fill_bytes=enc["bytes_written_per_launch"])
        enc["roofline"]["device_copy"] = copy
        log("device copy: %s" % copy)
    stream = stream_keep = None
    if not args.no_stream:
        stream, stream_buf, stream_ids = stream_leg()
        stream_keep = (stream_buf, stream_ids)
    ids = None
    if not args.no_ids:
        ids = ids_leg()
    small = None
    if not args.no_small:
        small = small_leg()
    cellwise = None
    if not args.no_cellwise:
        cellwise = cellwise_leg(enc["data"], enc["offs"])
    decode = None
    if not args.no_decode:
        decode = decode_leg(enc["data"], enc["offs"])
    serve = None
    if not args.no_serve:
        serve = serve_leg(args.serve_requests)
    bpe = bpe_in = None
    if not args.no_bpe:
        bt = tuple(int(x) for x in args.bpe_tuning.split(",")) if args.bpe_tuning else None
        bpe, b_data, b_offs, merges = bpe_leg(tuning=bt, per_seq_leg=not args.no_bpe_per_seq)
        bpe_in = (b_data, b_offs, merges)
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(enc["data"], enc["offs"], bpe=bpe_in, stream=stream_keep)
        log("cpu oracle: %.3e tokens/s (one thread), %.3e tokens/s (%d threads)" % (
            cpu["value"], cpu["threaded"]["value"], cpu["threaded"]["cores"]))
        if stream is not None and "stream" in cpu:
            stream["ids_match_oracle"] = cpu["stream"]["gpu_stream_ids_match_oracle"]
    stream_keep = None
    line = {
        "metric": METRIC,
        "value": enc["value"],
        "unit": "tokens/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": enc["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": "batched k-mer encode: 4096 x 8192 bases (order-3 Markov, 40% soft-masked, 2% N runs, "
                        "1e-4 invalid bytes), non-overlapping k = 3,4,5,6 written in one pass over the bytes (one "
                        "launch per step), CLS/SEP, right-padded int32 ids + int8 mask, inputs resident in HBM",
            "tokens_per_step": enc["tokens_per_step"],
            "launch_ms": enc["launch_ms"],
            "autotuned": enc["tuning"],
            "four_single_vocab_launches": enc["per_vocab"],
        },
        "roofline": enc["roofline"],
        "cpu_baseline": cpu,
        "stream": stream,
        "bpe": bpe,
        "serve": serve,
        "small_batch": small,
        "embed_and_variants": cellwise,
        "decode": decode,
        "ids_path": ids,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
