"""GPU parity of the PADDED row-band kernels (tuning bands=1: a workgroup
per band; bands=3: resident workgroups taking bands in turn) against the
oracle, id by id and mask byte by mask byte: every kind, k = 1..8 and 15,
several vocabularies in one pass, both pad sides, with and without CLS/SEP,
wide padding, stage sizes from one short row to many rows per band,
misaligned inputs and outputs, the full batched workload, batches whose row
scans run as a separate launch, and the device-side errors (flags raised,
nothing written outside the outputs)."""
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


def _fuzz_batch(seed, n, max_len):
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, max_len + 1, n)
    lens[rng.integers(0, n, max(1, n // 10))] = 0
    total = int(lens.sum())
    data = synth.uniform_bytes(seed, total)
    dna = np.frombuffer(b"ACGTNacgtn", np.uint8)
    pick = rng.random(total) < 0.9
    data[pick] = dna[rng.integers(0, 10, int(pick.sum()))]
    return data, synth.offsets_from_lengths(lens)


MODE = {"bands": 1}


@pytest.fixture(autouse=True, params=[1, 3], ids=["per_band", "persistent"])
def band_mode(request):
    MODE["bands"] = request.param
    yield request.param


def _banded(v, stage):
    dt.set_tuning(v, tile_bytes=stage, bands=MODE["bands"])
    return v


def _check(vs, kinds_k, data, offs, cls, side, pad_extra=0, byte_shift=0, id_shift=0, lut=None, pad_id=0):
    """Encode through dnatok_encode_multi (one vocabulary: dnatok_encode) into
    buffers offset by id_shift elements, input offset by byte_shift bytes."""
    torch = _torch()
    n = len(offs) - 1
    wants = []
    for (kind, k) in kinds_k:
        w_ids, w_off = oracle.encode(kind, data, offs, k=k, lut=lut, add_cls_sep=cls)
        wants.append((w_ids, w_off, max(1, int(np.diff(w_off).max(initial=0)) + pad_extra)))
    buf = np.zeros(len(data) + 32, np.uint8)
    buf[byte_shift:byte_shift + len(data)] = data
    d_buf = _dev(buf)
    d_bytes = d_buf[byte_shift:]
    d_offs = _dev(offs)
    outs, opts = [], []
    for (w_ids, w_off, W) in wants:
        ids = torch.full((n * W + id_shift + 8,), -7, dtype=torch.int32, device="cuda")
        mask = torch.full((n * W + id_shift + 8,), -7, dtype=torch.int8, device="cuda")
        oo = torch.empty(n + 1, dtype=torch.int64, device="cuda")
        outs.append((ids, oo, mask))
        opts.append(dt.make_opts(cls, dt.PADDED, side, W))
    print("bands(%d): n=%d nbytes=%d vocabs=%s cls=%d side=%d extra=%d shifts=%d/%d" % (
        MODE["bands"], n, len(data), kinds_k, cls, side, pad_extra, byte_shift, id_shift), flush=True)
    stream = torch.cuda.current_stream().cuda_stream
    if len(vs) == 1:
        ids, oo, mask = outs[0]
        dt.dnatok_encode(vs[0].handle, d_bytes.data_ptr(), len(data), d_offs.data_ptr(), n,
                         ids.data_ptr() + 4 * id_shift, n * wants[0][2], oo.data_ptr(), mask.data_ptr() + id_shift,
                         opts[0], stream)
    else:
        import ctypes
        nv = len(vs)
        arr = lambda t, xs: (t * nv)(*xs)
        dt._check(dt.lib().dnatok_encode_multi(
            arr(ctypes.c_void_p, [v.handle for v in vs]), nv, d_bytes.data_ptr(), len(data), d_offs.data_ptr(), n,
            arr(ctypes.c_void_p, [o[0].data_ptr() + 4 * id_shift for o in outs]),
            arr(ctypes.c_int64, [n * w[2] for w in wants]), arr(ctypes.c_void_p, [o[1].data_ptr() for o in outs]),
            arr(ctypes.c_void_p, [o[2].data_ptr() + id_shift for o in outs]), arr(dt.dnatok_encode_opts, opts),
            ctypes.c_void_p(stream)))
    torch.cuda.synchronize()
    assert dt.sync_status() == 0
    for (w_ids, w_off, W), (ids, oo, mask) in zip(wants, outs):
        p_ids, p_mask = oracle.pad(w_ids, w_off, W, side, pad_id)
        assert np.array_equal(oo.cpu().numpy(), w_off)
        got = ids.cpu().numpy()
        gm = mask.cpu().numpy()
        assert np.all(got[:id_shift] == -7) and np.all(got[id_shift + n * W:] == -7)
        assert np.all(gm[:id_shift] == -7) and np.all(gm[id_shift + n * W:] == -7)
        g = got[id_shift:id_shift + n * W].reshape(n, W)
        bad = np.argwhere(g != p_ids)
        assert bad.size == 0, "first mismatch at %s: got %d want %d" % (bad[0], g[tuple(bad[0])], p_ids[tuple(bad[0])])
        assert np.array_equal(gm[id_shift:id_shift + n * W].reshape(n, W), p_mask)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 7, 8, 15])
def test_bands_fuzz_kmer(k):
    data, offs = _fuzz_batch(3000 + k, 1500, 140)
    for stage in (4096, 65536):
        v = _banded(dt.Vocab(dt.KMER, k=k), stage)
        _check([v], [(dt.KMER, k)], data, offs, True, dt.PAD_RIGHT, pad_extra=3, byte_shift=stage % 7)
        _check([v], [(dt.KMER, k)], data, offs, False, dt.PAD_LEFT, id_shift=1 + k % 3)
        v.close()


def test_bands_single_and_lut256():
    data, offs = _fuzz_batch(3100, 2000, 140)
    lut = oracle.fallback_lut()
    for stage in (4096, 16384):
        v = _banded(dt.Vocab(dt.SINGLE), stage)
        _check([v], [(dt.SINGLE, 1)], data, offs, True, dt.PAD_LEFT, pad_extra=5, id_shift=3, byte_shift=5)
        _check([v], [(dt.SINGLE, 1)], data, offs, False, dt.PAD_RIGHT)
        lv = _banded(dt.Vocab(dt.LUT256, lut256=lut, pad_id=0, cls_id=7, sep_id=8), stage)
        torch = _torch()
        n = len(offs) - 1
        w_ids, w_off = oracle.encode(oracle.LUT256, data, offs, lut=lut, add_cls_sep=True, cls_id=7, sep_id=8)
        W = int(np.diff(w_off).max()) + 2
        p_ids, p_mask = oracle.pad(w_ids, w_off, W, dt.PAD_RIGHT, 0)
        ids, oo, mask = dt.encode(lv, _dev(data), _dev(offs), h_offsets=offs, add_cls_sep=True, layout=dt.PADDED,
                                  pad_to=W)
        torch.cuda.synchronize()
        assert dt.sync_status() == 0
        assert np.array_equal(ids.cpu().numpy(), p_ids) and np.array_equal(mask.cpu().numpy(), p_mask)
        assert n == ids.shape[0]


def test_bands_multi_vocab_fuzz_and_wide_padding():
    data, offs = _fuzz_batch(3200, 1800, 140)
    ks = [1, 2, 3, 4, 5, 6, 7, 8]
    for stage in (4096, 32768):
        vs = [dt.Vocab(dt.KMER, k=k) for k in ks]
        _banded(vs[0], stage)
        _check(vs, [(dt.KMER, k) for k in ks], data, offs, True, dt.PAD_RIGHT, id_shift=2)
        _check(vs, [(dt.KMER, k) for k in ks], data, offs, False, dt.PAD_LEFT, pad_extra=1777, byte_shift=9)


def test_bands_full_batched_workload():
    data, offs = synth.workload_markov_batch()
    ks = [3, 4, 5, 6]
    for stage in (4096, 8192, 32768):
        vs = [dt.Vocab(dt.KMER, k=k) for k in ks]
        _banded(vs[0], stage)
        _check(vs, [(dt.KMER, k) for k in ks], data, offs, True, dt.PAD_RIGHT)
    v = _banded(dt.Vocab(dt.KMER, k=5), 16384)
    _check([v], [(dt.KMER, 5)], data[:offs[700]], offs[:701], True, dt.PAD_LEFT, pad_extra=11)


def test_bands_many_rows_row_scan_launched_apart():
    data, offs = _fuzz_batch(3300, 20000, 40)
    vs = [dt.Vocab(dt.KMER, k=k) for k in (3, 6)]
    _banded(vs[0], 8192)
    _check(vs, [(dt.KMER, 3), (dt.KMER, 6)], data, offs, True, dt.PAD_RIGHT)
    v = _banded(dt.Vocab(dt.SINGLE), 4096)
    _check([v], [(dt.SINGLE, 1)], data, offs, False, dt.PAD_LEFT, id_shift=1)


def test_bands_empty_rows_and_batches():
    torch = _torch()
    v = _banded(dt.Vocab(dt.KMER, k=4), 4096)
    offs = np.zeros(9, np.int64)
    data = np.zeros(0, np.uint8)
    _check([v], [(dt.KMER, 4)], data, offs, True, dt.PAD_RIGHT, pad_extra=2)
    _check([v], [(dt.KMER, 4)], data, offs, False, dt.PAD_LEFT, pad_extra=5)
    oo = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    ids = torch.empty(4, dtype=torch.int32, device="cuda")
    mask = torch.empty(4, dtype=torch.int8, device="cuda")
    dt.dnatok_encode(v.handle, None, 0, _dev(np.zeros(1, np.int64)).data_ptr(), 0, ids.data_ptr(), 4,
                     oo.data_ptr(), mask.data_ptr(), dt.make_opts(True, dt.PADDED, 0, 3), None)
    torch.cuda.synchronize()
    assert dt.sync_status() == 0 and int(oo[0].item()) == 0


def test_bands_device_errors_are_flagged_and_bounded():
    torch = _torch()
    v = _banded(dt.Vocab(dt.KMER, k=3), 4096)
    data, offs = _fuzz_batch(3400, 400, 200)
    want_ids, want_off = oracle.encode(oracle.KMER, data, offs, k=3)
    n = len(offs) - 1
    stream = torch.cuda.current_stream().cuda_stream
    out_off = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    d_bytes = _dev(data)
    # a width below the longest row: flag raised, nothing written past n * W
    W = int(np.diff(want_off).max()) - 1
    pid = torch.full((n * W + 64,), -7, dtype=torch.int32, device="cuda")
    pm = torch.full((n * W + 64,), -7, dtype=torch.int8, device="cuda")
    dt.dnatok_encode(v.handle, d_bytes.data_ptr(), len(data), _dev(offs).data_ptr(), n, pid.data_ptr(), n * W,
                     out_off.data_ptr(), pm.data_ptr(), dt.make_opts(layout=dt.PADDED, pad_to=W), stream)
    assert dt.sync_status() == dt.DERR_ROW_WIDTH
    assert np.all(pid.cpu().numpy()[n * W:] == -7) and np.all(pm.cpu().numpy()[n * W:] == -7)
    # rows that fit are still right
    got = pid.cpu().numpy()[:n * W].reshape(n, W)
    lens = np.diff(want_off)
    ok_rows = np.nonzero(lens <= W)[0]
    p_ids, _ = oracle.pad(want_ids, want_off, int(lens.max()))
    assert np.array_equal(got[ok_rows], p_ids[ok_rows, :W])
    # decreasing and out-of-range offsets: flagged, bounded (the bands span
    # more than their stage and read bytes from global memory)
    W = int(np.diff(want_off).max())
    bad = offs.copy()
    bad[10] = bad[12] + 5
    bad2 = offs.copy()
    bad2[-1] = len(data) + 100
    bad2[200] = 0
    for b in (bad, bad2):
        pid = torch.full((n * W + 64,), -7, dtype=torch.int32, device="cuda")
        dt.dnatok_encode(v.handle, d_bytes.data_ptr(), len(data), _dev(b).data_ptr(), n, pid.data_ptr(), n * W,
                         out_off.data_ptr(), pm.data_ptr(), dt.make_opts(layout=dt.PADDED, pad_to=W), stream)
        assert dt.sync_status() & dt.DERR_OFFSETS
        assert np.all(pid.cpu().numpy()[n * W:] == -7)


def _want_variant(kind, k, data, offs, cls, variant, lut=None):
    src = oracle.revcomp(data, offs) if variant & dt.VARIANT_REVCOMP else data
    if variant & dt.VARIANT_OVERLAP:
        return oracle.encode_overlap(src, offs, k, add_cls_sep=cls)
    return oracle.encode(kind, src, offs, k=k, lut=lut, add_cls_sep=cls)


@pytest.mark.parametrize("k", [1, 2, 3, 5, 6, 8, 9, 15])
def test_bands_variants_kmer(k):
    torch = _torch()
    data, offs = _fuzz_batch(3500 + k, 1200, 150)
    n = len(offs) - 1
    for stage in (4096, 32768):
        v = _banded(dt.Vocab(dt.KMER, k=k), stage)
        for variant in (dt.VARIANT_REVCOMP, dt.VARIANT_OVERLAP, dt.VARIANT_REVCOMP | dt.VARIANT_OVERLAP):
            for cls, side, extra in ((True, dt.PAD_RIGHT, 0), (False, dt.PAD_LEFT, 3)):
                w_ids, w_off = _want_variant(dt.KMER, k, data, offs, cls, variant)
                W = max(1, int(np.diff(w_off).max()) + extra)
                p_ids, p_mask = oracle.pad(w_ids, w_off, W, side)
                print("bands variant k=%d stage=%d variant=%d cls=%d side=%d" % (k, stage, variant, cls, side),
                      flush=True)
                ids, oo, mask = dt.encode(v, _dev(data), _dev(offs), h_offsets=offs, add_cls_sep=cls,
                                          layout=dt.PADDED, pad_side=side, pad_to=W, variant=variant)
                torch.cuda.synchronize()
                assert dt.sync_status() == 0
                assert np.array_equal(oo.cpu().numpy(), w_off)
                g = ids.cpu().numpy()
                bad = np.argwhere(g != p_ids)
                assert bad.size == 0, "first mismatch at %s: got %d want %d" % (
                    bad[0], g[tuple(bad[0])], p_ids[tuple(bad[0])])
                assert np.array_equal(mask.cpu().numpy(), p_mask)
                assert ids.shape == (n, W)
        v.close()


def test_bands_variants_tables_and_full_batch():
    torch = _torch()
    data, offs = _fuzz_batch(3600, 1500, 150)
    lut = oracle.fallback_lut()
    for kind, kw in ((dt.SINGLE, {}), (dt.LUT256, {"lut256": lut})):
        v = _banded(dt.Vocab(kind, **kw), 8192)
        for cls, side in ((True, dt.PAD_LEFT), (False, dt.PAD_RIGHT)):
            w_ids, w_off = _want_variant(kind, 1, data, offs, cls, dt.VARIANT_REVCOMP, lut=kw.get("lut256"))
            W = int(np.diff(w_off).max()) + 1
            p_ids, p_mask = oracle.pad(w_ids, w_off, W, side)
            ids, oo, mask = dt.encode(v, _dev(data), _dev(offs), h_offsets=offs, add_cls_sep=cls, layout=dt.PADDED,
                                      pad_side=side, pad_to=W, variant=dt.VARIANT_REVCOMP)
            torch.cuda.synchronize()
            assert dt.sync_status() == 0
            assert np.array_equal(ids.cpu().numpy(), p_ids) and np.array_equal(mask.cpu().numpy(), p_mask)
    # the batched workload, 6-mers, as the benchmark's variant legs run it
    data, offs = synth.workload_markov_batch()
    for variant in (dt.VARIANT_REVCOMP, dt.VARIANT_REVCOMP | dt.VARIANT_OVERLAP):
        v = _banded(dt.Vocab(dt.KMER, k=6), 16384)
        w_ids, w_off = _want_variant(dt.KMER, 6, data, offs, True, variant)
        W = int(np.diff(w_off).max())
        p_ids, p_mask = oracle.pad_threads(w_ids, w_off, W)
        ids, oo, mask = dt.encode(v, _dev(data), _dev(offs), h_offsets=offs, add_cls_sep=True, layout=dt.PADDED,
                                  pad_to=W, variant=variant)
        torch.cuda.synchronize()
        assert dt.sync_status() == 0
        assert np.array_equal(oo.cpu().numpy(), w_off)
        assert np.array_equal(ids.cpu().numpy(), p_ids) and np.array_equal(mask.cpu().numpy(), p_mask)


def test_bands_rows_longer_than_the_stage_go_in_parts():
    """Rows longer than the stage are cut into parts (tokens owned by the part
    their first byte falls in; the first part writes the leading pads and
    CLS, the last non-empty part SEP and the trailing pads): ragged rows of
    up to 20,000 bytes through a 4 KiB stage, every kind and variant, both
    pad sides, extra padding, misaligned input and output."""
    torch = _torch()
    data, offs = _fuzz_batch(3700, 90, 20000)
    lut = oracle.fallback_lut()
    cases = [(dt.KMER, k, var) for k in (1, 3, 6, 8, 13) for var in (0, dt.VARIANT_REVCOMP, dt.VARIANT_OVERLAP,
                                                                         dt.VARIANT_REVCOMP | dt.VARIANT_OVERLAP)]
    cases += [(dt.SINGLE, 1, 0), (dt.SINGLE, 1, dt.VARIANT_REVCOMP), (dt.LUT256, 1, dt.VARIANT_REVCOMP)]
    n = len(offs) - 1
    for kind, k, variant in cases:
        v = _banded(dt.Vocab(kind, k=k, lut256=lut if kind == dt.LUT256 else None), 4096)
        for cls, side, extra in ((True, dt.PAD_RIGHT, 5), (False, dt.PAD_LEFT, 0)):
            w_ids, w_off = _want_variant(kind, k, data, offs, cls, variant, lut=lut if kind == dt.LUT256 else None)
            W = max(1, int(np.diff(w_off).max()) + extra)
            p_ids, p_mask = oracle.pad(w_ids, w_off, W, side)
            print("parts kind=%d k=%d variant=%d cls=%d side=%d" % (kind, k, variant, cls, side), flush=True)
            ids, oo, mask = dt.encode(v, _dev(data), _dev(offs), h_offsets=offs, add_cls_sep=cls, layout=dt.PADDED,
                                      pad_side=side, pad_to=W, variant=variant)
            torch.cuda.synchronize()
            assert dt.sync_status() == 0
            assert np.array_equal(oo.cpu().numpy(), w_off)
            g = ids.cpu().numpy()
            bad = np.argwhere(g != p_ids)
            assert bad.size == 0, "first mismatch at %s: got %d want %d" % (
                bad[0], g[tuple(bad[0])], p_ids[tuple(bad[0])])
            assert np.array_equal(mask.cpu().numpy(), p_mask)
        v.close()
    # several vocabularies, misaligned input and outputs, through 4 KiB parts
    ks = [2, 3, 5, 6]
    vs = [dt.Vocab(dt.KMER, k=k) for k in ks]
    _banded(vs[0], 4096)
    _check(vs, [(dt.KMER, k) for k in ks], data, offs, True, dt.PAD_RIGHT, byte_shift=3, id_shift=1)
    _check(vs, [(dt.KMER, k) for k in ks], data, offs, False, dt.PAD_LEFT, pad_extra=9)
    assert n == 90
