"""dnatok_encode_noalloc, the encode entry point that allocates nothing: its
outputs equal dnatok_encode's (bit-exact) and the oracle's, for two calls in a
row with the second batch smaller, across kinds, layouts and a variant; it
works while every library allocation is made to fail (so it made none); a
batch beyond its fixed scratch is refused with EBUDGET before anything is
enqueued."""
import contextlib
import os

import numpy as np
import pytest

import oracle
import paper_2601_05531_amd as dt
import synth

pytestmark = pytest.mark.gpu

FAIL_ENV = "DNATOK_TEST_FAIL_ALLOC"


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    return torch


@contextlib.contextmanager
def no_library_allocation():
    """Every device or pinned allocation the library attempts fails."""
    os.environ[FAIL_ENV] = "1"
    try:
        yield
    finally:
        os.environ.pop(FAIL_ENV, None)


def _merges():
    corpus = synth.genome(synth.substream(95, 0), synth.substream(95, 1), 3, 300_000)
    return oracle.bpe_train(corpus, 300)


def _run(fn, v, data, offs, opts, stream):
    """One encode through the C-ABI entry point `fn` into fresh outputs
    pre-filled with a sentinel; returns (ids, out_offsets, mask) on the host."""
    torch = _torch()
    n = len(offs) - 1
    total, W = dt.plan(v, offs, bool(opts.add_cls_sep), int(opts.variant))
    if opts.layout == dt.PADDED:
        opts.pad_to = W
        cap = n * W
    else:
        cap = total
    d_in = torch.from_numpy(data).cuda()
    d_off = torch.from_numpy(offs).cuda()
    ids = torch.full((max(cap, 1),), -7, dtype=torch.int32, device="cuda")
    oo = torch.full((n + 1,), -7, dtype=torch.int64, device="cuda")
    mask = torch.full((max(cap, 1),), -7, dtype=torch.int8, device="cuda") if opts.layout == dt.PADDED else None
    torch.cuda.synchronize()
    fn(v.handle, d_in.data_ptr(), data.size, d_off.data_ptr(), n, ids.data_ptr(), cap, oo.data_ptr(),
       None if mask is None else mask.data_ptr(), opts, stream.cuda_stream)
    stream.synchronize()
    assert dt.sync_status(stream) == 0
    return (ids[:cap].cpu().numpy(), oo.cpu().numpy(), None if mask is None else mask[:cap].cpu().numpy(),
            int(opts.pad_to))


CASES = [
    ("6-mer PADDED cls", dict(kind=dt.KMER, k=6), dict(add_cls_sep=True, layout=dt.PADDED)),
    ("single PACKED", dict(kind=dt.SINGLE, k=1), dict(add_cls_sep=False, layout=dt.PACKED)),
    ("5-mer PACKED overlap revcomp", dict(kind=dt.KMER, k=5),
     dict(add_cls_sep=True, layout=dt.PACKED, variant=dt.VARIANT_OVERLAP | dt.VARIANT_REVCOMP)),
    ("BPE PADDED left", dict(kind=dt.BPE, k=1), dict(add_cls_sep=True, layout=dt.PADDED, pad_side=dt.PAD_LEFT)),
    ("BPE PACKED", dict(kind=dt.BPE, k=1), dict(add_cls_sep=False, layout=dt.PACKED)),
]


@pytest.mark.parametrize("name,vk,ok", CASES, ids=[c[0] for c in CASES])
def test_noalloc_equals_encode_two_calls_second_smaller(name, vk, ok):
    torch = _torch()
    merges = _merges() if vk["kind"] == dt.BPE else None
    v = dt.Vocab(vk["kind"], k=vk["k"], merges=merges)
    big = synth.workload_markov_batch(700, 3001)
    small = synth.workload_markov_batch(37, 999, seed=synth.substream(96, 1))
    stream = torch.cuda.Stream()
    for data, offs in (big, small):
        print("%s: n=%d nbytes=%d" % (name, len(offs) - 1, data.size), flush=True)
        with no_library_allocation():
            got = _run(dt.dnatok_encode_noalloc, v, data, offs, dt.make_opts(**ok), stream)
        ref = _run(dt.dnatok_encode, v, data, offs, dt.make_opts(**ok), stream)
        for g, r in zip(got[:3], ref[:3]):
            if r is not None:
                assert np.array_equal(g, r)
        # and both against the oracle
        variant = ok.get("variant", 0)
        src = oracle.revcomp(data, offs) if variant & dt.VARIANT_REVCOMP else data
        if variant & dt.VARIANT_OVERLAP:
            want, want_off = oracle.encode_overlap(src, offs, vk["k"], add_cls_sep=ok["add_cls_sep"])
        else:
            want, want_off = oracle.encode(vk["kind"], src, offs, k=vk["k"], merges=merges,
                                           add_cls_sep=ok["add_cls_sep"])
        assert np.array_equal(got[1], want_off)
        if ok["layout"] == dt.PADDED:
            W = got[3]  # the plan's width (for BPE an upper bound of the longest row)
            w_ids, w_mask = oracle.pad(want, want_off, W, ok.get("pad_side", dt.PAD_RIGHT))
            assert np.array_equal(got[0].reshape(-1, W), w_ids) and np.array_equal(got[2].reshape(-1, W), w_mask)
        else:
            assert np.array_equal(got[0][:int(got[1][-1])], want)
    v.close()


def test_noalloc_refuses_a_batch_beyond_its_scratch():
    torch = _torch()
    v = dt.Vocab(dt.BPE, merges=_merges())
    n = 10 << 20  # BPE scratch is about 4 bytes per input byte: beyond the fixed 32 MiB
    data = synth.iid(97, n, 0.01)
    offs = np.array([0, n // 2, n], dtype=np.int64)
    d_in = torch.from_numpy(data).cuda()
    d_off = torch.from_numpy(offs).cuda()
    ids = torch.full((n + 4,), -7, dtype=torch.int32, device="cuda")
    oo = torch.full((3,), -7, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    with pytest.raises(dt.DnatokError) as e:
        dt.dnatok_encode_noalloc(v.handle, d_in.data_ptr(), n, d_off.data_ptr(), 2, ids.data_ptr(), n + 4,
                                 oo.data_ptr(), None, dt.make_opts(False), None)
    assert e.value.code == dt.EBUDGET
    torch.cuda.synchronize()
    assert bool((ids == -7).all()) and bool((oo == -7).all())
    assert dt.sync_status() == 0
    # the same batch through dnatok_encode (which sizes its own scratch) still works
    dt.dnatok_encode(v.handle, d_in.data_ptr(), n, d_off.data_ptr(), 2, ids.data_ptr(), n + 4, oo.data_ptr(), None,
                     dt.make_opts(False), None)
    torch.cuda.synchronize()
    assert dt.sync_status() == 0
    assert int(oo[2].item()) > 0
    v.close()
