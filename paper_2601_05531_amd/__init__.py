"""Python binding of ``libdnatok.so`` (the MI355X DNA byte->identifier tokenizer).

Argument marshalling only: every step of the tokenizer runs in the HIP
library behind ``include/dnatok.h``. The functions named ``dnatok_*`` mirror
the C-ABI one to one (ints for device pointers and streams). The lower-case
helpers (``Vocab``, ``encode``, ``decode``) take PyTorch tensors, which serve
only as device memory and streams.

There is no fallback: if the library is not built, importing the binding
works but the first call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdnatok.so")

OK, EINVAL, EVOCAB, ENOMEM, EBUDGET, EDEVICE, ESTATE, ETOOSMALL = 0, -1, -2, -3, -4, -5, -6, -7
DERR_OFFSETS, DERR_CAPACITY, DERR_ROW_WIDTH, DERR_INTERNAL, DERR_IDS = 1, 2, 4, 8, 16
VARIANT_REVCOMP, VARIANT_OVERLAP = 1, 2
SINGLE, LUT256, KMER, BPE = 0, 1, 2, 3
PACKED, PADDED = 0, 1
PAD_RIGHT, PAD_LEFT = 0, 1
ID_PAD, ID_UNK, ID_CLS, ID_SEP, ID_MASK = 0, 1, 2, 3, 4


class DnatokError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("dnatok error %d: %s" % (code, msg))
        self.code = code


class dnatok_vocab_desc(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("k", ctypes.c_int32),
        ("lut256", ctypes.POINTER(ctypes.c_int32)),
        ("pad_id", ctypes.c_int32),
        ("cls_id", ctypes.c_int32),
        ("sep_id", ctypes.c_int32),
        ("n_merges", ctypes.c_int32),
        ("merges", ctypes.POINTER(ctypes.c_int32)),
    ]


class dnatok_encode_opts(ctypes.Structure):
    _fields_ = [
        ("add_cls_sep", ctypes.c_int32),
        ("layout", ctypes.c_int32),
        ("pad_side", ctypes.c_int32),
        ("variant", ctypes.c_int32),
        ("pad_to", ctypes.c_int64),
        ("offset_base", ctypes.c_int64),
    ]


class dnatok_stream_opts(ctypes.Structure):
    _fields_ = [
        ("window", ctypes.c_int64),
        ("chunk_bytes", ctypes.c_int64),
        ("n_slots", ctypes.c_int32),
        ("add_cls_sep", ctypes.c_int32),
        ("overlap", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("max_tokens", ctypes.c_int64),
        ("max_windows", ctypes.c_int64),
    ]


class dnatok_stream_result(ctypes.Structure):
    _fields_ = [
        ("d_ids", ctypes.c_void_p),
        ("d_window_offsets", ctypes.c_void_p),
        ("n_windows", ctypes.c_int64),
        ("n_tokens", ctypes.c_int64),
        ("n_bytes", ctypes.c_int64),
    ]


class dnatok_tuning(ctypes.Structure):
    _fields_ = [
        ("tile_bytes", ctypes.c_int32),
        ("blocks_per_cu", ctypes.c_int32),
        ("bpe_item_bytes", ctypes.c_int32),
        ("bpe_max_waves", ctypes.c_int32),
        ("spread", ctypes.c_int32),
        ("bands", ctypes.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class dnatok_encode_call(ctypes.Structure):
    _fields_ = [
        ("v", ctypes.c_void_p),
        ("d_bytes", ctypes.c_void_p),
        ("nbytes", ctypes.c_int64),
        ("d_offsets", ctypes.c_void_p),
        ("n", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("d_ids", ctypes.c_void_p),
        ("ids_capacity", ctypes.c_int64),
        ("d_out_offsets", ctypes.c_void_p),
        ("d_mask", ctypes.c_void_p),
        ("opts", dnatok_encode_opts),
    ]


class dnatok_server_opts(ctypes.Structure):
    _fields_ = [
        ("budget_bytes", ctypes.c_int64),
        ("n_streams", ctypes.c_int32),
        ("max_batch", ctypes.c_int32),
        ("max_batch_bytes", ctypes.c_int64),
        ("staging_bytes", ctypes.c_int64),
    ]


class dnatok_request_result(ctypes.Structure):
    _fields_ = [
        ("d_ids", ctypes.c_void_p),
        ("n_tokens", ctypes.c_int64),
        ("status", ctypes.c_int32),
        ("dev_flags", ctypes.c_uint32),
        ("t_submit", ctypes.c_double),
        ("t_start", ctypes.c_double),
        ("t_done", ctypes.c_double),
    ]


class dnatok_ids_opts(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32),
        ("overlap", ctypes.c_int32),
        ("threads", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("token_budget", ctypes.c_int64),
        ("max_rows", ctypes.c_int64),
    ]


class dnatok_ids_result(ctypes.Structure):
    _fields_ = [
        ("rows", ctypes.c_int64),
        ("token_len", ctypes.c_int64),
        ("micro_rows", ctypes.c_int64),
        ("n_micro", ctypes.c_int64),
        ("h2d_bytes", ctypes.c_int64),
        ("map_s", ctypes.c_double),
        ("h2d_s", ctypes.c_double),
        ("total_s", ctypes.c_double),
    ]


_lib = None


def lib():
    """The loaded ``libdnatok.so`` (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libdnatok.so is not built (run __graft_entry__.build()); "
                               "there is no CPU fallback")
        # PyTorch ships its own HIP runtime (soname libamdhip64.so.7, loaded by
        # file name libamdhip64.so). Loading torch first lets the dynamic
        # loader satisfy this library's libamdhip64.so.7 dependency with that
        # same runtime, so torch's stream handles and allocations are valid
        # here; loading this library first would bring up a second runtime.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.dnatok_last_error.restype = ctypes.c_char_p
        L.dnatok_last_error.argtypes = []
        L.dnatok_version.restype = i32
        L.dnatok_vocab_create.argtypes = [ctypes.POINTER(dnatok_vocab_desc), ctypes.POINTER(vp)]
        L.dnatok_vocab_destroy.argtypes = [vp]
        L.dnatok_vocab_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.dnatok_encode_plan.argtypes = [vp, vp, i32, ctypes.POINTER(dnatok_encode_opts),
                                         ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.dnatok_encode.argtypes = [vp, vp, i64, vp, i32, vp, i64, vp, vp,
                                    ctypes.POINTER(dnatok_encode_opts), vp]
        L.dnatok_encode_noalloc.argtypes = [vp, vp, i64, vp, i32, vp, i64, vp, vp,
                                            ctypes.POINTER(dnatok_encode_opts), vp]
        L.dnatok_sync_status.argtypes = [vp, ctypes.POINTER(ctypes.c_uint32)]
        L.dnatok_encode_multi.argtypes = [vp, i32, vp, i64, vp, i32, vp, vp, vp, vp, vp, vp]
        L.dnatok_autotune_multi.argtypes = [vp, i32, vp, i64, vp, i32, vp, vp, vp, vp, vp, vp, i32,
                                            ctypes.POINTER(dnatok_tuning), ctypes.POINTER(ctypes.c_float)]
        L.dnatok_decode.argtypes = [vp, vp, i64, vp, i32, vp, i64, vp, vp]
        L.dnatok_stream_create.argtypes = [vp, ctypes.POINTER(dnatok_stream_opts), vp, ctypes.POINTER(vp)]
        L.dnatok_stream_push.argtypes = [vp, vp, i64, vp, i32]
        L.dnatok_stream_flush.argtypes = [vp, ctypes.POINTER(dnatok_stream_result)]
        L.dnatok_stream_reset.argtypes = [vp]
        L.dnatok_stream_destroy.argtypes = [vp]
        u64p = ctypes.POINTER(ctypes.c_uint64)
        L.dnatok_server_create.argtypes = [ctypes.POINTER(dnatok_server_opts), ctypes.POINTER(vp)]
        L.dnatok_server_submit.argtypes = [vp, vp, vp, i64, i32, u64p]
        L.dnatok_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(dnatok_request_result)]
        L.dnatok_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(dnatok_request_result)]
        L.dnatok_server_release.argtypes = [vp, ctypes.c_uint64]
        L.dnatok_server_now.argtypes = [vp]
        L.dnatok_server_now.restype = ctypes.c_double
        L.dnatok_server_stats.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.dnatok_server_destroy.argtypes = [vp]
        L.dnatok_get_tuning.argtypes = [vp, ctypes.POINTER(dnatok_tuning)]
        L.dnatok_set_tuning.argtypes = [vp, ctypes.POINTER(dnatok_tuning)]
        L.dnatok_autotune.argtypes = [vp, vp, i64, vp, i32, vp, i64, vp, vp, ctypes.POINTER(dnatok_encode_opts),
                                      vp, i32, ctypes.POINTER(dnatok_tuning), ctypes.POINTER(ctypes.c_float)]
        L.dnatok_graph_create.argtypes = [ctypes.POINTER(dnatok_encode_call), i32, ctypes.POINTER(vp)]
        L.dnatok_graph_launch.argtypes = [vp, vp]
        L.dnatok_graph_destroy.argtypes = [vp]
        L.dnatok_embed.argtypes = [vp, vp, i64, vp, i32, vp, i64, i64, vp, i64, vp, vp, vp,
                                   ctypes.POINTER(dnatok_encode_opts), vp]
        L.dnatok_embed_ids.argtypes = [vp, i64, vp, i64, i64, vp, vp]
        L.dnatok_ids_create.argtypes = [vp, ctypes.POINTER(dnatok_ids_opts), vp, ctypes.POINTER(vp)]
        L.dnatok_ids_run.argtypes = [vp, vp, i64, i64, i64, vp, vp, i64, i64, vp, ctypes.POINTER(dnatok_ids_result)]
        L.dnatok_ids_destroy.argtypes = [vp]
        L.dnatok_ids_map.argtypes = [vp, i32, vp, i64, i64, i64, i32, vp, i32]
        for name in ("dnatok_vocab_create", "dnatok_vocab_destroy", "dnatok_vocab_info", "dnatok_encode_plan",
                     "dnatok_encode", "dnatok_sync_status", "dnatok_decode", "dnatok_stream_create",
                     "dnatok_stream_push", "dnatok_stream_flush", "dnatok_stream_reset", "dnatok_stream_destroy",
                     "dnatok_server_create", "dnatok_server_submit", "dnatok_server_poll", "dnatok_server_wait",
                     "dnatok_server_release", "dnatok_server_stats", "dnatok_server_destroy", "dnatok_get_tuning",
                     "dnatok_set_tuning", "dnatok_autotune", "dnatok_graph_create", "dnatok_graph_launch",
                     "dnatok_graph_destroy", "dnatok_encode_multi", "dnatok_autotune_multi", "dnatok_embed",
                     "dnatok_embed_ids", "dnatok_encode_noalloc", "dnatok_ids_create", "dnatok_ids_run",
                     "dnatok_ids_destroy", "dnatok_ids_map"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc: int):
    if rc != OK:
        raise DnatokError(rc, lib().dnatok_last_error().decode())
    return rc


# ---- C-ABI mirrors ------------------------------------------------------------

def dnatok_last_error() -> str:
    return lib().dnatok_last_error().decode()


def dnatok_version() -> int:
    return lib().dnatok_version()


def dnatok_vocab_create(desc: dnatok_vocab_desc) -> int:
    h = ctypes.c_void_p()
    _check(lib().dnatok_vocab_create(ctypes.byref(desc), ctypes.byref(h)))
    return h.value


def dnatok_vocab_destroy(handle: int) -> int:
    return _check(lib().dnatok_vocab_destroy(handle))


def dnatok_vocab_info(handle: int):
    vs, mt = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().dnatok_vocab_info(handle, ctypes.byref(vs), ctypes.byref(mt)))
    return vs.value, mt.value


def dnatok_encode_plan(handle: int, h_offsets: np.ndarray, n: int, opts: dnatok_encode_opts):
    tot, mx = ctypes.c_int64(), ctypes.c_int64()
    h_offsets = np.ascontiguousarray(h_offsets, dtype=np.int64)
    _check(lib().dnatok_encode_plan(handle, h_offsets.ctypes.data, n, ctypes.byref(opts),
                                    ctypes.byref(tot), ctypes.byref(mx)))
    return tot.value, mx.value


def dnatok_encode(handle, d_bytes, nbytes, d_offsets, n, d_ids, ids_capacity, d_out_offsets, d_mask, opts,
                  stream) -> int:
    return _check(lib().dnatok_encode(handle, d_bytes, nbytes, d_offsets, n, d_ids, ids_capacity, d_out_offsets,
                                      d_mask, ctypes.byref(opts), stream))


def dnatok_encode_noalloc(handle, d_bytes, nbytes, d_offsets, n, d_ids, ids_capacity, d_out_offsets, d_mask, opts,
                          stream) -> int:
    return _check(lib().dnatok_encode_noalloc(handle, d_bytes, nbytes, d_offsets, n, d_ids, ids_capacity,
                                              d_out_offsets, d_mask, ctypes.byref(opts), stream))


def dnatok_embed(handle, d_bytes, nbytes, d_offsets, n, d_table, n_rows, row_bytes, d_out, out_rows, d_out_offsets,
                 d_ids, d_mask, opts, stream) -> int:
    return _check(lib().dnatok_embed(handle, d_bytes, nbytes, d_offsets, n, d_table, n_rows, row_bytes, d_out,
                                     out_rows, d_out_offsets, d_ids, d_mask, ctypes.byref(opts), stream))


def dnatok_embed_ids(d_ids, n_ids, d_table, n_rows, row_bytes, d_out, stream) -> int:
    return _check(lib().dnatok_embed_ids(d_ids, n_ids, d_table, n_rows, row_bytes, d_out, stream))


def dnatok_sync_status(stream) -> int:
    f = ctypes.c_uint32()
    _check(lib().dnatok_sync_status(stream, ctypes.byref(f)))
    return f.value


def dnatok_decode(handle, d_ids, n_ids, d_offsets, n, d_out, out_capacity, d_out_offsets, stream) -> int:
    return _check(lib().dnatok_decode(handle, d_ids, n_ids, d_offsets, n, d_out, out_capacity, d_out_offsets,
                                      stream))


def dnatok_stream_create(vocab_handle, opts: dnatok_stream_opts, compute_stream) -> int:
    h = ctypes.c_void_p()
    _check(lib().dnatok_stream_create(vocab_handle, ctypes.byref(opts), compute_stream, ctypes.byref(h)))
    return h.value


def dnatok_stream_push(handle, h_pinned, nbytes, record_ends, n_ends) -> int:
    return _check(lib().dnatok_stream_push(handle, h_pinned, nbytes, record_ends, n_ends))


def dnatok_stream_flush(handle) -> dnatok_stream_result:
    r = dnatok_stream_result()
    _check(lib().dnatok_stream_flush(handle, ctypes.byref(r)))
    return r


def dnatok_stream_reset(handle) -> int:
    return _check(lib().dnatok_stream_reset(handle))


def dnatok_stream_destroy(handle) -> int:
    return _check(lib().dnatok_stream_destroy(handle))


# ---- torch-facing helpers ----------------------------------------------------------

def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _ptr(t):
    return None if t is None else t.data_ptr()


class Vocab:
    """Owning wrapper of a ``dnatok_vocab`` handle on the current device."""

    def __init__(self, kind: int, k: int = 1, lut256=None, merges=None, pad_id: int = ID_PAD,
                 cls_id: int = ID_CLS, sep_id: int = ID_SEP):
        self.kind, self.k = kind, k
        d = dnatok_vocab_desc()
        d.kind, d.k = kind, k
        d.pad_id, d.cls_id, d.sep_id = pad_id, cls_id, sep_id
        self._lut = None if lut256 is None else np.ascontiguousarray(lut256, dtype=np.int32)
        self._merges = None if merges is None else np.ascontiguousarray(merges, dtype=np.int32).reshape(-1, 2)
        if self._lut is not None:
            d.lut256 = self._lut.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        if self._merges is not None:
            d.n_merges = len(self._merges)
            d.merges = self._merges.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        self.handle = dnatok_vocab_create(d)
        self.vocab_size, self.max_token_bytes = dnatok_vocab_info(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            dnatok_vocab_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_opts(add_cls_sep=False, layout=PACKED, pad_side=PAD_RIGHT, pad_to=0, offset_base=0, variant=0):
    o = dnatok_encode_opts()
    o.add_cls_sep, o.layout, o.pad_side, o.pad_to, o.offset_base = int(add_cls_sep), layout, pad_side, pad_to, offset_base
    o.variant = variant
    return o


def plan(vocab: Vocab, h_offsets, add_cls_sep=False, variant=0):
    h_offsets = np.ascontiguousarray(h_offsets, dtype=np.int64)
    return dnatok_encode_plan(vocab.handle, h_offsets, len(h_offsets) - 1, make_opts(add_cls_sep, variant=variant))


def encode(vocab: Vocab, d_bytes, d_offsets, h_offsets=None, add_cls_sep=False, layout=PACKED,
           pad_side=PAD_RIGHT, pad_to=None, out=None, stream=None, variant=0):
    """Encode a ragged batch held in device tensors.

    ``d_bytes``: uint8 cuda tensor; ``d_offsets``: int64 cuda tensor [n+1];
    ``h_offsets``: the same offsets on the host (numpy) for output sizing
    (copied from the device when omitted). Returns ``(ids, out_offsets, mask)``
    (``mask`` is None for PACKED). ``out`` may pass preallocated
    ``(ids, out_offsets, mask)``. ``variant``: 0 or an OR of VARIANT_REVCOMP
    and VARIANT_OVERLAP.
    """
    import torch
    n = d_offsets.numel() - 1
    if h_offsets is None:
        h_offsets = d_offsets.cpu().numpy()
    total, max_len = plan(vocab, h_offsets, add_cls_sep, variant)
    dev = d_bytes.device
    if layout == PADDED:
        if pad_to is None:
            W = max_len
        elif vocab.kind == BPE:
            # the BPE plan is only an upper bound: keep the caller's width (a
            # longer row raises DNATOK_DERR_ROW_WIDTH on the device)
            W = int(pad_to)
        else:
            W = max(int(pad_to), max_len)
        cap = n * W
    else:
        W, cap = 0, total
    if out is None:
        ids = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        out_off = torch.empty(n + 1, dtype=torch.int64, device=dev)
        mask = torch.empty(max(cap, 1), dtype=torch.int8, device=dev) if layout == PADDED else None
    else:
        ids, out_off, mask = out
    opts = make_opts(add_cls_sep, layout, pad_side, W, variant=variant)
    dnatok_encode(vocab.handle, _ptr(d_bytes), d_bytes.numel(), _ptr(d_offsets), n, _ptr(ids), ids.numel(),
                  _ptr(out_off), _ptr(mask), opts, _stream_ptr(stream))
    if layout == PADDED:
        return ids[:cap].view(n, W) if n else ids[:0].view(0, W), out_off, mask[:cap].view(n, W) if n else mask[:0]
    if vocab.kind == BPE:
        # the plan is an upper bound for BPE (one token per base); the real
        # total is known once the device has encoded (a synchronising read)
        total = int(out_off[n].item())
    return ids[:total], out_off, None


def embed(vocab: Vocab, d_bytes, d_offsets, table, h_offsets=None, add_cls_sep=False, layout=PACKED,
          pad_side=PAD_RIGHT, pad_to=None, variant=0, want_ids=False, want_mask=True, out=None, stream=None):
    """Encode fused with the embedding lookup (``dnatok_embed``).

    ``table``: a 2-D cuda tensor [n_rows, D] of any dtype (rows are copied bit
    for bit). Returns ``(emb, out_offsets, ids, mask)``: ``emb`` is
    [total, D] (PACKED) or [n, W, D] (PADDED) in the table's dtype; ``ids``
    and ``mask`` are None unless asked for (``mask``: PADDED only). ``out``
    may pass a preallocated ``emb`` buffer of at least that many rows.
    """
    import torch
    n = d_offsets.numel() - 1
    if h_offsets is None:
        h_offsets = d_offsets.cpu().numpy()
    total, max_len = plan(vocab, h_offsets, add_cls_sep, variant)
    dev = d_bytes.device
    if layout == PADDED:
        W = max_len if pad_to is None else max(int(pad_to), max_len)
        rows = n * W
    else:
        W, rows = 0, total
    row_bytes = table.stride(0) * table.element_size()
    assert table.dim() == 2 and table.is_contiguous()
    emb = out if out is not None else torch.empty((max(rows, 1), table.shape[1]), dtype=table.dtype, device=dev)
    out_off = torch.empty(n + 1, dtype=torch.int64, device=dev)
    ids = torch.empty(max(rows, 1), dtype=torch.int32, device=dev) if want_ids else None
    mask = torch.empty(max(rows, 1), dtype=torch.int8, device=dev) if (want_mask and layout == PADDED) else None
    opts = make_opts(add_cls_sep, layout, pad_side, W, variant=variant)
    dnatok_embed(vocab.handle, _ptr(d_bytes), d_bytes.numel(), _ptr(d_offsets), n, _ptr(table), table.shape[0],
                 row_bytes, _ptr(emb), emb.shape[0], _ptr(out_off), _ptr(ids), _ptr(mask), opts, _stream_ptr(stream))
    if layout == PADDED:
        shape = (n, W)
        return (emb[:rows].view(n, W, table.shape[1]), out_off,
                ids[:rows].view(shape) if ids is not None else None,
                mask[:rows].view(shape) if mask is not None else None)
    return emb[:rows], out_off, (ids[:rows] if ids is not None else None), None


def embed_ids(d_ids, table, stream=None):
    """Embedding lookup of an int32 cuda id tensor (``dnatok_embed_ids``):
    returns ``table[ids]`` computed on the device, shape ids.shape + (D,)."""
    import torch
    assert table.dim() == 2 and table.is_contiguous() and d_ids.dtype == torch.int32
    ids = d_ids.contiguous()
    out = torch.empty((max(ids.numel(), 1), table.shape[1]), dtype=table.dtype, device=ids.device)
    dnatok_embed_ids(_ptr(ids), ids.numel(), _ptr(table), table.shape[0], table.stride(0) * table.element_size(),
                     _ptr(out), _stream_ptr(stream))
    return out[:ids.numel()].view(tuple(ids.shape) + (table.shape[1],))


def decode(vocab: Vocab, d_ids, d_offsets, out_capacity=None, stream=None):
    """Decode PACKED rows. Returns ``(bytes uint8 cuda tensor, out_offsets)``;
    the bytes tensor is sized by ``out_capacity`` (default n_ids * max_token_bytes)."""
    import torch
    n = d_offsets.numel() - 1
    cap = out_capacity if out_capacity is not None else max(1, d_ids.numel() * vocab.max_token_bytes)
    out = torch.empty(max(cap, 1), dtype=torch.uint8, device=d_ids.device)
    out_off = torch.empty(n + 1, dtype=torch.int64, device=d_ids.device)
    dnatok_decode(vocab.handle, _ptr(d_ids), d_ids.numel(), _ptr(d_offsets), n, _ptr(out), cap, _ptr(out_off),
                  _stream_ptr(stream))
    return out, out_off


class Stream:
    """Owning wrapper of a ``dnatok_stream``: pinned host chunks in, windows of
    ``window`` bases encoded on the device (see ``dnatok_stream_*``)."""

    def __init__(self, vocab: Vocab, window: int, chunk_bytes: int, max_tokens: int, max_windows: int,
                 n_slots: int = 3, add_cls_sep: bool = False, overlap: bool = True, stream=None):
        o = dnatok_stream_opts()
        o.window, o.chunk_bytes, o.n_slots = window, chunk_bytes, n_slots
        o.add_cls_sep, o.overlap = int(add_cls_sep), int(overlap)
        o.max_tokens, o.max_windows = max_tokens, max_windows
        self.vocab = vocab
        self.handle = dnatok_stream_create(vocab.handle, o, _stream_ptr(stream))

    def push(self, h_chunk, record_ends=()):
        """``h_chunk``: pinned uint8 CPU tensor (a slice of one is fine)."""
        ends = np.ascontiguousarray(record_ends, dtype=np.int64)
        dnatok_stream_push(self.handle, h_chunk.data_ptr(), h_chunk.numel(),
                           ends.ctypes.data if len(ends) else None, len(ends))

    def flush(self, copy: bool = True):
        """Returns ``(ids, window_offsets, result)``: device tensors over the
        stream's output (torch-owned copies, or zero-copy views valid until
        reset/close when ``copy`` is False)."""
        r = dnatok_stream_flush(self.handle)
        ids = device_view(r.d_ids, r.n_tokens, "<i4")
        woff = device_view(r.d_window_offsets, r.n_windows + 1, "<i8")
        if copy:
            ids, woff = ids.clone(), woff.clone()
        return ids, woff, r

    def reset(self):
        dnatok_stream_reset(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            dnatok_stream_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _DeviceArray:
    """Exposes library-owned device memory through __cuda_array_interface__."""

    def __init__(self, ptr, n, typestr):
        self.__cuda_array_interface__ = {"shape": (int(n),), "typestr": typestr, "data": (int(ptr or 0), False),
                                         "version": 3, "strides": None}


def device_view(ptr, n, typestr):
    """Zero-copy torch tensor over device memory the library owns."""
    import torch
    if n == 0:
        return torch.empty(0, dtype={"<i4": torch.int32, "<i8": torch.int64, "|u1": torch.uint8}[typestr],
                           device="cuda")
    return torch.as_tensor(_DeviceArray(ptr, n, typestr), device="cuda")


def sync_status(stream=None) -> int:
    return dnatok_sync_status(_stream_ptr(stream))


# ---- serving loop ------------------------------------------------------------------

def dnatok_server_create(opts: dnatok_server_opts) -> int:
    h = ctypes.c_void_p()
    _check(lib().dnatok_server_create(ctypes.byref(opts), ctypes.byref(h)))
    return h.value


def dnatok_server_submit(server: int, vocab: int, h_bytes: int, nbytes: int, add_cls_sep: int) -> int:
    t = ctypes.c_uint64()
    _check(lib().dnatok_server_submit(server, vocab, h_bytes, nbytes, add_cls_sep, ctypes.byref(t)))
    return t.value


def dnatok_server_poll(server: int, ticket: int):
    r = dnatok_request_result()
    rc = lib().dnatok_server_poll(server, ticket, ctypes.byref(r))
    if rc < 0:
        _check(rc)
    return (r if rc == 0 else None)


def dnatok_server_wait(server: int, ticket: int) -> dnatok_request_result:
    r = dnatok_request_result()
    _check(lib().dnatok_server_wait(server, ticket, ctypes.byref(r)))
    return r


def dnatok_server_release(server: int, ticket: int) -> int:
    return _check(lib().dnatok_server_release(server, ticket))


def dnatok_server_now(server: int) -> float:
    return lib().dnatok_server_now(server)


def dnatok_server_stats(server: int):
    a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib().dnatok_server_stats(server, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def dnatok_server_destroy(server: int) -> int:
    return _check(lib().dnatok_server_destroy(server))


class Server:
    """Owning wrapper of a ``dnatok_server`` on the current device."""

    def __init__(self, budget_bytes: int = 16 << 30, n_streams: int = 4, max_batch: int = 256,
                 max_batch_bytes: int = 16 << 20, staging_bytes: int | None = None):
        o = dnatok_server_opts()
        o.budget_bytes, o.n_streams, o.max_batch = budget_bytes, n_streams, max_batch
        o.max_batch_bytes = max_batch_bytes
        o.staging_bytes = max_batch_bytes if staging_bytes is None else staging_bytes
        self.handle = dnatok_server_create(o)
        self._keep = {}

    def submit(self, vocab: Vocab, data, add_cls_sep: bool = True) -> int:
        """``data``: a numpy uint8 array (copied at once) or a pinned uint8
        torch tensor (read by the device later: keep it until done)."""
        if isinstance(data, np.ndarray):
            a = np.ascontiguousarray(data, dtype=np.uint8)
            t = dnatok_server_submit(self.handle, vocab.handle, a.ctypes.data, a.size, int(add_cls_sep))
        else:
            t = dnatok_server_submit(self.handle, vocab.handle, data.data_ptr(), data.numel(), int(add_cls_sep))
            self._keep[t] = data
        return t

    def wait(self, ticket: int):
        """Returns (device ids view, result struct); the view is valid until release."""
        r = dnatok_server_wait(self.handle, ticket)
        if r.status != OK:
            raise DnatokError(r.status, "request %d failed" % ticket)
        ids = device_view(r.d_ids, r.n_tokens, "<i4")
        return ids, r

    def release(self, ticket: int):
        self._keep.pop(ticket, None)
        dnatok_server_release(self.handle, ticket)

    def now(self) -> float:
        return dnatok_server_now(self.handle)

    def stats(self):
        return dnatok_server_stats(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            dnatok_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- tuning, autotuner, captured graphs ----------------------------------------------

def dnatok_get_tuning(vocab: int) -> dnatok_tuning:
    t = dnatok_tuning()
    _check(lib().dnatok_get_tuning(vocab, ctypes.byref(t)))
    return t


def dnatok_set_tuning(vocab: int, t: dnatok_tuning) -> int:
    return _check(lib().dnatok_set_tuning(vocab, ctypes.byref(t)))


def dnatok_autotune(vocab, d_bytes, nbytes, d_offsets, n, d_ids, ids_capacity, d_out_offsets, d_mask, opts, stream,
                    reps=3):
    t, ms = dnatok_tuning(), ctypes.c_float()
    _check(lib().dnatok_autotune(vocab, d_bytes, nbytes, d_offsets, n, d_ids, ids_capacity, d_out_offsets, d_mask,
                                 ctypes.byref(opts), stream, reps, ctypes.byref(t), ctypes.byref(ms)))
    return t, ms.value


def set_tuning(vocab: Vocab, tile_bytes=0, blocks_per_cu=0, bpe_item_bytes=0, bpe_max_waves=0, spread=0, bands=0):
    dnatok_set_tuning(vocab.handle, dnatok_tuning(tile_bytes, blocks_per_cu, bpe_item_bytes, bpe_max_waves, spread,
                                                  bands))


def autotune(vocab: Vocab, d_bytes, d_offsets, h_offsets=None, add_cls_sep=False, layout=PACKED, pad_side=PAD_RIGHT,
             pad_to=None, reps=3, stream=None, variant=0):
    """Time every candidate tiling on this batch and keep the fastest in the
    vocabulary. Returns (tuning dict, median ms)."""
    import torch
    n = d_offsets.numel() - 1
    if h_offsets is None:
        h_offsets = d_offsets.cpu().numpy()
    total, max_len = plan(vocab, h_offsets, add_cls_sep, variant)
    if layout == PADDED:
        W = max_len if pad_to is None else int(pad_to)
        cap = n * W
    else:
        W, cap = 0, total
    ids = torch.empty(max(cap, 1), dtype=torch.int32, device=d_bytes.device)
    oo = torch.empty(n + 1, dtype=torch.int64, device=d_bytes.device)
    mask = torch.empty(max(cap, 1), dtype=torch.int8, device=d_bytes.device) if layout == PADDED else None
    t, ms = dnatok_autotune(vocab.handle, _ptr(d_bytes), d_bytes.numel(), _ptr(d_offsets), n, _ptr(ids), ids.numel(),
                            _ptr(oo), _ptr(mask), make_opts(add_cls_sep, layout, pad_side, W, variant=variant),
                            _stream_ptr(stream), reps)
    return t.as_dict(), ms


class Graph:
    """Captured dnatok_encode calls over fixed buffers (see dnatok_graph_create).

    ``calls``: a list of dicts with keys vocab, d_bytes, d_offsets, d_ids,
    d_out_offsets and optionally d_mask, add_cls_sep, layout, pad_side,
    pad_to, variant (tensors on the device)."""

    def __init__(self, calls):
        arr = (dnatok_encode_call * len(calls))()
        self._keep = []
        for c, d in zip(arr, calls):
            c.v = d["vocab"].handle
            c.d_bytes = _ptr(d["d_bytes"])
            c.nbytes = d["d_bytes"].numel()
            c.d_offsets = _ptr(d["d_offsets"])
            c.n = d["d_offsets"].numel() - 1
            c.d_ids = _ptr(d["d_ids"])
            c.ids_capacity = d["d_ids"].numel()
            c.d_out_offsets = _ptr(d["d_out_offsets"])
            c.d_mask = _ptr(d.get("d_mask"))
            c.opts = make_opts(d.get("add_cls_sep", False), d.get("layout", PACKED), d.get("pad_side", PAD_RIGHT),
                               d.get("pad_to", 0), variant=d.get("variant", 0))
            self._keep.append(d)
        h = ctypes.c_void_p()
        _check(lib().dnatok_graph_create(arr, len(calls), ctypes.byref(h)))
        self.handle = h.value

    def launch(self, stream=None):
        _check(lib().dnatok_graph_launch(self.handle, _stream_ptr(stream)))

    def close(self):
        if getattr(self, "handle", None):
            lib().dnatok_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- several k-mer vocabularies in one pass -------------------------------------------

class MultiCall:
    """Marshalled arguments of dnatok_encode_multi (host arrays kept alive)."""

    def __init__(self, vocabs, d_bytes, d_offsets, outs, opts):
        nv = len(vocabs)
        self.nv = nv
        self.vocabs = (ctypes.c_void_p * nv)(*[v.handle for v in vocabs])
        self.ids = (ctypes.c_void_p * nv)(*[_ptr(o[0]) for o in outs])
        self.caps = (ctypes.c_int64 * nv)(*[o[0].numel() for o in outs])
        self.oofs = (ctypes.c_void_p * nv)(*[_ptr(o[1]) for o in outs])
        self.masks = (ctypes.c_void_p * nv)(*[_ptr(o[2]) for o in outs])
        self.opts = (dnatok_encode_opts * nv)(*opts)
        self.d_bytes, self.nbytes = _ptr(d_bytes), d_bytes.numel()
        self.d_offsets, self.n = _ptr(d_offsets), d_offsets.numel() - 1
        self._keep = (vocabs, d_bytes, d_offsets, outs)

    def args(self):
        return (self.vocabs, self.nv, self.d_bytes, self.nbytes, self.d_offsets, self.n, self.ids, self.caps,
                self.oofs, self.masks, self.opts)

    def run(self, stream=None):
        _check(lib().dnatok_encode_multi(*self.args(), _stream_ptr(stream)))

    def autotune(self, reps=3, stream=None):
        t, ms = dnatok_tuning(), ctypes.c_float()
        _check(lib().dnatok_autotune_multi(*self.args(), _stream_ptr(stream), reps, ctypes.byref(t),
                                           ctypes.byref(ms)))
        return t.as_dict(), ms.value


def encode_multi(vocabs, d_bytes, d_offsets, h_offsets=None, add_cls_sep=False, layout=PACKED, pad_side=PAD_RIGHT,
                 stream=None):
    """Encode one batch for several k-mer vocabularies in one pass. Returns a
    list of (ids, out_offsets, mask) per vocabulary, as ``encode``."""
    import torch
    n = d_offsets.numel() - 1
    if h_offsets is None:
        h_offsets = d_offsets.cpu().numpy()
    outs, opts, shapes = [], [], []
    for v in vocabs:
        total, max_len = plan(v, h_offsets, add_cls_sep)
        W = max_len if layout == PADDED else 0
        cap = n * W if layout == PADDED else total
        ids = torch.empty(max(cap, 1), dtype=torch.int32, device=d_bytes.device)
        oo = torch.empty(n + 1, dtype=torch.int64, device=d_bytes.device)
        mask = torch.empty(max(cap, 1), dtype=torch.int8, device=d_bytes.device) if layout == PADDED else None
        outs.append((ids, oo, mask))
        opts.append(make_opts(add_cls_sep, layout, pad_side, W))
        shapes.append((cap, W, total))
    MultiCall(vocabs, d_bytes, d_offsets, outs, opts).run(stream)
    res = []
    for (ids, oo, mask), (cap, W, total) in zip(outs, shapes):
        if layout == PADDED:
            res.append((ids[:cap].view(n, W), oo, mask[:cap].view(n, W)))
        else:
            res.append((ids[:total], oo, None))
    return res


# ---- IDs path (host mapping, staged id transfer) ----------------------------------

def dnatok_ids_map(lut256, pad_id: int, h_bytes: np.ndarray, n_rows: int, row_len: int, token_len: int, width: int,
                   threads: int = 0) -> np.ndarray:
    """Host mapping step alone: returns int32 or int64 ids [n_rows, T']."""
    lut = np.ascontiguousarray(lut256, dtype=np.int32)
    assert lut.shape == (256,)
    src = np.ascontiguousarray(h_bytes, dtype=np.uint8)
    T = token_len or row_len
    out = np.empty((n_rows, T), dtype=np.int32 if width == 4 else np.int64)
    _check(lib().dnatok_ids_map(lut.ctypes.data, pad_id, src.ctypes.data if src.size else None, n_rows, row_len,
                                token_len, width, out.ctypes.data if out.size else None, threads))
    return out


class IdsPath:
    """Owning wrapper of a ``dnatok_ids`` (see ``dnatok_ids_*``)."""

    def __init__(self, vocab: Vocab, width: int = 8, overlap: bool = False, threads: int = 0, token_budget: int = 0,
                 max_rows: int = 0, stream=None):
        o = dnatok_ids_opts(width, int(overlap), threads, 0, token_budget, max_rows)
        h = ctypes.c_void_p()
        _check(lib().dnatok_ids_create(vocab.handle, ctypes.byref(o), _stream_ptr(stream), ctypes.byref(h)))
        self.handle = h.value
        self.vocab = vocab

    def run(self, h_bytes, n_rows: int, row_len: int, token_len: int = 0, d_ids=None, table=None, d_out=None):
        """``h_bytes``: host uint8 (numpy array or pinned tensor) of n_rows x
        row_len; ``d_ids`` int64 device tensor of n_rows x T' and/or
        ``d_out`` device tensor of n_rows x T' table rows. Returns the
        ``dnatok_ids_result``."""
        if isinstance(h_bytes, np.ndarray):
            src = np.ascontiguousarray(h_bytes, dtype=np.uint8)
            ptr = src.ctypes.data if src.size else None
        else:
            ptr = h_bytes.data_ptr()
        r = dnatok_ids_result()
        n_rows_t = 0 if table is None else table.shape[0]
        row_bytes = 0 if table is None else table[0].numel() * table.element_size()
        _check(lib().dnatok_ids_run(self.handle, ptr, n_rows, row_len, token_len, _ptr(d_ids), _ptr(table), n_rows_t,
                                    row_bytes, _ptr(d_out), ctypes.byref(r)))
        return r

    def close(self):
        if getattr(self, "handle", None):
            _check(lib().dnatok_ids_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
