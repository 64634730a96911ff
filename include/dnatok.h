/*
 * dnatok.h — C-ABI of the MI355X DNA byte->identifier tokenizer.
 *
 * The operation (paper, Design): genomic tokenization reduces to mapping the
 * ASCII bytes of DNA strings to the integer identifiers an embedder consumes
 * (embed_tokens: Z^{B x T} -> R^{B x T x D}); the bytes path stages raw 8-bit
 * ASCII, moves it to the device once and applies a device-resident 256-entry
 * lookup table there (Design, "Encoding paths", bytes path; the bytes branch
 * of the EmbedFromStrings algorithm). This library is that bytes path for a
 * ragged batch, for single-nucleotide, non-overlapping k-mer and ranked-merge
 * BPE vocabularies (introduction; table of genomic tokenization schemes).
 *
 * Conventions
 *  - Every function returns an int status: DNATOK_OK (0) or a negative code.
 *    dnatok_last_error() describes the most recent failure of the calling
 *    thread. Nothing aborts and no C++ exception crosses this boundary.
 *  - Pointers named d_* are device memory of the device that was current
 *    when the vocabulary was created; h_* are host memory. The caller owns
 *    every buffer it passes; the library owns the handles it returns and the
 *    device tables and workspaces behind them.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls that take a stream only enqueue work on it and return at once;
 *    their device outputs are ready when the stream reaches that point.
 *  - All offsets and sizes are int64 (a 2 GiB stream already overflows
 *    32-bit indexing, cf. the 32-bit index overflow the paper guards against
 *    in "Robustness and compatibility").
 *  - Vocabulary handles are immutable after creation and may be shared by
 *    threads. Stream handles have a single owner.
 *
 * Id space (the paper delegates special ids to the upstream vocabulary; the
 * fixed reading used here): PAD=0 (the discovery algorithm's default pad
 * id), UNK=1, CLS=2, SEP=3, MASK=4, then the vocabulary's own ids.
 */
#ifndef DNATOK_H
#define DNATOK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define DNATOK_OK 0
#define DNATOK_EINVAL (-1)    /* bad argument (null pointer, size, enum) */
#define DNATOK_EVOCAB (-2)    /* vocabulary description rejected */
#define DNATOK_ENOMEM (-3)    /* device or pinned allocation failed */
#define DNATOK_EBUDGET (-4)   /* request exceeds a memory budget */
#define DNATOK_EDEVICE (-5)   /* a HIP runtime call failed */
#define DNATOK_ESTATE (-6)    /* handle in the wrong state for this call */
#define DNATOK_ETOOSMALL (-7) /* an output capacity is too small */

/* ---- device-side error flags (dnatok_sync_status) ------------------------ */
#define DNATOK_DERR_OFFSETS 1u   /* offsets not non-decreasing within [0, nbytes] */
#define DNATOK_DERR_CAPACITY 2u  /* PACKED output exceeds ids_capacity (excess not written) */
#define DNATOK_DERR_ROW_WIDTH 4u /* PADDED row longer than pad_to (excess not written) */
#define DNATOK_DERR_INTERNAL 8u  /* a bounded device loop hit its limit (a library fault): output invalid */
#define DNATOK_DERR_IDS 16u      /* dnatok_embed_ids: an id outside the table (its row is written as zeros) */

/* ---- ids and enums --------------------------------------------------------- */
#define DNATOK_ID_PAD 0
#define DNATOK_ID_UNK 1
#define DNATOK_ID_CLS 2
#define DNATOK_ID_SEP 3
#define DNATOK_ID_MASK 4

enum dnatok_kind {
    DNATOK_SINGLE = 0, /* A5 C6 G7 T8 N9 (either case), other bytes UNK; |V| = 10 */
    DNATOK_LUT256 = 1, /* id = lut256[byte]; the user's table defines the id space */
    DNATOK_KMER = 2,   /* non-overlapping k-mers: 5 + radix-4 value, else UNK; |V| = 5 + 4^k */
    DNATOK_BPE = 3     /* ranked merges over ACGT runs: merge r -> id 10 + r; |V| = 10 + R */
};
enum dnatok_layout { DNATOK_PACKED = 0, DNATOK_PADDED = 1 };
enum dnatok_pad_side { DNATOK_PAD_RIGHT = 0, DNATOK_PAD_LEFT = 1 };

typedef struct dnatok_vocab dnatok_vocab;

/*
 * Vocabulary description (host memory, read during dnatok_vocab_create only).
 *  kind      dnatok_kind.
 *  k         KMER frame length, 1..15 (ids fit in int32). Ignored otherwise.
 *  lut256    LUT256: 256 host int32 ids, indexed by byte value (the paper's
 *            ascii_lut[0..255], Design, discovery algorithm). Ids must be >= 0.
 *  pad_id, cls_id, sep_id
 *            LUT256 only: the ids written for pads and specials (the
 *            discovery algorithm's id_pad). Other kinds use 0, 2, 3.
 *  merges    BPE: host int32[n_merges][2], row r = (left id, right id) of the
 *            merge of rank r. Each operand must be a base id 5..8 or 10 + r'
 *            with r' < r, and no pair may repeat (a well-formed table; the
 *            rank-ordered rounds the device runs equal the one-merge-at-a-time
 *            definition only for such tables).
 */
typedef struct dnatok_vocab_desc {
    int32_t kind;
    int32_t k;
    const int32_t *lut256;
    int32_t pad_id;
    int32_t cls_id;
    int32_t sep_id;
    int32_t n_merges;
    const int32_t *merges;
} dnatok_vocab_desc;

/*
 * Encode options.
 *  add_cls_sep  0/1: each row becomes [CLS] body [SEP].
 *  layout       PACKED: rows back to back, row i at d_out_offsets[i].
 *               PADDED: an n x pad_to matrix plus an int8 mask (1 on tokens,
 *               CLS/SEP included; 0 on pads), pads = PAD id.
 *  pad_side     PADDED: RIGHT keeps tokens at the row start; LEFT right-aligns
 *               them (the paper's left padding, EmbedFromStrings algorithm).
 *  pad_to       PADDED row width W (> 0). The paper pads and never truncates,
 *               so W must be at least the longest row (dnatok_encode_plan
 *               returns it).
 *  variant      0, or an OR of DNATOK_VARIANT_* flags (SINGLE, LUT256 and
 *               KMER only; BPE gives EVOCAB):
 *               REVCOMP encodes each row's reverse complement (the row read
 *               back to front with A<->T and C<->G swapped, case kept, N and
 *               other bytes unchanged; the paper's discussion names reverse
 *               complementation as the augmentation to run on the GPU);
 *               OVERLAP (KMER only, else EINVAL) writes stride-1 k-mers, the
 *               overlapping scheme of the paper's introduction: L - k + 1
 *               windows, one UNK for a non-empty row shorter than k.
 *  offset_base  added to every value written to d_out_offsets (lets chunked
 *               callers write one global offsets array).
 */
#define DNATOK_VARIANT_REVCOMP 1
#define DNATOK_VARIANT_OVERLAP 2

typedef struct dnatok_encode_opts {
    int32_t add_cls_sep;
    int32_t layout;
    int32_t pad_side;
    int32_t variant;
    int64_t pad_to;
    int64_t offset_base;
} dnatok_encode_opts;

/* Human-readable description of the calling thread's last failure. */
const char *dnatok_last_error(void);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int32_t dnatok_version(void);

/*
 * Build a vocabulary and upload its device tables to the current device
 * (the paper's static vocabulary built once and copied to GPU memory at
 * initialization, Discussion, "Dynamic Vocabularies and Online BPE"; the
 * 256-entry table that "fits easily in L1 cache or shared memory", bytes
 * path). On success *out owns the tables until dnatok_vocab_destroy.
 * Errors: EINVAL (null), EVOCAB (bad kind/k/table), ENOMEM/EDEVICE.
 */
int dnatok_vocab_create(const dnatok_vocab_desc *desc, dnatok_vocab **out);

/* Free a vocabulary. Work already enqueued with it must have completed. */
int dnatok_vocab_destroy(dnatok_vocab *v);

/*
 * vocab_size: number of ids (max id + 1). max_token_bytes: the most bases one
 * id decodes to (1, k, or the longest merge). Either pointer may be NULL.
 */
int dnatok_vocab_info(const dnatok_vocab *v, int32_t *vocab_size, int32_t *max_token_bytes);

/*
 * Host-side sizing of an encode from host offsets (n + 1 non-decreasing
 * int64). total_tokens: exact PACKED length for SINGLE/LUT256/KMER (L, or
 * ceil(L/k) per row, plus 2 with CLS/SEP), an upper bound (L + specials) for
 * BPE. max_len: the longest row in the same sense — the smallest valid
 * PADDED pad_to (the paper's rule T' = max(token_len, T) is max(pad_to,
 * max_len)). Either output may be NULL. Errors: EINVAL.
 */
int dnatok_encode_plan(const dnatok_vocab *v, const int64_t *h_offsets, int32_t n,
                       const dnatok_encode_opts *opts, int64_t *total_tokens, int64_t *max_len);

/*
 * Encode a ragged batch on the device (bytes path: the LUT, k-mer packing,
 * specials and padding all run in one HIP launch; BPE adds its merge rounds).
 *  d_bytes        device uint8[nbytes], any alignment.
 *  d_offsets      device int64[n + 1]: row i is d_bytes[off[i] .. off[i+1]).
 *                 Must be non-decreasing within [0, nbytes].
 *  d_ids          device int32 output, ids_capacity elements. PACKED: row i
 *                 at [out_off[i], out_off[i+1]). PADDED: n x pad_to.
 *  d_out_offsets  device int64[n + 1], always written: offset_base + the
 *                 PACKED offsets of the true row lengths.
 *  d_mask         device int8[n x pad_to], PADDED only (else NULL).
 * The call is asynchronous on `stream`. Host-checkable errors return at
 * once: EINVAL, ETOOSMALL (PADDED and ids_capacity < n * pad_to), ENOMEM.
 * Violations only the device can see (bad offsets, PACKED overflow, a row
 * longer than pad_to) never write outside the given buffers; they raise a
 * DNATOK_DERR_* flag read by dnatok_sync_status, and d_out_offsets still
 * reports the true sizes. Concurrent calls on different streams are safe;
 * the library keeps one small device workspace per stream.
 */
int dnatok_encode(const dnatok_vocab *v, const uint8_t *d_bytes, int64_t nbytes, const int64_t *d_offsets,
                  int32_t n, int32_t *d_ids, int64_t ids_capacity, int64_t *d_out_offsets, int8_t *d_mask,
                  const dnatok_encode_opts *opts, void *stream);

/*
 * dnatok_encode for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Arguments, outputs and errors are those of dnatok_encode (every kind,
 * layout and variant; the same kernels), but the call allocates nothing:
 * the scan counters, status words and multi-pass scratch the kernels need
 * live in one fixed 32 MiB device array per GPU, part of the library's code
 * object, held from the first call on that GPU until the process ends. A
 * batch whose needs exceed it fails with DNATOK_EBUDGET before anything is
 * enqueued: more than 16,384 scan tiles (about 67 million rows), or, for
 * BPE, more scratch than the array holds (about 4 bytes per input byte plus
 * 48 per row: batches up to about 8 million bases). Every call on a GPU shares that
 * GPU's array: calls that overlap on one GPU (on different streams, or from
 * different threads) race and give wrong results; order them. Device-side
 * error flags of these calls are reported by dnatok_sync_status on any
 * stream of the device. The first call on a GPU also enqueues a small kernel
 * on `stream` that clears the array's counters.
 */
int dnatok_encode_noalloc(const dnatok_vocab *v, const uint8_t *d_bytes, int64_t nbytes, const int64_t *d_offsets,
                          int32_t n, int32_t *d_ids, int64_t ids_capacity, int64_t *d_out_offsets, int8_t *d_mask,
                          const dnatok_encode_opts *opts, void *stream);

/*
 * Encode one ragged batch for several k-mer vocabularies (any k, 1..8 of
 * them) in a single pass over its bytes: each tile is read and classified
 * once and every vocabulary's ids (and mask) are written from it. The
 * paper's throughput experiments sweep token settings over the same input
 * (Results, "Encoding Throughput"); this serves such a batch with one read
 * of the input instead of one per vocabulary. Arrays are host arrays of
 * length n_vocabs: vocabs, d_ids (device pointers), ids_capacity,
 * d_out_offsets (device pointers), d_mask (device pointers; entries may be
 * NULL for PACKED) and opts, which must agree in add_cls_sep, layout and
 * pad_side (pad_to and offset_base may differ). Each vocabulary's outputs
 * are exactly those of dnatok_encode. A single vocabulary of any kind is
 * passed through to dnatok_encode. Errors: as dnatok_encode; EVOCAB for a
 * non-k-mer vocabulary among several.
 */
int dnatok_encode_multi(const dnatok_vocab *const *vocabs, int32_t n_vocabs, const uint8_t *d_bytes, int64_t nbytes,
                        const int64_t *d_offsets, int32_t n, int32_t *const *d_ids, const int64_t *ids_capacity,
                        int64_t *const *d_out_offsets, int8_t *const *d_mask, const dnatok_encode_opts *opts,
                        void *stream);

/*
 * Encode fused with the embedding lookup: the ids dnatok_encode would write
 * (any layout and variant; SINGLE, LUT256 and KMER) are looked up in an
 * embedding table on the device and the table rows are written out, the
 * ids never leaving the kernel (paper: Design, the embedder embed_tokens
 * mapping B x T identifiers to B x T x D activations, called by the
 * EmbedFromStrings algorithm on the device-resident ids).
 *  d_table        device table of n_rows rows of row_bytes bytes each (any
 *                 element type: rows are copied bit for bit), caller-owned.
 *                 n_rows must be at least the vocabulary size (EINVAL).
 *  d_out          device output of out_rows rows of row_bytes: row c is the
 *                 table row of output cell c (PACKED: token c; PADDED: cell
 *                 c of the n x pad_to matrix, pads looking up the pad id).
 *  d_out_offsets  device int64[n + 1], as for dnatok_encode.
 *  d_ids          optional (NULL): also write the ids, as dnatok_encode
 *                 would, with room for out_rows ids.
 *  d_mask         PADDED: optional int8[n x pad_to] mask, as dnatok_encode.
 * row_bytes is 1 .. 2^20; 16-byte aligned table, output and row_bytes take
 * the fastest copy. Asynchronous on `stream`. Errors: EINVAL, ETOOSMALL
 * (PADDED and out_rows < n * pad_to), EVOCAB (BPE: encode first, then
 * dnatok_embed_ids); device-side errors raise DNATOK_DERR_* as for encode.
 */
int dnatok_embed(const dnatok_vocab *v, const uint8_t *d_bytes, int64_t nbytes, const int64_t *d_offsets, int32_t n,
                 const void *d_table, int64_t n_rows, int64_t row_bytes, void *d_out, int64_t out_rows,
                 int64_t *d_out_offsets, int32_t *d_ids, int8_t *d_mask, const dnatok_encode_opts *opts,
                 void *stream);

/*
 * Embedding lookup of given ids (the embedder of the paper's Design section
 * applied to an id tensor, e.g. BPE output): row i of d_out (n_ids rows of
 * row_bytes) is row d_ids[i] of the table. An id outside [0, n_rows) writes
 * a zero row and raises DNATOK_DERR_IDS. Asynchronous. Errors: EINVAL.
 */
int dnatok_embed_ids(const int32_t *d_ids, int64_t n_ids, const void *d_table, int64_t n_rows, int64_t row_bytes,
                     void *d_out, void *stream);

/*
 * Wait for `stream`, then return (and clear) the DNATOK_DERR_* flags the
 * device raised for calls on it since the last check. *flags may be NULL.
 */
int dnatok_sync_status(void *stream, uint32_t *flags);

/*
 * Decode PACKED rows of ids back to bases (the inverse table the paper lists
 * as future work, "Decode Operations"): base, k-mer and merge ids -> their
 * uppercase bases; N -> 'N'; UNK -> 'N' repeated over the width it stands for
 * (k for KMER, 1 otherwise); PAD/CLS/SEP/MASK -> nothing; ids outside the
 * vocabulary decode like UNK. Not defined for LUT256 (EVOCAB): a user table
 * has no canonical inverse.
 *  d_ids          device int32[n_ids].
 *  d_offsets      device int64[n + 1] into d_ids (non-decreasing, <= n_ids).
 *  d_out          device uint8 output, out_capacity bytes; an upper bound is
 *                 n_ids * max_token_bytes.
 *  d_out_offsets  device int64[n + 1] byte offsets of the decoded rows.
 * Asynchronous; overflow and bad offsets raise DNATOK_DERR_* as for encode.
 */
int dnatok_decode(const dnatok_vocab *v, const int32_t *d_ids, int64_t n_ids, const int64_t *d_offsets,
                  int32_t n, uint8_t *d_out, int64_t out_capacity, int64_t *d_out_offsets, void *stream);

/* ---- host-to-device stream ------------------------------------------------------
 *
 * A pinned-memory host-to-device stream overlapped with encode (paper:
 * Design, "Pipelined streaming": separate streams, pre-allocated device
 * buffers, events ordering copies against compute; the paper pipelines
 * 32/64-bit ids, this stream moves raw bytes and encodes on the device, as
 * the bytes path prescribes). Long records (chromosomes) are cut into
 * windows of `window` bases counted from each record's start, the last
 * window of a record being shorter; the output equals dnatok_encode over
 * the ragged batch of all windows in order (PACKED).
 *
 * Pushed chunks land in a ring of `n_slots` device buffers. Each slot has a
 * prefix area in front of its data so the unfinished window at the end of
 * one chunk (at most window - 1 bytes) is copied device-to-device in front
 * of the next chunk and every window stays contiguous. Copies run on a side
 * stream the library owns; encodes run on the caller's compute stream;
 * events order slot reuse, so the host never waits inside the loop.
 * overlap = 0 issues copy and encode on the compute stream in order (the
 * paper's streaming baseline).
 */
typedef struct dnatok_stream dnatok_stream;

typedef struct dnatok_stream_opts {
    int64_t window;       /* bases per window, >= 1 */
    int64_t chunk_bytes;  /* largest push, > 0 */
    int32_t n_slots;      /* device landing buffers, >= 2 (3 = triple buffering) */
    int32_t add_cls_sep;  /* 0/1: [CLS] window [SEP] */
    int32_t overlap;      /* 1: copies overlapped with encode; 0: sequential baseline */
    int32_t reserved;
    int64_t max_tokens;   /* capacity of the library-owned output id buffer */
    int64_t max_windows;  /* capacity of the window offset buffer (max_windows + 1 entries) */
} dnatok_stream_opts;

typedef struct dnatok_stream_result {
    const int32_t *d_ids;            /* device int32[n_tokens], library-owned */
    const int64_t *d_window_offsets; /* device int64[n_windows + 1], library-owned */
    int64_t n_windows;
    int64_t n_tokens;
    int64_t n_bytes;                 /* bytes pushed */
} dnatok_stream_result;

/*
 * Create a stream for vocabulary v (SINGLE, LUT256 or KMER: their token
 * counts are known on the host; BPE -> EVOCAB) whose encodes run on
 * `compute_stream`. Allocates the slots, the output buffers and a copy
 * stream. Errors: EINVAL, EVOCAB, ENOMEM, EDEVICE.
 */
int dnatok_stream_create(const dnatok_vocab *v, const dnatok_stream_opts *opts, void *compute_stream,
                         dnatok_stream **out);

/*
 * Push nbytes (<= chunk_bytes) of pinned host memory (hipHostMalloc or
 * torch pin_memory; pageable memory -> EINVAL). record_ends lists, in
 * non-decreasing order, the positions in [0, nbytes] at which a record ends
 * inside this chunk (n_ends may be 0: the current record continues). The
 * call only enqueues work; h_pinned must stay valid and unchanged until
 * dnatok_stream_flush returns. Capacity (ETOOSMALL) and argument errors are
 * found on the host before anything is enqueued, so a failed push leaves no
 * partial or duplicated windows; after a failure the stream refuses further
 * pushes (ESTATE) until reset.
 */
int dnatok_stream_push(dnatok_stream *s, const uint8_t *h_pinned, int64_t nbytes, const int64_t *record_ends,
                       int32_t n_ends);

/*
 * End the current record (its unfinished window becomes the last window),
 * wait for all work, and describe the output. The stream then refuses
 * pushes (ESTATE) until dnatok_stream_reset.
 */
int dnatok_stream_flush(dnatok_stream *s, dnatok_stream_result *out);

/* Forget all windows and start a new stream, keeping the buffers. */
int dnatok_stream_reset(dnatok_stream *s);

int dnatok_stream_destroy(dnatok_stream *s);

/* ---- IDs path (host mapping, staged id transfer) ------------------------------
 *
 * The paper's other encoding path (Design, "IDs path (CPU staging)"; the
 * host-side branch of the EmbedFromStrings algorithm; "Pipelined
 * streaming"): equal-length strings are mapped to ids on the host through
 * the 256-entry table into persistent pinned staging (int32 or int64),
 * left-padded to token_len, sent to the device one micro-batch at a time,
 * widened to int64 on the device when staged as int32, and handed to the
 * embedder (here the library's embedding lookup). Micro-batches hold
 * b = min(B_emb, max(1, floor(M / T'))) rows for a token budget M. The
 * sequential form copies and computes each micro-batch in order on one
 * stream after mapping every row (the paper's streaming baseline); the
 * pipelined form maps each micro-batch just before its copy, so the host
 * maps micro-batch n + 1 while micro-batch n is copied, and copies
 * micro-batch n + 1 on a side stream into the other of two ping-pong device
 * buffers while micro-batch n is widened and embedded (two int64 buffers
 * with int64 staging; two int32 copy buffers plus two int64 buffers with
 * int32 staging), events ordering the two streams. The bytes path
 * (dnatok_encode, dnatok_stream_*) is this library's main path; this one
 * exists for callers and comparisons that want the paper's host mapping.
 */
typedef struct dnatok_ids dnatok_ids;

typedef struct dnatok_ids_opts {
    int32_t width;        /* bytes per staged id: 4 (int32, widened on the device) or 8 (int64) */
    int32_t overlap;      /* 1: pipelined (ping-pong buffers, copy stream); 0: sequential baseline */
    int32_t threads;      /* host mapping threads, 0 = the host's hardware threads (at most 16) */
    int32_t reserved;
    int64_t token_budget; /* M: ids per micro-batch call (0 = 1,048,576, the paper's default) */
    int64_t max_rows;     /* B_emb: most rows per micro-batch (0 = no cap) */
} dnatok_ids_opts;

typedef struct dnatok_ids_result {
    int64_t rows;            /* B */
    int64_t token_len;       /* T' */
    int64_t micro_rows;      /* b */
    int64_t n_micro;         /* micro-batches */
    int64_t h2d_bytes;       /* staged id bytes copied to the device */
    double map_s;            /* host mapping time (wall clock; pipelined: the sum over micro-batches) */
    double h2d_s;            /* sum of the copies' device times (HIP events on the copying stream) */
    double total_s;          /* the whole call, mapping to the last output written (wall clock) */
} dnatok_ids_result;

/*
 * Create an IDs path for vocabulary v (SINGLE or LUT256: the kinds whose ids
 * are a byte table; others EVOCAB). Its device work runs on compute_stream
 * (the copies of the pipelined form on a side stream it owns). Buffers are
 * sized by the first run and grow when a later run needs more (synchronous,
 * outside the timed loop). Errors: EINVAL, EVOCAB, ENOMEM, EDEVICE.
 */
int dnatok_ids_create(const dnatok_vocab *v, const dnatok_ids_opts *opts, void *compute_stream, dnatok_ids **out);

/*
 * Run the IDs path on n_rows strings of row_len bytes each, back to back in
 * host memory h_bytes (pageable or pinned), left-padded to token_len ids
 * (0 = row_len; must be >= row_len). Outputs (either may be NULL, not both):
 *  d_ids   device int64[n_rows x T'], the ids the embedder received.
 *  d_out   device [n_rows x T'] rows of row_bytes: row c = d_table row of
 *          id c (d_table: n_table_rows rows of row_bytes, any element type).
 * Returns when every output is written (the call synchronizes), with
 * timings in *res (may be NULL). Errors: EINVAL, ENOMEM, EDEVICE; an id
 * outside the table raises DNATOK_DERR_IDS (dnatok_sync_status on the
 * compute stream).
 */
int dnatok_ids_run(dnatok_ids *p, const uint8_t *h_bytes, int64_t n_rows, int64_t row_len, int64_t token_len,
                   int64_t *d_ids, const void *d_table, int64_t n_table_rows, int64_t row_bytes, void *d_out,
                   dnatok_ids_result *res);

int dnatok_ids_destroy(dnatok_ids *p);

/*
 * The host mapping step alone (host memory only, no device involved): rows
 * of row_len bytes -> ids through lut256 (256 int32), left-padded with
 * pad_id to token_len, written as int32 (width 4) or int64 (width 8) to
 * h_out[n_rows x token_len], on `threads` threads (0 = hardware threads, at
 * most 16). Errors: EINVAL.
 */
int dnatok_ids_map(const int32_t *lut256, int32_t pad_id, const uint8_t *h_bytes, int64_t n_rows, int64_t row_len,
                   int64_t token_len, int32_t width, void *h_out, int32_t threads);

/* ---- tuning, autotuner and captured graphs ----------------------------------
 *
 * The paper attributes much of the remaining cost of batched encoding to
 * launch overhead and memory layout (Discussion, "Performance
 * Characteristics and Scaling Behavior"). These calls pick the tiling of a
 * vocabulary's kernels by measurement and replay a fixed encode without
 * per-launch host work. Tuning changes scheduling only: ids are the same for
 * every setting.
 */
typedef struct dnatok_tuning {
    int32_t tile_bytes;     /* SINGLE/LUT256/KMER: input bytes per tile, power of two 4096..65536 (0 = default) */
    int32_t blocks_per_cu;  /* SINGLE/LUT256/KMER: workgroups per CU, 0 = as many as fit */
    int32_t bpe_item_bytes; /* BPE: nominal item length S, power of two 1024..65536 (0 = 8192) */
    int32_t bpe_max_waves;  /* BPE: most waves per workgroup of the length classes: 1, 2, 4 or 8 (0 = 8) */
    int32_t spread;         /* SINGLE/LUT256/KMER: 0 = every workgroup walks a static share of the tiles;
                               1..100 = one tile per workgroup: the first resident round by workgroup
                               index, the rest from a ticket counter, with this percentage of the tiles
                               as extra workgroups, so the parts of the chip that finish early take more */
    int32_t bands;          /* SINGLE/LUT256/KMER, PADDED layout: 0 = default, 1 = row bands (a workgroup
                               stages the bytes of a few whole rows, or of a part of a longer row, at most
                               tile_bytes, and writes all their cells), 2 = tiles, 3 = row bands taken by
                               resident workgroups in turn, the next band's bytes fetched while the current
                               one is written (a band staging more than 16 KiB less 64 bytes runs as 1) */
} dnatok_tuning;

int dnatok_get_tuning(const dnatok_vocab *v, dnatok_tuning *out);

/* Set (EINVAL for out-of-range fields); applies to calls made afterwards. */
int dnatok_set_tuning(dnatok_vocab *v, const dnatok_tuning *t);

/*
 * Time every candidate tiling of v on this batch (the arguments of
 * dnatok_encode; the outputs are overwritten) with HIP events on `stream`:
 * one warm-up and `reps` timed samples each, a sample being 4 back-to-back
 * launches (median of the time per launch); the three fastest again, 3 *
 * reps samples each, interleaved. The fastest setting is stored in v and
 * returned in *best / *best_ms (ms per launch). Synchronizes `stream`;
 * not allowed during graph capture (ESTATE). Errors as dnatok_encode.
 */
int dnatok_autotune(dnatok_vocab *v, const uint8_t *d_bytes, int64_t nbytes, const int64_t *d_offsets, int32_t n,
                    int32_t *d_ids, int64_t ids_capacity, int64_t *d_out_offsets, int8_t *d_mask,
                    const dnatok_encode_opts *opts, void *stream, int32_t reps, dnatok_tuning *best,
                    float *best_ms);

/* The autotuner for dnatok_encode_multi: the tiling is that of vocabs[0],
 * which the multi-vocabulary pass uses; the fastest setting is stored there. */
int dnatok_autotune_multi(dnatok_vocab *const *vocabs, int32_t n_vocabs, const uint8_t *d_bytes, int64_t nbytes,
                          const int64_t *d_offsets, int32_t n, int32_t *const *d_ids, const int64_t *ids_capacity,
                          int64_t *const *d_out_offsets, int8_t *const *d_mask, const dnatok_encode_opts *opts,
                          void *stream, int32_t reps, dnatok_tuning *best, float *best_ms);

typedef struct dnatok_graph dnatok_graph;

/* The arguments of one dnatok_encode (minus the stream). */
typedef struct dnatok_encode_call {
    const dnatok_vocab *v;
    const uint8_t *d_bytes;
    int64_t nbytes;
    const int64_t *d_offsets;
    int32_t n;
    int32_t reserved;
    int32_t *d_ids;
    int64_t ids_capacity;
    int64_t *d_out_offsets;
    int8_t *d_mask;
    dnatok_encode_opts opts;
} dnatok_encode_call;

/*
 * Capture n_calls encodes, in order, with exactly these buffers, sizes and
 * options into one executable HIP graph (each encode is run once eagerly
 * first, which also sizes the graph's private workspace). Each
 * dnatok_graph_launch replays them all on `stream`, reading whatever the
 * buffers hold at that point; replays of one graph must not overlap (order
 * them on one stream or with events). Vocabularies and buffers must outlive
 * the graph. Errors: as dnatok_encode for any call, EDEVICE.
 */
int dnatok_graph_create(const dnatok_encode_call *calls, int32_t n_calls, dnatok_graph **out);
int dnatok_graph_launch(dnatok_graph *g, void *stream);
int dnatok_graph_destroy(dnatok_graph *g);

/* ---- serving loop -----------------------------------------------------------
 *
 * Online tokenization (Discussion, "When Does DNATok Matter?": the serving
 * use case, where tokenization sits on the latency path of every request,
 * and the latency-bound real-model scenario of the Results). A server owns a
 * worker thread, a device memory arena of budget_bytes and n_streams HIP
 * streams. Requests (one sequence each, any of the server's vocabularies,
 * host bytes) are admitted in arrival order while the arena has room for
 * their input and output; admitted requests that share the vocabulary and
 * the specials flag of the oldest waiting request are encoded together as
 * one ragged batch (one dnatok_encode) on a free stream, so requests that
 * arrive while others run join the next batch and batches on different
 * streams overlap on the device (continuous batching). Vocabulary tables stay
 * resident; results stay in the arena until released. A request's ids are
 * exactly those of dnatok_encode on that sequence alone.
 */
typedef struct dnatok_server dnatok_server;

typedef struct dnatok_server_opts {
    int64_t budget_bytes;     /* device bytes for requests: inputs, outputs, offsets and BPE scratch */
    int32_t n_streams;        /* batches in flight at once, 1..16 */
    int32_t max_batch;        /* most requests in one batch, >= 1 */
    int64_t max_batch_bytes;  /* most input bytes in one batch, and in one request (a larger request: EBUDGET) */
    int64_t staging_bytes;    /* pinned host staging per stream for pageable inputs, >= max_batch_bytes */
} dnatok_server_opts;

typedef struct dnatok_request_result {
    const int32_t *d_ids; /* device int32[n_tokens] in the server's arena, valid until release */
    int64_t n_tokens;
    int32_t status;       /* DNATOK_OK, or the error that failed the request */
    uint32_t dev_flags;   /* device error flags of the request's batch (dnatok_sync_status bits) */
    double t_submit;      /* seconds on the server clock (dnatok_server_now) */
    double t_start;       /* its batch was enqueued on a stream */
    double t_done;        /* the worker saw its batch complete */
} dnatok_request_result;

/* Errors: EINVAL (bad options), ENOMEM (arena, pinned staging), EDEVICE. */
int dnatok_server_create(const dnatok_server_opts *opts, dnatok_server **out);

/*
 * Queue one request. h_bytes may be pinned or pageable host memory and is
 * copied before the call returns when pageable; pinned memory is read by the
 * device later and must stay unchanged until the request is done. The
 * vocabulary must outlive the request. Errors: EINVAL, EBUDGET (the request
 * is longer than max_batch_bytes, whose size the per-stream scratch is
 * reserved for, or its input and output alone exceed the arena), ESTATE
 * (server shutting down). A rejected request leaves nothing queued.
 */
int dnatok_server_submit(dnatok_server *s, const dnatok_vocab *v, const uint8_t *h_bytes, int64_t nbytes,
                         int32_t add_cls_sep, uint64_t *ticket);

/* Non-blocking: 0 and *out filled when the request is done, 1 while it is pending, < 0 on error. */
int dnatok_server_poll(dnatok_server *s, uint64_t ticket, dnatok_request_result *out);

/* Block until the request is done; fills *out. EINVAL for an unknown ticket. */
int dnatok_server_wait(dnatok_server *s, uint64_t ticket, dnatok_request_result *out);

/* Return a done request's output memory to the arena (its d_ids become invalid). */
int dnatok_server_release(dnatok_server *s, uint64_t ticket);

/* Server clock (seconds, monotonic) used by the result timestamps. */
double dnatok_server_now(const dnatok_server *s);

/* Counters: requests done, batches launched, peak arena bytes in use. */
int dnatok_server_stats(const dnatok_server *s, int64_t *requests, int64_t *batches, int64_t *peak_bytes);

/* Finish queued work, stop the worker, free everything (outstanding results too). */
int dnatok_server_destroy(dnatok_server *s);

#ifdef __cplusplus
}
#endif

#endif /* DNATOK_H */
