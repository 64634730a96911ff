/*
 * CPU ORACLE for the DNA byte->identifier tokenizer.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this file's library. It shares no
 * code, header, table or constant generator with the GPU library: every rule
 * below is written out here from the paper, in plain loops, for a reader to
 * check by eye.
 *
 * What is computed (paper: Design, "Encoding paths" and the bytes path of the
 * EmbedFromStrings algorithm; vocabulary kinds from the introduction and the
 * table of genomic tokenization schemes):
 *
 *   Id space (the paper leaves special ids to the upstream vocabulary; the
 *   reading used here): PAD=0 (the paper's default pad id is 0, discovery
 *   algorithm), UNK=1, CLS=2, SEP=3, MASK=4.
 *
 *   SINGLE (single-nucleotide): A=5 C=6 G=7 T=8 N=9, lowercase folded to
 *   uppercase (the discovery algorithm maps A/a, C/c, G/g, T/t, N/n to one
 *   id each); every other byte -> UNK.
 *
 *   LUT256: id = table[byte], the user's 256-entry ASCII->identifier table
 *   (the bytes path applies ascii_lut[Bytes] directly). The discovery
 *   algorithm's fixed-DNA fallback table is one such table.
 *
 *   KMER(k) (non-overlapping k-mers): frames start at the first base of the
 *   sequence and advance by k. A full frame of ACGT (either case) gets
 *   id = 5 + sum_j d(b_j) * 4^(k-1-j), d(A)=0 d(C)=1 d(G)=2 d(T)=3, the first
 *   base most significant. A frame holding N or any other byte, and a short
 *   final frame (L mod k != 0), gets UNK. A sequence of L bases gives
 *   ceil(L/k) tokens.
 *
 *   BPE (ranked merges, the BPE of Sennrich et al. that the introduction
 *   cites): bases A..T are 5..8, N is 9, other bytes UNK. Merges never cross
 *   an N or an invalid byte: each maximal ACGT run is segmented on its own.
 *   Within a run, repeat: take the adjacent pair with the lowest merge rank;
 *   stop if no adjacent pair has a rank; otherwise replace every
 *   non-overlapping occurrence of that pair, scanning left to right, by the
 *   merge's id 10 + rank.
 *
 *   Specials: with CLS/SEP on, a row is [CLS] body [SEP].
 *
 *   Layouts: PACKED writes rows back to back with int64 offsets
 *   (out_offsets[0] = 0, out_offsets[i+1] = out_offsets[i] + len_i).
 *   PADDED writes an n x W matrix; W must be at least every row's length
 *   (the paper pads and never truncates); RIGHT keeps tokens at the start of
 *   the row, LEFT right-aligns them (the paper's left padding); the int8 mask
 *   is 1 on tokens (CLS/SEP included) and 0 on pads.
 *
 *   Reverse complement (the augmentation the paper's discussion of data
 *   augmentation names as the natural one to run on the GPU): each row is
 *   read back to front with A<->T and C<->G swapped (case kept); N, n and
 *   every other byte stay as they are. An encode of the reverse complement
 *   is the encode of that row.
 *
 *   Overlapping k-mers (stride 1, the older scheme the introduction
 *   describes): a window starts at every base s with s + k <= L, giving
 *   L - k + 1 tokens, each with the k-mer id rule above (UNK if the window
 *   holds a byte other than ACGT in either case). A non-empty row shorter
 *   than k gives one UNK, as a short final frame does for non-overlapping
 *   k-mers; an empty row gives none.
 *
 *   Decode (the inverse table the paper lists as future work): base, k-mer
 *   and merge ids -> their uppercase bases (merges expanded recursively);
 *   N -> "N"; UNK -> "N" repeated over the width it stands for (k for KMER,
 *   1 otherwise); PAD/CLS/SEP/MASK -> nothing; any id outside the
 *   vocabulary decodes like UNK.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { PAD = 0, UNK = 1, CLS = 2, SEP = 3, MASK = 4 };
enum { KIND_SINGLE = 0, KIND_LUT256 = 1, KIND_KMER = 2, KIND_BPE = 3 };
enum { LAYOUT_PACKED = 0, LAYOUT_PADDED = 1 };
enum { SIDE_RIGHT = 0, SIDE_LEFT = 1 };

/* ---- byte rules ------------------------------------------------------- */

/* Base digit of an A/C/G/T byte in either case, or -1. */
static int base_digit(uint8_t b) {
    switch (b) {
    case 'A': case 'a': return 0;
    case 'C': case 'c': return 1;
    case 'G': case 'g': return 2;
    case 'T': case 't': return 3;
    default: return -1;
    }
}

static int is_n(uint8_t b) { return b == 'N' || b == 'n'; }

static int32_t single_id(uint8_t b) {
    int d = base_digit(b);
    if (d >= 0) return 5 + d;
    if (is_n(b)) return 9;
    return UNK;
}

/* ---- BPE merge lookup (sorted (left, right) -> rank, bsearch) ------------ */

typedef struct { int32_t left, right, rank; } merge_entry;

static int cmp_pair(const void *x, const void *y) {
    const merge_entry *a = (const merge_entry *)x, *b = (const merge_entry *)y;
    if (a->left != b->left) return a->left < b->left ? -1 : 1;
    if (a->right != b->right) return a->right < b->right ? -1 : 1;
    return 0;
}

typedef struct { merge_entry *sorted; int32_t n; const int32_t *merges; } rank_table;

static rank_table make_rank_table(const int32_t *merges, int32_t n_merges) {
    rank_table t;
    t.n = n_merges;
    t.merges = merges;
    t.sorted = (merge_entry *)malloc(sizeof(merge_entry) * (size_t)(n_merges > 0 ? n_merges : 1));
    for (int32_t r = 0; r < n_merges; ++r) {
        t.sorted[r].left = merges[2 * r];
        t.sorted[r].right = merges[2 * r + 1];
        t.sorted[r].rank = r;
    }
    qsort(t.sorted, (size_t)n_merges, sizeof(merge_entry), cmp_pair);
    return t;
}

/* Rank of the pair (a, b), or -1 if it is not a merge. */
static int32_t pair_rank(const rank_table *t, int32_t a, int32_t b) {
    merge_entry key = {a, b, 0};
    const merge_entry *hit = (const merge_entry *)bsearch(&key, t->sorted, (size_t)t->n, sizeof(merge_entry), cmp_pair);
    return hit ? hit->rank : -1;
}

/* Segment one ACGT run (symbols in sym[0..m)) in place; returns the new length. */
static int64_t bpe_run(const rank_table *t, int32_t *sym, int64_t m) {
    for (;;) {
        int32_t best = -1;
        for (int64_t p = 0; p + 1 < m; ++p) {
            int32_t r = pair_rank(t, sym[p], sym[p + 1]);
            if (r >= 0 && (best < 0 || r < best)) best = r;
        }
        if (best < 0) return m;
        int32_t left = t->merges[2 * best], right = t->merges[2 * best + 1];
        int64_t w = 0, p = 0;
        while (p < m) {
            if (p + 1 < m && sym[p] == left && sym[p + 1] == right) {
                sym[w++] = 10 + best;
                p += 2;
            } else {
                sym[w++] = sym[p++];
            }
        }
        m = w;
    }
}

/* ---- one row -------------------------------------------------------------- */

/* Body tokens of one row written to out (capacity >= L); returns the count. */
static int64_t encode_body(int kind, int k, const int32_t *lut, const rank_table *rt,
                           const uint8_t *row, int64_t L, int32_t *out) {
    int64_t c = 0;
    if (kind == KIND_SINGLE) {
        for (int64_t i = 0; i < L; ++i) out[c++] = single_id(row[i]);
    } else if (kind == KIND_LUT256) {
        for (int64_t i = 0; i < L; ++i) out[c++] = lut[row[i]];
    } else if (kind == KIND_KMER) {
        for (int64_t start = 0; start < L; start += k) {
            if (start + k > L) { out[c++] = UNK; continue; } /* short final frame */
            int32_t id = 0;
            int ok = 1;
            for (int j = 0; j < k; ++j) {
                int d = base_digit(row[start + j]);
                if (d < 0) { ok = 0; break; }
                id = id * 4 + d;
            }
            out[c++] = ok ? 5 + id : UNK;
        }
    } else { /* KIND_BPE */
        int64_t i = 0;
        while (i < L) {
            int d = base_digit(row[i]);
            if (d < 0) { out[c++] = is_n(row[i]) ? 9 : UNK; ++i; continue; }
            int64_t m = 0;
            while (i < L && base_digit(row[i]) >= 0) { out[c + m] = 5 + base_digit(row[i]); ++m; ++i; }
            c += bpe_run(rt, out + c, m);
        }
    }
    return c;
}

/*
 * PACKED encode of a ragged batch: row i is bytes[offsets[i] .. offsets[i+1]).
 * Writes out_ids (capacity ids_cap) and out_offsets[0..n]. Returns the total
 * token count, -1 if ids_cap is too small, -2 on bad arguments.
 */
int64_t oracle_encode(int kind, int k, const int32_t *lut, int32_t cls_id, int32_t sep_id,
                      const int32_t *merges, int32_t n_merges,
                      const uint8_t *bytes, const int64_t *offsets, int32_t n, int add_cls_sep,
                      int32_t *out_ids, int64_t ids_cap, int64_t *out_offsets) {
    if (kind == KIND_KMER && (k < 1 || k > 15)) return -2;
    if (kind == KIND_LUT256 && !lut) return -2;
    rank_table rt = {0, 0, 0};
    if (kind == KIND_BPE) rt = make_rank_table(merges, n_merges);
    if (kind != KIND_LUT256) { cls_id = CLS; sep_id = SEP; }
    int64_t total = 0;
    int64_t maxL = 0;
    for (int32_t i = 0; i < n; ++i)
        if (offsets[i + 1] - offsets[i] > maxL) maxL = offsets[i + 1] - offsets[i];
    int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(maxL > 0 ? maxL : 1));
    int64_t status = 0;
    out_offsets[0] = 0;
    for (int32_t i = 0; i < n; ++i) {
        int64_t L = offsets[i + 1] - offsets[i];
        if (L < 0) { status = -2; break; }
        int64_t nb = encode_body(kind, k, lut, &rt, bytes + offsets[i], L, tmp);
        int64_t len = nb + (add_cls_sep ? 2 : 0);
        if (total + len > ids_cap) { status = -1; break; }
        int64_t w = total;
        if (add_cls_sep) out_ids[w++] = cls_id;
        for (int64_t j = 0; j < nb; ++j) out_ids[w++] = tmp[j];
        if (add_cls_sep) out_ids[w++] = sep_id;
        total += len;
        out_offsets[i + 1] = total;
    }
    free(tmp);
    free(rt.sorted);
    return status < 0 ? status : total;
}

/*
 * Reverse complement of every row: out[offsets[i] + t] is the complement of
 * bytes[offsets[i + 1] - 1 - t]. Returns 0, or -2 on decreasing offsets.
 */
int oracle_revcomp(const uint8_t *bytes, const int64_t *offsets, int32_t n, uint8_t *out) {
    for (int32_t i = 0; i < n; ++i) {
        int64_t lo = offsets[i], hi = offsets[i + 1];
        if (hi < lo) return -2;
        for (int64_t t = 0; t < hi - lo; ++t) {
            uint8_t b = bytes[hi - 1 - t];
            uint8_t c = b;
            switch (b) {
            case 'A': c = 'T'; break;
            case 'T': c = 'A'; break;
            case 'C': c = 'G'; break;
            case 'G': c = 'C'; break;
            case 'a': c = 't'; break;
            case 't': c = 'a'; break;
            case 'c': c = 'g'; break;
            case 'g': c = 'c'; break;
            default: break;
            }
            out[lo + t] = c;
        }
    }
    return 0;
}

/*
 * PACKED encode with overlapping k-mers (stride 1). Same contract as
 * oracle_encode for the KMER kind.
 */
int64_t oracle_encode_overlap(int k, const uint8_t *bytes, const int64_t *offsets, int32_t n, int add_cls_sep,
                              int32_t *out_ids, int64_t ids_cap, int64_t *out_offsets) {
    if (k < 1 || k > 15) return -2;
    int64_t total = 0;
    out_offsets[0] = 0;
    for (int32_t i = 0; i < n; ++i) {
        const uint8_t *row = bytes + offsets[i];
        int64_t L = offsets[i + 1] - offsets[i];
        if (L < 0) return -2;
        int64_t nb = (L >= k) ? L - k + 1 : (L > 0 ? 1 : 0);
        int64_t len = nb + (add_cls_sep ? 2 : 0);
        if (total + len > ids_cap) return -1;
        int64_t w = total;
        if (add_cls_sep) out_ids[w++] = CLS;
        if (L > 0 && L < k) {
            out_ids[w++] = UNK;
        } else {
            for (int64_t s = 0; s + k <= L; ++s) {
                int32_t id = 0;
                int ok = 1;
                for (int j = 0; j < k; ++j) {
                    int d = base_digit(row[s + j]);
                    if (d < 0) { ok = 0; break; }
                    id = id * 4 + d;
                }
                out_ids[w++] = ok ? 5 + id : UNK;
            }
        }
        if (add_cls_sep) out_ids[w++] = SEP;
        total += len;
        out_offsets[i + 1] = total;
    }
    return total;
}

/*
 * PACKED -> PADDED (n x W ids, n x W mask). Returns 0, or -1 if some row is
 * longer than W (the paper pads and never truncates).
 */
int oracle_pad(const int32_t *ids, const int64_t *offsets, int32_t n, int64_t W, int side, int32_t pad_id,
               int32_t *out_ids, int8_t *out_mask) {
    for (int32_t i = 0; i < n; ++i) {
        int64_t len = offsets[i + 1] - offsets[i];
        if (len > W) return -1;
        int64_t lead = (side == SIDE_LEFT) ? W - len : 0;
        for (int64_t c = 0; c < W; ++c) {
            int64_t t = c - lead;
            int is_tok = (t >= 0 && t < len);
            out_ids[(int64_t)i * W + c] = is_tok ? ids[offsets[i] + t] : pad_id;
            out_mask[(int64_t)i * W + c] = (int8_t)(is_tok ? 1 : 0);
        }
    }
    return 0;
}

/* ---- decode ---------------------------------------------------------------- */

/* Uppercase expansion of one id into out (capacity cap); returns the byte count. */
static int64_t expand(int kind, int k, const int32_t *merges, int32_t n_merges, int32_t id, uint8_t *out, int64_t cap) {
    static const uint8_t B[4] = {'A', 'C', 'G', 'T'};
    int32_t vocab = (kind == KIND_SINGLE) ? 10
                  : (kind == KIND_KMER) ? 5 + (int32_t)(1u << (2 * k))
                  : 10 + n_merges;
    if (id == PAD || id == CLS || id == SEP || id == MASK) return 0;
    int width = (kind == KIND_KMER) ? k : 1;
    if (id == UNK || id < 0 || id >= vocab) {
        for (int j = 0; j < width && j < cap; ++j) out[j] = 'N';
        return width;
    }
    if (kind == KIND_KMER) {
        int32_t v = id - 5;
        for (int j = k - 1; j >= 0; --j) { if (j < cap) out[j] = B[v & 3]; v >>= 2; }
        return k;
    }
    if (id <= 8) { if (cap > 0) out[0] = B[id - 5]; return 1; }
    if (id == 9) { if (cap > 0) out[0] = 'N'; return 1; }
    /* merge id: left expansion then right expansion */
    int32_t r = id - 10;
    int64_t a = expand(kind, k, merges, n_merges, merges[2 * r], out, cap);
    int64_t b = expand(kind, k, merges, n_merges, merges[2 * r + 1], out + (a < cap ? a : cap), cap > a ? cap - a : 0);
    return a + b;
}

/*
 * Decode PACKED rows ids[offsets[i] .. offsets[i+1]) into bytes. Returns the
 * total byte count, -1 if out_cap is too small, -2 on an unsupported kind.
 */
int64_t oracle_decode(int kind, int k, const int32_t *merges, int32_t n_merges,
                      const int32_t *ids, const int64_t *offsets, int32_t n,
                      uint8_t *out, int64_t out_cap, int64_t *out_offsets) {
    if (kind == KIND_LUT256) return -2;
    int64_t total = 0;
    out_offsets[0] = 0;
    uint8_t buf[1 << 16];
    for (int32_t i = 0; i < n; ++i) {
        for (int64_t t = offsets[i]; t < offsets[i + 1]; ++t) {
            int64_t w = expand(kind, k, merges, n_merges, ids[t], buf, (int64_t)sizeof(buf));
            if (w > (int64_t)sizeof(buf)) return -2;
            if (total + w > out_cap) return -1;
            memcpy(out + total, buf, (size_t)w);
            total += w;
        }
        out_offsets[i + 1] = total;
    }
    return total;
}

/*
 * Well-formedness of a ranked merge table: every operand is a base id (5..8)
 * or the id 10 + r' of an earlier merge r' < r, and no pair appears twice.
 * Returns 0 if well formed, else 1 + the first offending rank.
 */
int32_t oracle_bpe_check(const int32_t *merges, int32_t n_merges) {
    for (int32_t r = 0; r < n_merges; ++r) {
        for (int s = 0; s < 2; ++s) {
            int32_t x = merges[2 * r + s];
            int ok = (x >= 5 && x <= 8) || (x >= 10 && x < 10 + r);
            if (!ok) return 1 + r;
        }
        for (int32_t q = 0; q < r; ++q)
            if (merges[2 * q] == merges[2 * r] && merges[2 * q + 1] == merges[2 * r + 1]) return 1 + r;
    }
    return 0;
}
