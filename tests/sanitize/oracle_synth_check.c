/*
 * Host-only driver for the sanitizer test: runs every entry point of the C
 * oracle and of the seeded generators on small inputs, edge cases included,
 * with output buffers allocated at exactly the size each call needs, so an
 * AddressSanitizer / UndefinedBehaviorSanitizer build reports any read or
 * write outside them and any undefined arithmetic. Prints "ok" and exits 0
 * when every call returned what it should.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int64_t oracle_encode(int kind, int k, const int32_t *lut, int32_t cls_id, int32_t sep_id, const int32_t *merges,
                      int32_t n_merges, const uint8_t *bytes, const int64_t *offsets, int32_t n, int add_cls_sep,
                      int32_t *out_ids, int64_t ids_cap, int64_t *out_offsets);
int oracle_revcomp(const uint8_t *bytes, const int64_t *offsets, int32_t n, uint8_t *out);
int64_t oracle_encode_overlap(int k, const uint8_t *bytes, const int64_t *offsets, int32_t n, int add_cls_sep,
                              int32_t *out_ids, int64_t ids_cap, int64_t *out_offsets);
int oracle_pad(const int32_t *ids, const int64_t *offsets, int32_t n, int64_t W, int side, int32_t pad_id,
               int32_t *out_ids, int8_t *out_mask);
int64_t oracle_decode(int kind, int k, const int32_t *merges, int32_t n_merges, const int32_t *ids,
                      const int64_t *offsets, int32_t n, uint8_t *out, int64_t out_cap, int64_t *out_offsets);
int32_t oracle_bpe_check(const int32_t *merges, int32_t n_merges);
int32_t oracle_bpe_train(const uint8_t *corpus, int64_t n, int32_t R, int32_t *out_merges);

uint64_t synth_substream(uint64_t base_seed, uint64_t a, uint64_t b);
void synth_iid(uint64_t seed, uint8_t *out, int64_t n, double p_n);
void synth_markov(uint64_t table_seed, uint64_t seq_seed, int order, uint8_t *out, int64_t n, double *cum_scratch);
void synth_softmask(uint64_t seed, uint8_t *buf, int64_t n, double mu_mask, double mu_open);
void synth_nruns(uint64_t seed, uint8_t *buf, int64_t n, double mu_run, double mu_gap);
void synth_invalid(uint64_t seed, uint8_t *buf, int64_t n, double p);
void synth_bytes(uint64_t seed, uint8_t *out, int64_t n);
void synth_raw(uint64_t seed, uint64_t *out, int64_t n);

static int failures = 0;
#define CHECK(c)                                                            \
    do {                                                                    \
        if (!(c)) {                                                         \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++failures;                                                     \
        }                                                                   \
    } while (0)

static void *xmalloc(size_t n) {
    void *p = malloc(n ? n : 1);
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    return p;
}

/* Tokens of a row of L bytes: L, ceil(L/k) or the overlapping count, + specials. */
static int64_t row_tokens(int kind, int k, int overlap, int64_t L, int cls) {
    int64_t body = L;
    if (kind == 2) body = overlap ? (L >= k ? L - k + 1 : (L > 0 ? 1 : 0)) : (L + k - 1) / k;
    return body + 2 * cls;
}

int main(void) {
    /* generators: every entry point, small sizes, order 0 and 5 */
    enum { N = 20000 };
    uint8_t *g = (uint8_t *)xmalloc(N);
    double *scratch = (double *)xmalloc(sizeof(double) * 4 * 1024);
    synth_markov(synth_substream(42, 1, 2), 7, 5, g, N, scratch);
    synth_markov(3, 4, 0, g, 10, scratch);
    synth_markov(3, 4, 3, g, 2, scratch); /* shorter than the order */
    synth_markov(synth_substream(42, 1, 2), 9, 3, g, N, scratch);
    synth_softmask(11, g, N, 300.0, 450.0);
    synth_nruns(12, g, N, 50.0, 2450.0);
    synth_invalid(13, g, N, 1e-2);
    uint8_t *iid = (uint8_t *)xmalloc(4096);
    synth_iid(14, iid, 4096, 0.05);
    uint8_t *anyb = (uint8_t *)xmalloc(300);
    synth_bytes(15, anyb, 300);
    uint64_t raw[17];
    synth_raw(16, raw, 17);

    /* a ragged batch over the decorated genome: empty rows, one byte, long rows */
    const int64_t lens[] = {0, 1, 2, 5, 6, 7, 0, 15, 16, 17, 31, 32, 33, 100, 997, 4096, 0, 1, 13000};
    const int32_t n = (int32_t)(sizeof(lens) / sizeof(lens[0]));
    int64_t *offs = (int64_t *)xmalloc(sizeof(int64_t) * (n + 1));
    offs[0] = 0;
    for (int32_t i = 0; i < n; ++i) offs[i + 1] = offs[i] + lens[i];
    CHECK(offs[n] <= N);

    int32_t lut[256];
    for (int b = 0; b < 256; ++b) lut[b] = b % 7;

    /* a trained table for BPE (from an uppercase corpus) */
    uint8_t *corpus = (uint8_t *)xmalloc(N);
    synth_markov(21, 22, 3, corpus, N, scratch);
    int32_t *merges = (int32_t *)xmalloc(sizeof(int32_t) * 2 * 200);
    const int32_t R = oracle_bpe_train(corpus, N, 200, merges);
    CHECK(R > 0 && R <= 200);
    CHECK(oracle_bpe_check(merges, R) == 0);
    int32_t bad[4] = {5, 5, 5, 5}; /* a repeated pair */
    CHECK(oracle_bpe_check(bad, 2) != 0);
    CHECK(oracle_bpe_train(corpus, 1, 10, merges + 2 * R) == 0); /* one-byte corpus: no pair to merge */
    CHECK(oracle_bpe_train(corpus, 0, 10, merges + 2 * R) >= 0);

    for (int kind = 0; kind <= 3; ++kind) {
        const int kmax = (kind == 2) ? 15 : 1;
        for (int k = 1; k <= kmax; ++k) {
            for (int cls = 0; cls <= 1; ++cls) {
                int64_t total = 0, width = 1;
                for (int32_t i = 0; i < n; ++i) {
                    const int64_t t = (kind == 3) ? lens[i] + 2 * cls : row_tokens(kind, k, 0, lens[i], cls);
                    total += t;
                    if (t > width) width = t;
                }
                int32_t *ids = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)total);
                int64_t *oo = (int64_t *)xmalloc(sizeof(int64_t) * (n + 1));
                const int64_t got = oracle_encode(kind, k, lut, 2, 3, merges, R, g, offs, n, cls, ids, total, oo);
                CHECK(got >= 0 && got <= total && oo[n] == got);
                if (kind != 3) CHECK(got == total);
                if (got > 0) {
                    /* too small an output is refused, not overrun */
                    CHECK(oracle_encode(kind, k, lut, 2, 3, merges, R, g, offs, n, cls, ids, got - 1, oo) < 0);
                }
                const int64_t W = width + 3;
                int32_t *pid = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)(n * W));
                int8_t *pm = (int8_t *)xmalloc((size_t)(n * W));
                for (int side = 0; side <= 1; ++side) CHECK(oracle_pad(ids, oo, n, W, side, 0, pid, pm) == 0);
                free(pid);
                free(pm);
                if (kind != 1 && got >= 0) {
                    int64_t widest = (kind == 2) ? k : 1;
                    if (kind == 3) widest = 64; /* a 200-merge table's tokens are short */
                    const int64_t cap = got * widest;
                    uint8_t *dec = (uint8_t *)xmalloc((size_t)cap);
                    int64_t *doo = (int64_t *)xmalloc(sizeof(int64_t) * (n + 1));
                    const int64_t dl = oracle_decode(kind, k, merges, R, ids, oo, n, dec, cap, doo);
                    CHECK(dl >= 0 && dl <= cap);
                    free(dec);
                    free(doo);
                }
                free(ids);
                free(oo);
            }
        }
    }
    /* overlapping windows, every k */
    for (int k = 1; k <= 15; ++k) {
        for (int cls = 0; cls <= 1; ++cls) {
            int64_t total = 0;
            for (int32_t i = 0; i < n; ++i) total += row_tokens(2, k, 1, lens[i], cls);
            int32_t *ids = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)total);
            int64_t *oo = (int64_t *)xmalloc(sizeof(int64_t) * (n + 1));
            CHECK(oracle_encode_overlap(k, g, offs, n, cls, ids, total, oo) == total);
            free(ids);
            free(oo);
        }
    }
    /* reverse complement of every row */
    uint8_t *rc = (uint8_t *)xmalloc((size_t)offs[n]);
    CHECK(oracle_revcomp(g, offs, n, rc) == 0);
    uint8_t *rc2 = (uint8_t *)xmalloc((size_t)offs[n]);
    CHECK(oracle_revcomp(rc, offs, n, rc2) == 0);
    CHECK(memcmp(rc2, g, (size_t)offs[n]) == 0);
    /* all 256 byte values through every kind */
    uint8_t all[256];
    for (int b = 0; b < 256; ++b) all[b] = (uint8_t)b;
    int64_t o2[2] = {0, 256};
    int32_t ids256[258];
    int64_t oo2[2];
    for (int kind = 0; kind <= 3; ++kind)
        CHECK(oracle_encode(kind, 3, lut, 2, 3, merges, R, all, o2, 1, 1, ids256, 258, oo2) >= 0);

    free(rc);
    free(rc2);
    free(g);
    free(scratch);
    free(iid);
    free(anyb);
    free(offs);
    free(corpus);
    free(merges);
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("ok\n");
    return 0;
}
