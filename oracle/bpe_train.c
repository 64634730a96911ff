/*
 * BPE trainer (oracle side). TEST INFRASTRUCTURE ONLY: it writes the ranked
 * merge tables the BPE workloads encode with; the GPU library never links it.
 *
 * The paper benchmarks BPE vocabularies only through upstream tokenizers and
 * learns none itself (static vocabularies built offline, "Dynamic
 * Vocabularies and Online BPE"). The rule below is the classic greedy BPE
 * learner of Sennrich et al., which the introduction cites, on one DNA
 * string:
 *
 *   symbols start as bases (A=5 C=6 G=7 T=8, either case); any other byte is
 *   a barrier that no pair crosses. Repeat up to R times: count every
 *   adjacent pair of symbols (overlapping occurrences of a pair (X, X) each
 *   count); take the pair with the highest count, ties to the smallest
 *   (left id, right id); stop if that count is below 2; replace every
 *   non-overlapping occurrence, scanning left to right, by a new symbol with
 *   id 10 + r, where r is the merge's rank.
 *
 * Counting from scratch each step costs R passes over the corpus, so counts
 * are kept incrementally (a linked list over positions, a dense pair-count
 * matrix, per-pair occurrence lists and a lazy max-heap). A pure-Python
 * recount of the same rule pins this file on small corpora.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define DEAD (-1)
#define WALL (-2)

typedef struct { int32_t *p; int64_t n, cap; } vec32;

static void vec_push(vec32 *v, int32_t x) {
    if (v->n == v->cap) {
        v->cap = v->cap ? v->cap * 2 : 8;
        v->p = (int32_t *)realloc(v->p, sizeof(int32_t) * (size_t)v->cap);
    }
    v->p[v->n++] = x;
}

typedef struct { int32_t count, a, b; } hent;

/* heap order: higher count first, then smaller a, then smaller b */
static int hless(const hent *x, const hent *y) {
    if (x->count != y->count) return x->count > y->count;
    if (x->a != y->a) return x->a < y->a;
    return x->b < y->b;
}

typedef struct { hent *h; int64_t n, cap; } heap;

static void heap_push(heap *H, hent e) {
    if (H->n == H->cap) {
        H->cap = H->cap ? H->cap * 2 : 1024;
        H->h = (hent *)realloc(H->h, sizeof(hent) * (size_t)H->cap);
    }
    int64_t i = H->n++;
    H->h[i] = e;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (!hless(&H->h[i], &H->h[p])) break;
        hent t = H->h[i]; H->h[i] = H->h[p]; H->h[p] = t;
        i = p;
    }
}

static hent heap_pop(heap *H) {
    hent top = H->h[0];
    H->h[0] = H->h[--H->n];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < H->n && hless(&H->h[l], &H->h[m])) m = l;
        if (r < H->n && hless(&H->h[r], &H->h[m])) m = r;
        if (m == i) break;
        hent t = H->h[i]; H->h[i] = H->h[m]; H->h[m] = t;
        i = m;
    }
    return top;
}

static int cmp_i32(const void *x, const void *y) {
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    return (a > b) - (a < b);
}

static int base_id(uint8_t c) {
    switch (c) {
    case 'A': case 'a': return 5;
    case 'C': case 'c': return 6;
    case 'G': case 'g': return 7;
    case 'T': case 't': return 8;
    default: return WALL;
    }
}

/*
 * Learn up to R merges from corpus[0..n). Writes out_merges[2r], [2r+1] =
 * (left id, right id) of rank r. Returns the number learned, or -1 if the
 * corpus is too long for 32-bit positions, -2 on allocation failure.
 */
int32_t oracle_bpe_train(const uint8_t *corpus, int64_t n, int32_t R, int32_t *out_merges) {
    if (n >= 0x7FFFFFFF) return -1;
    if (R <= 0 || n < 2) return 0;
    const int64_t V = 10 + (int64_t)R;
    int32_t *tok = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *nxt = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *prv = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *cnt = (int32_t *)calloc((size_t)(V * V), sizeof(int32_t));
    int32_t *occ_id = (int32_t *)malloc(sizeof(int32_t) * (size_t)(V * V));
    int32_t *stamp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(V * V));
    if (!tok || !nxt || !prv || !cnt || !occ_id || !stamp) return -2;
    memset(occ_id, 0xFF, sizeof(int32_t) * (size_t)(V * V));
    memset(stamp, 0xFF, sizeof(int32_t) * (size_t)(V * V));
    vec32 *occ = NULL;
    int64_t n_occ = 0, cap_occ = 0;
    heap H = {0, 0, 0};

#define PAIR(a, b) ((int64_t)(a) * V + (b))

    for (int64_t i = 0; i < n; ++i) {
        tok[i] = base_id(corpus[i]);
        nxt[i] = (i + 1 < n) ? (int32_t)(i + 1) : DEAD;
        prv[i] = (i > 0) ? (int32_t)(i - 1) : DEAD;
    }

    /* occurrence list of pair key k, created on first use */
#define GET_OCC(key, outp) do {                                                   \
        int64_t _k = (key);                                                        \
        if (occ_id[_k] < 0) {                                                      \
            if (n_occ == cap_occ) {                                                \
                cap_occ = cap_occ ? cap_occ * 2 : 4096;                            \
                occ = (vec32 *)realloc(occ, sizeof(vec32) * (size_t)cap_occ);      \
            }                                                                      \
            occ[n_occ].p = NULL; occ[n_occ].n = 0; occ[n_occ].cap = 0;             \
            occ_id[_k] = (int32_t)n_occ++;                                         \
        }                                                                          \
        (outp) = &occ[occ_id[_k]];                                                 \
    } while (0)

    for (int64_t i = 0; i + 1 < n; ++i) {
        int32_t a = tok[i], b = tok[i + 1];
        if (a < 0 || b < 0) continue;
        cnt[PAIR(a, b)]++;
        vec32 *v; GET_OCC(PAIR(a, b), v); vec_push(v, (int32_t)i);
    }
    for (int32_t a = 5; a <= 8; ++a)
        for (int32_t b = 5; b <= 8; ++b)
            if (cnt[PAIR(a, b)] > 0) heap_push(&H, (hent){cnt[PAIR(a, b)], a, b});

    int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * 2 * 16);
    int64_t n_touched = 0, cap_touched = 16;
    int32_t learned = 0;
    for (int32_t r = 0; r < R; ++r) {
        /* pop the best valid pair */
        int found = 0;
        hent best = {0, 0, 0};
        while (H.n > 0) {
            hent e = heap_pop(&H);
            int32_t cur = cnt[PAIR(e.a, e.b)];
            if (cur == e.count) { best = e; found = 1; break; }
            if (cur < e.count && cur > 0) heap_push(&H, (hent){cur, e.a, e.b});
            /* cur > e.count: a fresher entry for this pair is already queued */
        }
        if (!found || best.count < 2) break;
        const int32_t a = best.a, b = best.b, nid = 10 + r;
        out_merges[2 * r] = a;
        out_merges[2 * r + 1] = b;
        learned = r + 1;

        vec32 *v; GET_OCC(PAIR(a, b), v);
        int32_t *pos = v->p;
        int64_t npos = v->n;
        v->p = NULL; v->n = 0; v->cap = 0;
        qsort(pos, (size_t)npos, sizeof(int32_t), cmp_i32);
        n_touched = 0;
        for (int64_t q = 0; q < npos; ++q) {
            int32_t i = pos[q];
            if (q > 0 && pos[q - 1] == i) continue;
            if (tok[i] != a) continue;
            int32_t j = nxt[i];
            if (j == DEAD || tok[j] != b) continue;
            int32_t p = prv[i], k = nxt[j];
            /* remove the pairs that disappear */
            cnt[PAIR(a, b)]--;
            if (p != DEAD && tok[p] >= 0) cnt[PAIR(tok[p], a)]--;
            if (k != DEAD && tok[k] >= 0) cnt[PAIR(b, tok[k])]--;
            /* splice */
            tok[i] = nid;
            tok[j] = DEAD - 10; /* dead position, never a valid id */
            nxt[i] = k;
            if (k != DEAD) prv[k] = i;
            /* add the pairs that appear */
            if (p != DEAD && tok[p] >= 0) {
                int64_t key = PAIR(tok[p], nid);
                cnt[key]++;
                vec32 *w; GET_OCC(key, w); vec_push(w, p);
                if (stamp[key] != r) {
                    stamp[key] = r;
                    if (n_touched == cap_touched) { cap_touched *= 2; touched = (int32_t *)realloc(touched, sizeof(int32_t) * 2 * (size_t)cap_touched); }
                    touched[2 * n_touched] = tok[p]; touched[2 * n_touched + 1] = nid; n_touched++;
                }
            }
            if (k != DEAD && tok[k] >= 0) {
                int64_t key = PAIR(nid, tok[k]);
                cnt[key]++;
                vec32 *w; GET_OCC(key, w); vec_push(w, i);
                if (stamp[key] != r) {
                    stamp[key] = r;
                    if (n_touched == cap_touched) { cap_touched *= 2; touched = (int32_t *)realloc(touched, sizeof(int32_t) * 2 * (size_t)cap_touched); }
                    touched[2 * n_touched] = nid; touched[2 * n_touched + 1] = tok[k]; n_touched++;
                }
            }
        }
        free(pos);
        for (int64_t t = 0; t < n_touched; ++t) {
            int32_t x = touched[2 * t], y = touched[2 * t + 1];
            if (cnt[PAIR(x, y)] > 0) heap_push(&H, (hent){cnt[PAIR(x, y)], x, y});
        }
    }

    for (int64_t q = 0; q < n_occ; ++q) free(occ[q].p);
    free(occ); free(H.h); free(touched);
    free(tok); free(nxt); free(prv); free(cnt); free(occ_id); free(stamp);
    return learned;
#undef PAIR
#undef GET_OCC
}
