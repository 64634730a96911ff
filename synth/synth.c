/*
 * Seeded synthetic DNA generators.
 *
 * This module only produces inputs: it holds none of the tokenizer's
 * arithmetic (no byte classification, no token ids). Both the CPU oracle
 * and the GPU path consume what it writes.
 *
 * Random numbers: splitmix64 (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) seeds xoshiro256**
 * (Blackman and Vigna, "Scrambled linear pseudorandom number generators",
 * 2018). Uniform doubles take the top 53 bits.
 *
 * Models (the workload recipes of the paper's synthetic microbenchmarks,
 * made concrete):
 *   - i.i.d. bases: P('N') = p_n, otherwise uniform over "ACGT".
 *   - order-m Markov chain over ACGT: 4^m contexts, each transition row
 *     drawn from Dirichlet(1,1,1,1) (normalised Exp(1) draws).
 *   - soft-masking: alternating renewal process, lowercase runs with
 *     geometric length (mean mu_mask) and uppercase runs (mean mu_open).
 *   - N runs: alternating renewal process of gaps (mean mu_gap) and N runs
 *     (mean mu_run); an N takes the case of the base it replaces.
 *   - invalid bytes: each position independently with probability p,
 *     replaced by a byte drawn uniformly from the 246 values outside
 *     "ACGTNacgtn".
 */
#include <stdint.h>
#include <math.h>
#include <string.h>

typedef struct { uint64_t s[4]; } rng_t;

static uint64_t splitmix64_next(uint64_t *x) {
    uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static void rng_seed(rng_t *r, uint64_t seed) {
    uint64_t x = seed;
    for (int i = 0; i < 4; ++i) r->s[i] = splitmix64_next(&x);
}

static inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static inline uint64_t rng_next(rng_t *r) {
    uint64_t *s = r->s;
    uint64_t result = rotl(s[1] * 5, 7) * 9;
    uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl(s[3], 45);
    return result;
}

/* uniform in [0, 1) */
static inline double rng_u01(rng_t *r) { return (double)(rng_next(r) >> 11) * 0x1.0p-53; }
/* uniform in (0, 1] */
static inline double rng_u01_open0(rng_t *r) { return 1.0 - rng_u01(r); }

/* geometric on {1, 2, ...} with the given mean (>= 1) */
static int64_t rng_geom(rng_t *r, double mean) {
    if (mean <= 1.0) return 1;
    double p = 1.0 / mean;
    double u = rng_u01_open0(r);
    double g = ceil(log(u) / log1p(-p));
    if (g < 1.0) g = 1.0;
    if (g > 9.0e18) g = 9.0e18;
    return (int64_t)g;
}

static const uint8_t ACGT[4] = {'A', 'C', 'G', 'T'};

uint64_t synth_substream(uint64_t base_seed, uint64_t a, uint64_t b) {
    uint64_t x = base_seed ^ (a * 0xD1B54A32D192ED03ull) ^ (b * 0x8CB92BA72F3D8DD7ull);
    splitmix64_next(&x);
    return splitmix64_next(&x);
}

/* i.i.d. uppercase bases with P('N') = p_n, else uniform ACGT */
void synth_iid(uint64_t seed, uint8_t *out, int64_t n, double p_n) {
    rng_t r;
    rng_seed(&r, seed);
    for (int64_t i = 0; i < n; ++i) {
        double u = rng_u01(&r);
        if (u < p_n) out[i] = 'N';
        else out[i] = ACGT[(rng_next(&r) >> 62) & 3];
    }
}

/* Transition table of an order-m chain: cum[ctx*4 + j] = P(next <= j | ctx). */
static void markov_table(rng_t *r, int order, double *cum) {
    int64_t nctx = (int64_t)1 << (2 * order);
    for (int64_t c = 0; c < nctx; ++c) {
        double e[4], s = 0.0;
        for (int j = 0; j < 4; ++j) { e[j] = -log(rng_u01_open0(r)); s += e[j]; }
        double acc = 0.0;
        for (int j = 0; j < 4; ++j) { acc += e[j] / s; cum[c * 4 + j] = acc; }
        cum[c * 4 + 3] = 1.0;
    }
}

/*
 * Order-m Markov chain over uppercase ACGT. table_seed fixes the transition
 * rows (shared by every sequence of one genome model); seq_seed drives the
 * walk. cum_scratch must hold 4 * 4^order doubles.
 */
void synth_markov(uint64_t table_seed, uint64_t seq_seed, int order, uint8_t *out, int64_t n,
                  double *cum_scratch) {
    rng_t rt, r;
    rng_seed(&rt, table_seed);
    markov_table(&rt, order, cum_scratch);
    rng_seed(&r, seq_seed);
    uint64_t mask = ((uint64_t)1 << (2 * order)) - 1;
    uint64_t ctx = 0;
    for (int i = 0; i < order && i < n; ++i) {
        int d = (int)(rng_next(&r) >> 62);
        out[i] = ACGT[d];
        ctx = ((ctx << 2) | (uint64_t)d) & mask;
    }
    for (int64_t i = order; i < n; ++i) {
        double u = rng_u01(&r);
        const double *c = cum_scratch + ctx * 4;
        int d = (u < c[0]) ? 0 : (u < c[1]) ? 1 : (u < c[2]) ? 2 : 3;
        out[i] = ACGT[d];
        ctx = ((ctx << 2) | (uint64_t)d) & mask;
    }
}

/* Lowercase runs (mean mu_mask) alternating with uppercase runs (mean mu_open). */
void synth_softmask(uint64_t seed, uint8_t *buf, int64_t n, double mu_mask, double mu_open) {
    rng_t r;
    rng_seed(&r, seed);
    /* start in the stationary state */
    int masked = rng_u01(&r) < mu_mask / (mu_mask + mu_open);
    int64_t i = 0;
    while (i < n) {
        int64_t len = rng_geom(&r, masked ? mu_mask : mu_open);
        int64_t end = (n - i < len) ? n : i + len;
        if (masked)
            for (int64_t j = i; j < end; ++j) buf[j] = (uint8_t)(buf[j] | 0x20);
        i = end;
        masked = !masked;
    }
}

/* N runs (mean mu_run) separated by gaps (mean mu_gap); case follows the base replaced. */
void synth_nruns(uint64_t seed, uint8_t *buf, int64_t n, double mu_run, double mu_gap) {
    rng_t r;
    rng_seed(&r, seed);
    int in_run = rng_u01(&r) < mu_run / (mu_run + mu_gap);
    int64_t i = 0;
    while (i < n) {
        int64_t len = rng_geom(&r, in_run ? mu_run : mu_gap);
        int64_t end = (n - i < len) ? n : i + len;
        if (in_run)
            for (int64_t j = i; j < end; ++j) buf[j] = (buf[j] & 0x20) ? 'n' : 'N';
        i = end;
        in_run = !in_run;
    }
}

/* Each position independently becomes one of the 246 non-"ACGTNacgtn" bytes with prob. p. */
void synth_invalid(uint64_t seed, uint8_t *buf, int64_t n, double p) {
    if (p <= 0.0) return;
    static const char dna[] = "ACGTNacgtn";
    uint8_t others[256];
    int m = 0;
    for (int b = 0; b < 256; ++b) {
        int is_dna = 0;
        for (int j = 0; j < 10; ++j) is_dna |= (b == (uint8_t)dna[j]);
        if (!is_dna) others[m++] = (uint8_t)b;
    }
    rng_t r;
    rng_seed(&r, seed);
    int64_t i = rng_geom(&r, 1.0 / p) - 1;
    while (i < n) {
        buf[i] = others[rng_next(&r) % (uint64_t)m];
        i += rng_geom(&r, 1.0 / p);
    }
}

/* Uniform bytes over all 256 values (boundary fuzzing). */
void synth_bytes(uint64_t seed, uint8_t *out, int64_t n) {
    rng_t r;
    rng_seed(&r, seed);
    for (int64_t i = 0; i < n; ++i) out[i] = (uint8_t)(rng_next(&r) >> 56);
}

/* Raw 64-bit draws (tests pin the generator to its published definition). */
void synth_raw(uint64_t seed, uint64_t *out, int64_t n) {
    rng_t r;
    rng_seed(&r, seed);
    for (int64_t i = 0; i < n; ++i) out[i] = rng_next(&r);
}
