/*
 * Seeded synthetic input generators.
 *
 * This module is shared by the CPU oracle and by the GPU path's tests and
 * benchmark.  It holds none of the reachability or hash-table arithmetic:
 * only random numbers, transition tables of synthetic models and shuffled
 * duplicate streams.  Both sides receive its outputs as plain arrays.
 *
 * Random source: xorshift64 with the shift triple (13, 7, 17) from
 * G. Marsaglia, "Xorshift RNGs", J. Stat. Software 8(14), 2003.  A zero seed
 * (a fixed point of xorshift) is replaced by a fixed non-zero constant.
 *
 * The paper measures on BEEM models that are not available here; the
 * guarded-transition generator below produces models of the same kind
 * (interleaved processes with local control states and shared variables,
 * the explicit-state setting of the paper's Preliminaries section).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>

#define GEN_NONE 0xFFFFFFFFu
#define GEN_ZERO_SEED_SUBST 0x9E3779B97F4A7C15ull

static inline uint64_t xs64(uint64_t *s)
{
    uint64_t x = *s;
    x ^= x << 13;
    x ^= x >> 7;
    x ^= x << 17;
    *s = x;
    return x;
}

static inline uint64_t seed_of(uint64_t seed)
{
    return seed ? seed : GEN_ZERO_SEED_SUBST;
}

/* n raw xorshift64 outputs. */
void gen_xs64(uint64_t seed, uint64_t *out, uint64_t n)
{
    uint64_t s = seed_of(seed);
    for (uint64_t i = 0; i < n; ++i)
        out[i] = xs64(&s);
}

/* n 32-bit words; each xorshift64 output gives two words, low half first. */
void gen_words(uint64_t seed, uint32_t *out, uint64_t n)
{
    uint64_t s = seed_of(seed);
    uint64_t i = 0;
    for (; i + 1 < n; i += 2) {
        uint64_t x = xs64(&s);
        out[i] = (uint32_t)x;
        out[i + 1] = (uint32_t)(x >> 32);
    }
    if (i < n)
        out[i] = (uint32_t)xs64(&s);
}

/*
 * Guarded-transition model G(seed, P, L, S, D, K).
 * trans is [P][L][K][5] = {target, guard_var, guard_val, eff_var, eff_val}.
 * For every (p, l, k), in that loop order, five outputs x0..x4 are drawn:
 *   target = x0 % L, guard_var = x1 % S, guard_val = x2 % D,
 *   eff_var = x3 % S, eff_val = x4 % D.
 * With S == 0 there are no shared variables: guard_var and eff_var are
 * GEN_NONE and the guard/effect values are 0 (the draws still happen so the
 * target sequence does not depend on S).  Returns 0, or -1 on bad sizes.
 */
int gen_guarded_model(uint64_t seed, uint32_t P, uint32_t L, uint32_t S,
                      uint32_t D, uint32_t K, uint32_t *trans)
{
    if (!P || !L || !K || (S && !D))
        return -1;
    uint64_t s = seed_of(seed);
    size_t o = 0;
    for (uint32_t p = 0; p < P; ++p)
        for (uint32_t l = 0; l < L; ++l)
            for (uint32_t k = 0; k < K; ++k) {
                uint64_t x0 = xs64(&s), x1 = xs64(&s), x2 = xs64(&s);
                uint64_t x3 = xs64(&s), x4 = xs64(&s);
                trans[o + 0] = (uint32_t)(x0 % L);
                if (S) {
                    trans[o + 1] = (uint32_t)(x1 % S);
                    trans[o + 2] = (uint32_t)(x2 % D);
                    trans[o + 3] = (uint32_t)(x3 % S);
                    trans[o + 4] = (uint32_t)(x4 % D);
                } else {
                    trans[o + 1] = GEN_NONE;
                    trans[o + 2] = 0;
                    trans[o + 3] = GEN_NONE;
                    trans[o + 4] = 0;
                }
                o += 5;
            }
    return 0;
}

/* N independent cyclic L-state processes: one unguarded step l -> (l+1) % L. */
int gen_cyclic_model(uint32_t P, uint32_t L, uint32_t *trans)
{
    if (!P || !L)
        return -1;
    size_t o = 0;
    for (uint32_t p = 0; p < P; ++p)
        for (uint32_t l = 0; l < L; ++l) {
            trans[o + 0] = (l + 1) % L;
            trans[o + 1] = GEN_NONE;
            trans[o + 2] = 0;
            trans[o + 3] = GEN_NONE;
            trans[o + 4] = 0;
            o += 5;
        }
    return 0;
}

/* Uniform integer in [0, m) by Lemire's multiply-high reduction. */
static inline uint64_t below(uint64_t *s, uint64_t m)
{
    return (uint64_t)(((unsigned __int128)xs64(s) * m) >> 64);
}

/* Uniformly shuffled identity permutation of [0, n) (Durstenfeld's
 * in-place Fisher-Yates shuffle). */
void gen_permutation(uint64_t seed, uint32_t *perm, uint64_t n)
{
    uint64_t s = seed_of(seed);
    for (uint64_t i = 0; i < n; ++i)
        perm[i] = (uint32_t)i;
    for (uint64_t i = n; i > 1; --i) {
        uint64_t j = below(&s, i);
        uint32_t t = perm[i - 1];
        perm[i - 1] = perm[j];
        perm[j] = t;
    }
}

/*
 * Duplicate stream: n_distinct random rows of W words (gen_words with
 * `seed`) each occurring `copies` times, in the order of a Fisher-Yates
 * shuffle (seed ^ 0xD1B54A32D192ED03) of the multiset.  order[k] is the
 * distinct-row id at stream position k; rows is [n_distinct][W].
 * Materialising the stream is left to the caller (a gather).
 */
void gen_dup_stream(uint64_t seed, uint64_t n_distinct, uint32_t W,
                    uint32_t copies, uint32_t *rows, uint32_t *order)
{
    gen_words(seed, rows, n_distinct * (uint64_t)W);
    uint64_t n = n_distinct * copies;
    gen_permutation(seed ^ 0xD1B54A32D192ED03ull, order, n);
    for (uint64_t k = 0; k < n; ++k)
        order[k] = (uint32_t)(order[k] / copies);
}

/* Gather rows[order[k]] into out[k] (W words each). */
void gen_gather(const uint32_t *rows, const uint32_t *order, uint64_t n,
                uint32_t W, uint32_t *out)
{
    for (uint64_t k = 0; k < n; ++k) {
        const uint32_t *src = rows + (uint64_t)order[k] * W;
        uint32_t *dst = out + k * (uint64_t)W;
        for (uint32_t i = 0; i < W; ++i)
            dst[i] = src[i];
    }
}

/* Poisson arrival times: cumulative sums of -ln(U)/lambda, U in (0, 1]
 * from the top 53 bits of xorshift64 outputs. */
void gen_poisson_arrivals(uint64_t seed, double lambda, double *t, uint64_t n)
{
    uint64_t s = seed_of(seed);
    double acc = 0.0;
    for (uint64_t i = 0; i < n; ++i) {
        double u = ((double)(xs64(&s) >> 11) + 1.0) * (1.0 / 9007199254740992.0);
        acc += -log(u) / lambda;
        t[i] = acc;
    }
}
