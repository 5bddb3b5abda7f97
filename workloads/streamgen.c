/*
 * Seeded synthetic item streams for the k-majority workloads.
 *
 * This file holds input generation only: a counter-based random number
 * generator, a bounded Zipf sampler, id mappings and the adversarial
 * pattern.  It contains none of the Space Saving / COMBINE arithmetic, and
 * both the CPU oracle and the GPU library consume the bytes it writes.
 *
 * The paper evaluates on synthetic Zipf streams with skew 1.1 and 1.8
 * (Section 4, "Design of experiments", Table 1) but gives neither the
 * universe, the generator nor the seed, so every choice below is ours.
 *
 * Random numbers: SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) used as a counter-based
 * generator: draw (key, ctr) is the output of SplitMix64's mixing function
 * applied to key + (ctr + 1) * 0x9E3779B97F4A7C15, i.e. the (ctr+1)-th output
 * of a SplitMix64 sequence seeded with `key`.  Every item is therefore a pure
 * function of (seed, index), so generation is split over threads freely.
 *
 * Zipf(s, N): P(rank r) proportional to r^-s for r = 1..N, sampled by
 * rejection-inversion (W. Hormann and G. Derflinger, "Rejection-inversion
 * to generate variates from monotone discrete distributions", ACM TOMACS
 * 6(3), 1996), which works for every s > 0 and N up to 2^32 in O(1)
 * expected time per sample.
 *
 * Id mappings: a seeded Fisher-Yates permutation of [0, N) for small
 * universes, or the MurmurHash3 32-bit finaliser (a bijection on uint32)
 * applied to (r - 1) XOR key for universes up to 2^32.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN64 0x9E3779B97F4A7C15ULL

static inline uint64_t sm64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* (ctr+1)-th output of SplitMix64 seeded with key. */
uint64_t wl_draw(uint64_t key, uint64_t ctr) {
    return sm64_mix(key + (ctr + 1) * GOLDEN64);
}

/* Uniform double in [0, 1) with 53 random bits. */
static inline double unit53(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }

/* MurmurHash3 fmix32: xor-shifts and odd multiplies, each a bijection. */
uint32_t wl_fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

/* ---------------- rejection-inversion Zipf sampler ---------------- */

typedef struct {
    double s;       /* exponent */
    double n;       /* number of ranks N (as double, exact up to 2^53) */
    double h_x1;    /* H(1.5) - h(1) */
    double h_n;     /* H(N + 0.5) */
    double sq;      /* squeeze constant 2 - Hinv(H(2.5) - h(2)) */
} zipf_t;

/* log1p(x)/x, continuous at 0. */
static double helper1(double x) {
    if (fabs(x) > 1e-8) return log1p(x) / x;
    return 1.0 - x * (0.5 - x * (1.0 / 3.0 - 0.25 * x));
}

/* expm1(x)/x, continuous at 0. */
static double helper2(double x) {
    if (fabs(x) > 1e-8) return expm1(x) / x;
    return 1.0 + x * 0.5 * (1.0 + x * (1.0 / 3.0) * (1.0 + 0.25 * x));
}

/* h(x) = x^-s, the (unnormalised) hat density. */
static double zh(const zipf_t* z, double x) { return exp(-z->s * log(x)); }

/* H(x) = integral of h: (x^(1-s) - 1)/(1 - s), log(x) at s = 1. */
static double zH(const zipf_t* z, double x) {
    double lx = log(x);
    return helper2((1.0 - z->s) * lx) * lx;
}

/* Inverse of H. */
static double zHinv(const zipf_t* z, double y) {
    double t = y * (1.0 - z->s);
    if (t < -1.0) t = -1.0; /* guards rounding at the lower end */
    return exp(helper1(t) * y);
}

static void zipf_init(zipf_t* z, double s, double n) {
    z->s = s;
    z->n = n;
    z->h_x1 = zH(z, 1.5) - 1.0;
    z->h_n = zH(z, n + 0.5);
    z->sq = 2.0 - zHinv(z, zH(z, 2.5) - zh(z, 2.0));
}

/* Rank in [1, N] for item index i; attempt t uses counter (i << 8) | t. */
static uint64_t zipf_rank(const zipf_t* z, uint64_t key, uint64_t i) {
    uint64_t k = 1;
    for (unsigned t = 0; t < 256; ++t) {
        double u = z->h_n + unit53(wl_draw(key, (i << 8) | t)) * (z->h_x1 - z->h_n);
        double x = zHinv(z, u);
        double kd = floor(x + 0.5);
        if (kd < 1.0) kd = 1.0;
        if (kd > z->n) kd = z->n;
        k = (uint64_t)kd;
        if (kd - x <= z->sq || u >= zH(z, kd + 0.5) - zh(z, kd)) return k;
    }
    return k; /* acceptance probability per attempt exceeds 1/2; unreachable in practice */
}

/* ---------------- threaded drivers ---------------- */

enum { K_ZIPF_PERM = 0, K_ZIPF_HASH = 1, K_UNIFORM = 2, K_ADVERSARIAL = 3 };

typedef struct {
    int kind;
    uint32_t* out;
    uint64_t lo, hi;
    zipf_t z;
    uint64_t key;        /* random key for draws */
    uint32_t idkey;      /* xor key for hashed ids */
    const uint32_t* perm;
    uint32_t adv_d;      /* adversarial: number of round-robin ids */
} job_t;

static void* worker(void* arg) {
    job_t* j = (job_t*)arg;
    for (uint64_t i = j->lo; i < j->hi; ++i) {
        uint32_t v;
        switch (j->kind) {
        case K_ZIPF_PERM:
            v = j->perm[zipf_rank(&j->z, j->key, i) - 1];
            break;
        case K_ZIPF_HASH:
            v = wl_fmix32((uint32_t)(zipf_rank(&j->z, j->key, i) - 1) ^ j->idkey);
            break;
        case K_UNIFORM:
            v = (uint32_t)(wl_draw(j->key, i) >> 32);
            break;
        default: { /* adversarial: every 20th position (i % 20 == 19) holds the planted id */
            uint64_t g = i / 20, o = i % 20;
            if (o == 19) {
                v = wl_fmix32(j->adv_d ^ j->idkey);
            } else {
                uint64_t q = g * 19 + o;
                v = wl_fmix32((uint32_t)(q % j->adv_d) ^ j->idkey);
            }
        }
        }
        j->out[i] = v;
    }
    return NULL;
}

static int run_jobs(job_t proto, uint64_t n, int threads) {
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    if ((uint64_t)threads > n / 65536 + 1) threads = (int)(n / 65536 + 1);
    pthread_t tid[256];
    job_t jobs[256];
    for (int t = 0; t < threads; ++t) {
        jobs[t] = proto;
        jobs[t].lo = n * (uint64_t)t / (uint64_t)threads;
        jobs[t].hi = n * (uint64_t)(t + 1) / (uint64_t)threads;
    }
    int started = 0;
    for (int t = 1; t < threads; ++t) {
        if (pthread_create(&tid[t], NULL, worker, &jobs[t]) != 0) break;
        started = t;
    }
    worker(&jobs[0]);
    for (int t = 1; t <= started; ++t) pthread_join(tid[t], NULL);
    for (int t = started + 1; t < threads; ++t) worker(&jobs[t]); /* threads that failed to start */
    return 0;
}

/* Seeded Fisher-Yates permutation of [0, N): position i (from N-1 down to 1)
 * swaps with j uniform in [0, i], j = floor(draw * (i+1) / 2^64). */
int wl_permutation(uint32_t* perm, uint32_t n_univ, uint64_t key) {
    for (uint32_t i = 0; i < n_univ; ++i) perm[i] = i;
    for (uint32_t i = n_univ; i-- > 1;) {
        unsigned __int128 prod = (unsigned __int128)wl_draw(key, i) * (uint64_t)(i + 1);
        uint32_t j = (uint32_t)(prod >> 64);
        uint32_t t = perm[i];
        perm[i] = perm[j];
        perm[j] = t;
    }
    return 0;
}

/* Zipf(s) over ranks 1..n_univ (n_univ <= 2^28), ids = permutation of [0, n_univ). */
int wl_zipf_perm(uint32_t* out, uint64_t n, double s, uint32_t n_univ, uint64_t key_rank,
                 uint64_t key_perm, int threads) {
    if (!out || n_univ == 0 || !(s > 0.0)) return -1;
    uint32_t* perm = (uint32_t*)malloc((size_t)n_univ * sizeof(uint32_t));
    if (!perm) return -2;
    wl_permutation(perm, n_univ, key_perm);
    job_t p;
    memset(&p, 0, sizeof p);
    p.kind = K_ZIPF_PERM;
    p.out = out;
    zipf_init(&p.z, s, (double)n_univ);
    p.key = key_rank;
    p.perm = perm;
    run_jobs(p, n, threads);
    free(perm);
    return 0;
}

/* Zipf(s) over ranks 1..n_univ (n_univ <= 2^32), id = fmix32((r-1) ^ idkey). */
int wl_zipf_hashed(uint32_t* out, uint64_t n, double s, uint64_t n_univ, uint64_t key_rank,
                   uint32_t idkey, int threads) {
    if (!out || n_univ == 0 || n_univ > (1ULL << 32) || !(s > 0.0)) return -1;
    job_t p;
    memset(&p, 0, sizeof p);
    p.kind = K_ZIPF_HASH;
    p.out = out;
    zipf_init(&p.z, s, (double)n_univ);
    p.key = key_rank;
    p.idkey = idkey;
    run_jobs(p, n, threads);
    return 0;
}

/* i.i.d. uniform uint32 items. */
int wl_uniform(uint32_t* out, uint64_t n, uint64_t key, int threads) {
    if (!out) return -1;
    job_t p;
    memset(&p, 0, sizeof p);
    p.kind = K_UNIFORM;
    p.out = out;
    p.key = key;
    run_jobs(p, n, threads);
    return 0;
}

/* Round-robin over d hashed ids with a planted id at every 20th position
 * (positions i with i % 20 == 19).  The planted id is fmix32(d ^ idkey),
 * which is outside the round-robin set because fmix32 is a bijection. */
int wl_adversarial(uint32_t* out, uint64_t n, uint32_t d, uint32_t idkey, int threads) {
    if (!out || d == 0) return -1;
    job_t p;
    memset(&p, 0, sizeof p);
    p.kind = K_ADVERSARIAL;
    p.out = out;
    p.idkey = idkey;
    p.adv_d = d;
    run_jobs(p, n, threads);
    return 0;
}

/* Ranks only (for tests of the sampler's distribution). */
int wl_zipf_ranks(uint64_t* out, uint64_t n, double s, uint64_t n_univ, uint64_t key) {
    if (!out || n_univ == 0 || !(s > 0.0)) return -1;
    zipf_t z;
    zipf_init(&z, s, (double)n_univ);
    for (uint64_t i = 0; i < n; ++i) out[i] = zipf_rank(&z, key, i);
    return 0;
}
