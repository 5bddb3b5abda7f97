/*
 * CPU oracle for the Frequent (Misra-Gries) summary and its parallel merge --
 * TEST INFRASTRUCTURE ONLY, like pss_oracle.c in this directory.
 *
 * Section 2 of the paper names Frequent (Misra and Gries; Demaine et al.;
 * Karp et al.) as the counter-based method whose summaries the authors
 * merged in parallel before Space Saving, without restating either the
 * algorithm or the merge.  This file states the textbook forms, plainly:
 *
 *   Frequent for the k-majority problem keeps k - 1 counters (Misra and
 *   Gries; with k = 2 it is Boyer and Moore's majority vote): a monitored item
 *   adds 1 to its counter; an unmonitored item takes a free counter with
 *   count 1 while fewer than k - 1 are used; otherwise every counter loses 1
 *   (counters reaching 0 are freed) and the item itself is dropped.  D counts
 *   those decrement steps; each removes k occurrences, so D * k <= n, and for
 *   every item f - D <= f^ <= f (f^ = 0 when unmonitored).
 *
 *   Merge of two such summaries (the mergeable-summaries combine of Agarwal,
 *   Cormode, Huang, Phillips, Wei and Yi): add the counts of the union; if
 *   more than k - 1 items remain, subtract the k-th largest count c from all
 *   of them and keep those still positive; D = D1 + D2 + c.  The bounds above
 *   hold for the concatenated stream.
 *
 *   The parallel form follows Algorithm 1 with this merge as the reduction
 *   operator: the same chunk bounds, the same fixed binary tree.  The report
 *   is every monitored item whose upper bound f^ + D exceeds n / k, i.e.
 *   (f^ + D) * k > n, in the order (count descending, item ascending).
 *
 * All arithmetic is integer (uint64).  The entry layout is the 24-byte host
 * entry; the error field is 0 (the summary-wide bound D replaces it).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint32_t item;
    uint32_t reserved;
    uint64_t count;
    uint64_t error;
} fq_entry;

/* ------------------------------------------------------------------------
 * Sequential Frequent: counters in arrays 0..k-1 (compacted after every
 * decrement step), a chained hash map item -> counter index.
 * ---------------------------------------------------------------------- */

typedef struct {
    uint32_t k, size, nbuckets;
    uint32_t* item;
    uint64_t* count;
    int32_t* head;
    int32_t* next;
} fq_state;

static uint32_t fq_bucket(const fq_state* s, uint32_t x) { return (x * 2246822519u) & (s->nbuckets - 1); }

static int32_t fq_find(const fq_state* s, uint32_t x) {
    for (int32_t c = s->head[fq_bucket(s, x)]; c >= 0; c = s->next[c])
        if (s->item[c] == x) return c;
    return -1;
}

static void fq_rehash(fq_state* s) {
    for (uint32_t b = 0; b < s->nbuckets; ++b) s->head[b] = -1;
    for (uint32_t c = 0; c < s->size; ++c) {
        uint32_t b = fq_bucket(s, s->item[c]);
        s->next[c] = s->head[b];
        s->head[b] = (int32_t)c;
    }
}

/* k here is the number of counters */
static int fq_init(fq_state* s, uint32_t k) {
    memset(s, 0, sizeof(*s));
    s->k = k;
    s->nbuckets = 1;
    while (s->nbuckets < 2 * k) s->nbuckets <<= 1;
    s->item = (uint32_t*)calloc(k, sizeof(uint32_t));
    s->count = (uint64_t*)calloc(k, sizeof(uint64_t));
    s->head = (int32_t*)malloc(sizeof(int32_t) * s->nbuckets);
    s->next = (int32_t*)malloc(sizeof(int32_t) * k);
    if (!s->item || !s->count || !s->head || !s->next) return -1;
    for (uint32_t b = 0; b < s->nbuckets; ++b) s->head[b] = -1;
    return 0;
}

static void fq_free(fq_state* s) {
    free(s->item);
    free(s->count);
    free(s->head);
    free(s->next);
}

/* one item; returns 1 when it caused a decrement step */
static int fq_process(fq_state* s, uint32_t x) {
    int32_t c = fq_find(s, x);
    if (c >= 0) {
        s->count[c] += 1;
        return 0;
    }
    if (s->size < s->k) {
        uint32_t i = s->size++;
        s->item[i] = x;
        s->count[i] = 1;
        uint32_t b = fq_bucket(s, x);
        s->next[i] = s->head[b];
        s->head[b] = (int32_t)i;
        return 0;
    }
    /* every counter loses 1; the ones reaching 0 are freed; x is dropped */
    uint32_t w = 0;
    for (uint32_t i = 0; i < s->size; ++i) {
        s->count[i] -= 1;
        if (s->count[i] > 0) {
            s->item[w] = s->item[i];
            s->count[w] = s->count[i];
            ++w;
        }
    }
    s->size = w;
    fq_rehash(s);
    return 1;
}

/* Frequent for the k-majority problem (k - 1 counters) over items[0, len);
 * out holds up to k - 1 entries */
int oracle_frequent(const uint32_t* items, uint64_t len, uint32_t k, fq_entry* out, uint32_t* size,
                    uint64_t* decrements) {
    if (k < 2) return -1;
    fq_state s;
    if (fq_init(&s, k - 1) != 0) {
        fq_free(&s);
        return -2;
    }
    uint64_t d = 0;
    for (uint64_t i = 0; i < len; ++i) d += (uint64_t)fq_process(&s, items[i]);
    for (uint32_t c = 0; c < s.size; ++c) {
        out[c].item = s.item[c];
        out[c].reserved = 0;
        out[c].count = s.count[c];
        out[c].error = 0;
    }
    *size = s.size;
    *decrements = d;
    fq_free(&s);
    return 0;
}

/* ------------------------------------------------------------------------
 * Merge
 * ---------------------------------------------------------------------- */

static int fq_item_cmp(const void* pa, const void* pb) {
    const fq_entry* a = (const fq_entry*)pa;
    const fq_entry* b = (const fq_entry*)pb;
    return (a->item > b->item) - (a->item < b->item);
}

static int fq_count_desc(const void* pa, const void* pb) {
    const fq_entry* a = (const fq_entry*)pa;
    const fq_entry* b = (const fq_entry*)pb;
    if (a->count != b->count) return a->count > b->count ? -1 : 1;
    return (a->item > b->item) - (a->item < b->item);
}

int oracle_frequent_merge(const fq_entry* s1, uint32_t n1, uint64_t d1, const fq_entry* s2, uint32_t n2,
                          uint64_t d2, uint32_t k, fq_entry* out, uint32_t* nout, uint64_t* dout) {
    uint32_t n = n1 + n2;
    fq_entry* u = (fq_entry*)malloc(sizeof(fq_entry) * (n ? n : 1));
    if (!u) return -2;
    memcpy(u, s1, sizeof(fq_entry) * n1);
    memcpy(u + n1, s2, sizeof(fq_entry) * n2);
    /* union with added counts: sort by item, fold equal neighbours */
    qsort(u, n, sizeof(fq_entry), fq_item_cmp);
    uint32_t m = 0;
    for (uint32_t i = 0; i < n; ++i) {
        if (m > 0 && u[m - 1].item == u[i].item)
            u[m - 1].count += u[i].count;
        else
            u[m++] = u[i];
    }
    uint64_t c = 0;
    if (m > k - 1) {
        /* the k-th largest count */
        qsort(u, m, sizeof(fq_entry), fq_count_desc);
        c = u[k - 1].count;
    }
    uint32_t w = 0;
    for (uint32_t i = 0; i < m; ++i) {
        if (u[i].count > c) {
            out[w] = u[i];
            out[w].count -= c;
            out[w].error = 0;
            out[w].reserved = 0;
            ++w;
        }
    }
    free(u);
    *nout = w;
    *dout = d1 + d2 + c;
    return 0;
}

/* ------------------------------------------------------------------------
 * Parallel form: chunks, fixed tree, report
 * ---------------------------------------------------------------------- */

static uint64_t fq_chunk_begin(uint64_t n, uint32_t chunks, uint32_t c) {
    return (uint64_t)(((unsigned __int128)c * n) / chunks);
}

/* ent: count summaries at stride k; size[i], dec[i]: their sizes and D.
 * Level-wise pairs (2j, 2j+1) over chunk index, an odd last one promoted;
 * the root ends at position 0. */
int oracle_frequent_tree(fq_entry* ent, uint32_t* size, uint64_t* dec, uint32_t count, uint32_t k) {
    fq_entry* tmp = (fq_entry*)malloc(sizeof(fq_entry) * (k ? k : 1));
    if (!tmp) return -2;
    for (uint32_t step = 1; step < count; step <<= 1) {
        for (uint64_t a = 0; a + step < count; a += 2ull * step) {
            uint64_t b = a + step;
            uint32_t nout = 0;
            uint64_t dout = 0;
            int rc = oracle_frequent_merge(ent + a * k, size[a], dec[a], ent + b * k, size[b], dec[b], k, tmp, &nout,
                                           &dout);
            if (rc != 0) {
                free(tmp);
                return rc;
            }
            memcpy(ent + a * k, tmp, sizeof(fq_entry) * nout);
            size[a] = nout;
            dec[a] = dout;
        }
    }
    free(tmp);
    return 0;
}

int oracle_frequent_summary(const uint32_t* items, uint64_t n, uint32_t k, uint32_t chunks, fq_entry* out,
                            uint32_t* nout, uint64_t* dout) {
    if (k < 2 || chunks < 1) return -1;
    fq_entry* ent = (fq_entry*)malloc(sizeof(fq_entry) * (size_t)k * chunks);
    uint32_t* size = (uint32_t*)malloc(sizeof(uint32_t) * chunks);
    uint64_t* dec = (uint64_t*)malloc(sizeof(uint64_t) * chunks);
    if (!ent || !size || !dec) {
        free(ent);
        free(size);
        free(dec);
        return -2;
    }
    int rc = 0;
    for (uint32_t c = 0; c < chunks && rc == 0; ++c) {
        uint64_t b = fq_chunk_begin(n, chunks, c), e = fq_chunk_begin(n, chunks, c + 1);
        rc = oracle_frequent(items + b, e - b, k, ent + (size_t)c * k, &size[c], &dec[c]);
    }
    if (rc == 0) rc = oracle_frequent_tree(ent, size, dec, chunks, k);
    if (rc == 0) {
        memcpy(out, ent, sizeof(fq_entry) * size[0]);
        *nout = size[0];
        *dout = dec[0];
    }
    free(ent);
    free(size);
    free(dec);
    return rc;
}

/* report of a summary (entries e, D) over a stream of n items: the entries
 * with (count + D) * k > n, sorted by (count descending, item ascending),
 * moved to the front; returns their number */
uint32_t oracle_frequent_report(fq_entry* e, uint32_t count, uint64_t d, uint64_t n, uint32_t k) {
    qsort(e, count, sizeof(fq_entry), fq_count_desc);
    uint32_t w = 0;
    for (uint32_t i = 0; i < count; ++i)
        if ((unsigned __int128)(e[i].count + d) * k > n) e[w++] = e[i];
    return w;
}

int oracle_frequent_run(const uint32_t* items, uint64_t n, uint32_t k, uint32_t chunks, fq_entry* out,
                        uint32_t* nout) {
    uint32_t size = 0;
    uint64_t d = 0;
    int rc = oracle_frequent_summary(items, n, k, chunks, out, &size, &d);
    if (rc != 0) return rc;
    *nout = oracle_frequent_report(out, size, d, n, k);
    return 0;
}
