/*
 * CPU oracle for Parallel Space Saving -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded statement of what the GPU library must
 * compute, written from Cafaro, Pulimeno, Epicoco and Aloisio, "Parallel Space
 * Saving on Multi and Many-Core Processors" (arXiv 1606.04669).  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it; the
 * product path never does.  It shares no code, header or table with the GPU
 * library.  All arithmetic is integer (counts and errors are uint64).
 *
 * Readings of points the paper leaves open (each is also listed in the
 * design notes):
 *   R1  m of a summary with fewer than k monitored items is 0 (unused counters
 *       hold frequency 0); an empty summary is the identity of COMBINE.
 *   R2  When all k counters are used, the evicted counter is the one with the
 *       minimum estimated frequency and, among those, the smallest item id.
 *   R3  Error: a new item gets error 0; an eviction at minimum m installs the
 *       new item with count m+1 and error m.  COMBINE adds errors exactly as it
 *       adds counts (e1+e2, e1+m2, e2+m1).
 *   R4  Prune(k) keeps the first k candidates in the order (count descending,
 *       error ascending, item ascending); that order is also the output order.
 *   R5  The reduction is a fixed binary tree over chunk index: at every level
 *       summaries 2j and 2j+1 are combined (2j as S1) and an odd last summary
 *       is promoted unchanged.
 *   R6  Chunk c covers [floor(c*n/C), floor((c+1)*n/C)).
 *   R7  Reported items are those with count * k > n, i.e. count > floor(n/k).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint32_t item;
    uint32_t reserved;
    uint64_t count;
    uint64_t error;
} or_entry; /* same 24-byte layout as a host result entry */

/* ------------------------------------------------------------------------
 * Sequential Space Saving (Section 3, second paragraph; Metwally et al.).
 *
 * Counters live in arrays indexed 0..k-1.  Two plain helper structures:
 *  - a chained hash map item -> counter index (for "is x monitored?");
 *  - a binary min-heap of counter indices ordered by (count, item), whose
 *    root is the counter R2 evicts.
 * ---------------------------------------------------------------------- */

typedef struct {
    uint32_t k, size;
    uint32_t* item;
    uint64_t* count;
    uint64_t* error;
    /* hash map */
    uint32_t nbuckets; /* power of two */
    int32_t* head;     /* bucket -> first counter index or -1 */
    int32_t* next;     /* counter index -> next counter in chain or -1 */
    /* heap */
    uint32_t* heap;    /* heap[i] = counter index */
    uint32_t* where;   /* where[c] = position of counter c in heap */
} ss_state;

static uint32_t bucket_of(const ss_state* s, uint32_t x) {
    return (uint32_t)((x * 2654435761u) & (s->nbuckets - 1));
}

static int32_t map_find(const ss_state* s, uint32_t x) {
    for (int32_t c = s->head[bucket_of(s, x)]; c >= 0; c = s->next[c])
        if (s->item[c] == x) return c;
    return -1;
}

static void map_insert(ss_state* s, uint32_t c) {
    uint32_t b = bucket_of(s, s->item[c]);
    s->next[c] = s->head[b];
    s->head[b] = (int32_t)c;
}

static void map_remove(ss_state* s, uint32_t c) {
    uint32_t b = bucket_of(s, s->item[c]);
    int32_t* link = &s->head[b];
    while (*link != (int32_t)c) link = &s->next[*link];
    *link = s->next[c];
}

/* heap order: smaller count first, then smaller item id */
static int heap_less(const ss_state* s, uint32_t a, uint32_t b) {
    if (s->count[a] != s->count[b]) return s->count[a] < s->count[b];
    return s->item[a] < s->item[b];
}

static void heap_swap(ss_state* s, uint32_t i, uint32_t j) {
    uint32_t t = s->heap[i];
    s->heap[i] = s->heap[j];
    s->heap[j] = t;
    s->where[s->heap[i]] = i;
    s->where[s->heap[j]] = j;
}

static void sift_up(ss_state* s, uint32_t i) {
    while (i > 0) {
        uint32_t p = (i - 1) / 2;
        if (!heap_less(s, s->heap[i], s->heap[p])) break;
        heap_swap(s, i, p);
        i = p;
    }
}

static void sift_down(ss_state* s, uint32_t i) {
    for (;;) {
        uint32_t l = 2 * i + 1, r = l + 1, best = i;
        if (l < s->size && heap_less(s, s->heap[l], s->heap[best])) best = l;
        if (r < s->size && heap_less(s, s->heap[r], s->heap[best])) best = r;
        if (best == i) break;
        heap_swap(s, i, best);
        i = best;
    }
}

static int ss_init(ss_state* s, uint32_t k) {
    memset(s, 0, sizeof *s);
    s->k = k;
    s->nbuckets = 1;
    while (s->nbuckets < 2 * k) s->nbuckets <<= 1;
    s->item = malloc(sizeof(uint32_t) * k);
    s->count = malloc(sizeof(uint64_t) * k);
    s->error = malloc(sizeof(uint64_t) * k);
    s->head = malloc(sizeof(int32_t) * s->nbuckets);
    s->next = malloc(sizeof(int32_t) * k);
    s->heap = malloc(sizeof(uint32_t) * k);
    s->where = malloc(sizeof(uint32_t) * k);
    if (!s->item || !s->count || !s->error || !s->head || !s->next || !s->heap || !s->where) return -1;
    for (uint32_t b = 0; b < s->nbuckets; ++b) s->head[b] = -1;
    return 0;
}

static void ss_free(ss_state* s) {
    free(s->item); free(s->count); free(s->error);
    free(s->head); free(s->next); free(s->heap); free(s->where);
}

/* Process one item exactly as the sequential algorithm describes. */
static void ss_process(ss_state* s, uint32_t x) {
    int32_t c = map_find(s, x);
    if (c >= 0) { /* monitored: increment its estimated frequency */
        s->count[c] += 1;
        sift_down(s, s->where[c]);
        return;
    }
    if (s->size < s->k) { /* a free counter takes the item with frequency 1 */
        uint32_t f = s->size++;
        s->item[f] = x;
        s->count[f] = 1;
        s->error[f] = 0;
        map_insert(s, f);
        s->heap[f] = f;
        s->where[f] = f;
        sift_up(s, f);
        return;
    }
    /* all counters used: the minimum counter (R2) is incremented and its item
     * replaced by x; the old minimum becomes x's error bound (R3). */
    uint32_t v = s->heap[0];
    uint64_t m = s->count[v];
    map_remove(s, v);
    s->item[v] = x;
    s->count[v] = m + 1;
    s->error[v] = m;
    map_insert(s, v);
    sift_down(s, 0);
}

/* Space Saving over items[0, len) with k counters.
 * Writes up to k entries (unordered) to out, the number to *size and the
 * summary minimum (R1) to *m.  Returns 0, or -1 on allocation failure. */
int oracle_space_saving(const uint32_t* items, uint64_t len, uint32_t k, or_entry* out,
                        uint32_t* size, uint64_t* m) {
    if (k < 1) return -2;
    ss_state s;
    if (ss_init(&s, k) != 0) { ss_free(&s); return -1; }
    for (uint64_t i = 0; i < len; ++i) ss_process(&s, items[i]);
    for (uint32_t c = 0; c < s.size; ++c) {
        out[c].item = s.item[c];
        out[c].reserved = 0;
        out[c].count = s.count[c];
        out[c].error = s.error[c];
    }
    *size = s.size;
    *m = (s.size == k) ? s.count[s.heap[0]] : 0;
    ss_free(&s);
    return 0;
}

/* ------------------------------------------------------------------------
 * COMBINE (Algorithm 2) with Prune(k) under R1, R3 and R4.
 * ---------------------------------------------------------------------- */

/* R4 order: count descending, then error ascending, then item ascending */
static int key_cmp(const void* pa, const void* pb) {
    const or_entry* a = (const or_entry*)pa;
    const or_entry* b = (const or_entry*)pb;
    if (a->count != b->count) return a->count > b->count ? -1 : 1;
    if (a->error != b->error) return a->error < b->error ? -1 : 1;
    if (a->item != b->item) return a->item < b->item ? -1 : 1;
    return 0;
}

static int item_cmp(const void* pa, const void* pb) {
    uint32_t a = ((const or_entry*)pa)->item, b = ((const or_entry*)pb)->item;
    return a < b ? -1 : (a > b ? 1 : 0);
}

/* S_C = COMBINE(S1, S2).  m1, m2 are the two summaries' minima (R1).
 * out must hold k entries; the kept entries are written in R4 order.
 * Returns 0, or -1 on allocation failure. */
int oracle_combine(const or_entry* s1, uint32_t n1, uint64_t m1, const or_entry* s2, uint32_t n2,
                   uint64_t m2, uint32_t k, or_entry* out, uint32_t* nout, uint64_t* mout) {
    or_entry* cand = malloc(sizeof(or_entry) * ((size_t)n1 + n2 + 1));
    or_entry* s2s = malloc(sizeof(or_entry) * ((size_t)n2 + 1));
    char* taken = calloc((size_t)n2 + 1, 1);
    if (!cand || !s2s || !taken) { free(cand); free(s2s); free(taken); return -1; }
    memcpy(s2s, s2, sizeof(or_entry) * n2);
    qsort(s2s, n2, sizeof(or_entry), item_cmp); /* so that Find is a binary search */
    uint32_t nc = 0;
    /* first loop of Algorithm 2: every counter of S1 */
    for (uint32_t i = 0; i < n1; ++i) {
        or_entry key = s1[i];
        or_entry* hit = bsearch(&key, s2s, n2, sizeof(or_entry), item_cmp);
        or_entry e = s1[i];
        if (hit) {           /* item also in S2: add both estimates; remove from S2 */
            e.count = s1[i].count + hit->count;
            e.error = s1[i].error + hit->error;
            taken[hit - s2s] = 1;
        } else {             /* only in S1: S2's minimum bounds its missed occurrences */
            e.count = s1[i].count + m2;
            e.error = s1[i].error + m2;
        }
        e.reserved = 0;
        cand[nc++] = e;
    }
    /* second loop: counters of S2 not removed above */
    for (uint32_t j = 0; j < n2; ++j) {
        if (taken[j]) continue;
        or_entry e = s2s[j];
        e.count = s2s[j].count + m1;
        e.error = s2s[j].error + m1;
        e.reserved = 0;
        cand[nc++] = e;
    }
    /* Prune(k): keep the k candidates with the greatest frequencies (R4) */
    qsort(cand, nc, sizeof(or_entry), key_cmp);
    uint32_t keep = nc < k ? nc : k;
    memcpy(out, cand, sizeof(or_entry) * keep);
    *nout = keep;
    *mout = (keep == k) ? cand[keep - 1].count : 0;
    free(cand); free(s2s); free(taken);
    return 0;
}

/* ------------------------------------------------------------------------
 * Algorithm 1 with C chunks: partition (R6), Space Saving per chunk, fixed
 * binary COMBINE tree (R5).  Result: one summary of <= k entries (R4 order
 * when it came out of a COMBINE; chunk order otherwise).
 * ---------------------------------------------------------------------- */

uint64_t oracle_chunk_begin(uint64_t n, uint32_t chunks, uint32_t c) {
    return (uint64_t)(((unsigned __int128)c * n) / chunks);
}

/* Reduce `count` summaries stored at stride k in ent/size/mins, in place, by
 * the fixed tree.  On return summary 0 holds the result. */
int oracle_tree(or_entry* ent, uint32_t* size, uint64_t* mins, uint32_t count, uint32_t k) {
    or_entry* tmp = malloc(sizeof(or_entry) * (size_t)k);
    if (!tmp) return -1;
    uint32_t live = count;
    while (live > 1) {
        uint32_t half = live / 2;
        for (uint32_t j = 0; j < half; ++j) {
            uint32_t a = 2 * j, b = 2 * j + 1, nout;
            uint64_t mout;
            if (oracle_combine(ent + (size_t)a * k, size[a], mins[a], ent + (size_t)b * k, size[b],
                               mins[b], k, tmp, &nout, &mout) != 0) {
                free(tmp);
                return -1;
            }
            memcpy(ent + (size_t)j * k, tmp, sizeof(or_entry) * nout);
            size[j] = nout;
            mins[j] = mout;
        }
        if (live & 1) { /* odd last summary is promoted unchanged */
            uint32_t a = live - 1, j = half;
            memmove(ent + (size_t)j * k, ent + (size_t)a * k, sizeof(or_entry) * size[a]);
            size[j] = size[a];
            mins[j] = mins[a];
        }
        live = half + (live & 1);
    }
    free(tmp);
    return 0;
}

/* Summary of items[0,n) with k counters over C chunks (no pruning by
 * threshold).  out holds k entries.  Returns 0 or a negative error. */
int oracle_summary(const uint32_t* items, uint64_t n, uint32_t k, uint32_t chunks, or_entry* out,
                   uint32_t* nout, uint64_t* mout) {
    if (k < 1 || chunks < 1) return -2;
    or_entry* ent = malloc(sizeof(or_entry) * (size_t)k * chunks);
    uint32_t* size = malloc(sizeof(uint32_t) * chunks);
    uint64_t* mins = malloc(sizeof(uint64_t) * chunks);
    if (!ent || !size || !mins) { free(ent); free(size); free(mins); return -1; }
    for (uint32_t c = 0; c < chunks; ++c) {
        uint64_t lo = oracle_chunk_begin(n, chunks, c), hi = oracle_chunk_begin(n, chunks, c + 1);
        if (oracle_space_saving(items + lo, hi - lo, k, ent + (size_t)c * k, &size[c], &mins[c]) != 0) {
            free(ent); free(size); free(mins);
            return -1;
        }
    }
    int rc = oracle_tree(ent, size, mins, chunks, k);
    if (rc == 0) {
        memcpy(out, ent, sizeof(or_entry) * size[0]);
        *nout = size[0];
        *mout = mins[0];
    }
    free(ent); free(size); free(mins);
    return rc;
}

/* Sort a summary's entries into the R4 order (in place). */
void oracle_sort_canonical(or_entry* e, uint32_t count) {
    qsort(e, count, sizeof(or_entry), key_cmp);
}

/* Pruned(global, n, k): entries with count > floor(n/k), R4 order.
 * Entries are sorted in place; returns how many qualify (a prefix). */
uint32_t oracle_prune_threshold(or_entry* e, uint32_t count, uint64_t n, uint32_t k) {
    qsort(e, count, sizeof(or_entry), key_cmp);
    uint64_t thr = n / k;
    uint32_t q = 0;
    while (q < count && e[q].count > thr) ++q;
    return q;
}

/* ParallelSpaceSaving(A, n, p=C, k): the k-majority candidates of items[0,n).
 * out must hold k entries; *nout = number reported.  Precondition of the
 * problem statement: 2 <= k <= n (returns -3 otherwise). */
int oracle_run(const uint32_t* items, uint64_t n, uint32_t k, uint32_t chunks, or_entry* out,
               uint32_t* nout) {
    if (k < 2 || (uint64_t)k > n) return -3;
    uint32_t size;
    uint64_t m;
    int rc = oracle_summary(items, n, k, chunks, out, &size, &m);
    if (rc != 0) return rc;
    *nout = oracle_prune_threshold(out, size, n, k);
    return 0;
}
