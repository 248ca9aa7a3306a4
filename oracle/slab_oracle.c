/*
 * CPU oracle for the slab hash -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the package's smoke check and the benchmark's CPU-baseline leg may load
 * this code. It shares nothing with the GPU library: no headers, no helpers, no constants
 * generators. It is a plain, sequential, obviously-correct chained hash map with the semantics
 * of "A Dynamic Hash Table for the GPU" (Ashkiani, Farach-Colton, Owens):
 *
 *   - B buckets, each the head of a list of slabs holding M elements each and one shared next
 *     pointer (Design description: "Slab list"; "Slab Hash: A Dynamic Hash Table").
 *   - bucket of key k: h(k; a, b) = ((a k + b) mod p) mod B, the universal hash stated in the
 *     "Slab Hash" subsection. Here p = 4294967291 (the largest prime below 2^32) and a, b are
 *     passed in by the caller.
 *   - REPLACE(k, v): look through the whole list for k; if present overwrite its value, else
 *     insert at the first empty spot from the head, appending a slab when the tail is full
 *     ("Supported Operations": REPLACE; "Insertion" subsection).
 *   - DELETE(k): mark the matching element as deleted; a deleted spot is never treated as empty
 *     when keys are unique, so it is not reused ("Deletion" subsection and its footnote).
 *     Not found is a no-op.
 *   - SEARCH(k): return the value of the live element with key k, or not-found ("Search").
 *
 * With duplicates allowed (om_set_duplicates; "Supported Operations": the multiset variants):
 *   - INSERT(k, v): put (k, v) in the first empty spot from the head, with no uniqueness check
 *     ("Insertion": INSERT), appending a slab when no spot is empty.
 *   - DELETE(k): the first live element with key k from the head becomes an empty spot, which a
 *     later INSERT may fill ("Deletion": with duplicates a deleted element is marked empty).
 *   - SEARCH(k): the first live element with key k from the head.
 *   - DELETEALL(k) / SEARCHALL(k): every live element with key k, in list order, in both modes.
 *
 * A bucket's spots are kept here as one array in list order (deleted spots keep their place;
 * with duplicates allowed, emptied spots stay in the array until INSERT fills them); slab j of
 * the list holds array entries [jM, (j+1)M). Slabs per bucket = max(1, ceil(occupied / M)), the base slab always existing.
 * Memory utilisation follows the formula of the "Slab Hash" subsection:
 *   u = x / (M x + y) * n / sum_i k_i,  x = element bytes, y = pointer (and aux) bytes.
 *
 * The key 0xFFFFFFFF is reserved (the empty marker); an operation carrying it fails with
 * status 0 and raises OM_ERR_RESERVED. With a finite pool, an insert that would need a new slab
 * when all pool slabs are in use fails with status 0 and raises OM_ERR_NOMEM.
 *
 * Per-op status: replace 1 = new key, 2 = replaced, 0 = failed; delete 1 = deleted, 0 = absent;
 * search 1 = found, 0 = not found (value 0xFFFFFFFF).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OM_PRIME 4294967291ull
#define OM_RESERVED 0xFFFFFFFFu
#define OM_ERR_RESERVED 1u
#define OM_ERR_NOMEM 2u

enum { OM_DELETED = 0, OM_LIVE = 1, OM_HOLE = 2 };

typedef struct {
    uint32_t key;
    uint32_t val;
    uint32_t live; /* OM_LIVE, OM_DELETED (kept, never reused) or OM_HOLE (empty, reusable) */
} om_slot;

typedef struct {
    om_slot *s;
    uint32_t n;   /* spots in use or once used: live, deleted and holes */
    uint32_t cap;
} om_bucket;

typedef struct {
    uint32_t B, M;
    uint64_t a, b;
    uint64_t pool_cap;  /* slabs available beyond the base slabs; UINT64_MAX = unbounded */
    uint64_t pool_used; /* slabs in use beyond the base slabs */
    uint32_t err;
    uint32_t dup; /* 1 = duplicates allowed (multiset operations) */
    om_bucket *bk;
} om_table;

/* Universal hash of the "Slab Hash" subsection, evaluated exactly in 64-bit integers:
   a < p and k < 2^32 so a*k + b < 2^64. */
uint32_t om_bucket_of(const om_table *t, uint32_t k)
{
    uint64_t x = t->a * (uint64_t)k + t->b;
    return (uint32_t)((x % OM_PRIME) % (uint64_t)t->B);
}

om_table *om_create(uint32_t B, uint32_t M, uint64_t a, uint64_t b, uint64_t pool_cap)
{
    if (B == 0 || M == 0 || a == 0 || a >= OM_PRIME || b >= OM_PRIME)
        return NULL;
    om_table *t = (om_table *)calloc(1, sizeof(om_table));
    if (!t)
        return NULL;
    t->B = B;
    t->M = M;
    t->a = a;
    t->b = b;
    t->pool_cap = pool_cap;
    t->bk = (om_bucket *)calloc(B, sizeof(om_bucket));
    if (!t->bk) {
        free(t);
        return NULL;
    }
    return t;
}

void om_destroy(om_table *t)
{
    if (!t)
        return;
    for (uint32_t i = 0; i < t->B; i++)
        free(t->bk[i].s);
    free(t->bk);
    free(t);
}

uint32_t om_error(const om_table *t) { return t->err; }

/* Choose the operation set before any operation: 0 = unique keys (REPLACE, deleted spots kept),
   1 = duplicates allowed (INSERT, deleted spots become empty). */
void om_set_duplicates(om_table *t, uint32_t on) { t->dup = on ? 1u : 0u; }

static uint32_t slabs_for(uint32_t occ, uint32_t M)
{
    return occ == 0 ? 1u : (occ + M - 1) / M;
}

/* Index of the live element with key k in bucket bk, or -1. Scans the list from its head. */
static int64_t find_live(const om_bucket *bk, uint32_t k)
{
    for (uint32_t i = 0; i < bk->n; i++)
        if (bk->s[i].live == OM_LIVE && bk->s[i].key == k)
            return (int64_t)i;
    return -1;
}

static int append(om_table *t, om_bucket *bk, uint32_t k, uint32_t v);

/* REPLACE(k, v). */
int om_replace(om_table *t, uint32_t k, uint32_t v)
{
    if (k == OM_RESERVED) {
        t->err |= OM_ERR_RESERVED;
        return 0;
    }
    om_bucket *bk = &t->bk[om_bucket_of(t, k)];
    int64_t i = find_live(bk, k);
    if (i >= 0) {
        bk->s[i].val = v;
        return 2;
    }
    return append(t, bk, k, v);
}

/* INSERT(k, v) with duplicates allowed: the first empty spot from the head, else the tail. */
int om_insert(om_table *t, uint32_t k, uint32_t v)
{
    if (k == OM_RESERVED) {
        t->err |= OM_ERR_RESERVED;
        return 0;
    }
    om_bucket *bk = &t->bk[om_bucket_of(t, k)];
    for (uint32_t i = 0; i < bk->n; i++)
        if (bk->s[i].live == OM_HOLE) {
            bk->s[i].key = k;
            bk->s[i].val = v;
            bk->s[i].live = OM_LIVE;
            return 1;
        }
    return append(t, bk, k, v);
}

/* Put (k, v) in the spot after the last used one. */
static int append(om_table *t, om_bucket *bk, uint32_t k, uint32_t v)
{
    /* Not present: the first empty spot is the next one in insertion order. When every spot of
       the list's slabs is occupied (the tail slab is full) a new slab is linked at the tail. */
    if (bk->n > 0 && bk->n % t->M == 0) {
        if (t->pool_used >= t->pool_cap) {
            t->err |= OM_ERR_NOMEM;
            return 0;
        }
        t->pool_used++;
    }
    if (bk->n == bk->cap) {
        uint32_t nc = bk->cap ? bk->cap * 2 : 8;
        om_slot *ns = (om_slot *)realloc(bk->s, (size_t)nc * sizeof(om_slot));
        if (!ns)
            abort();
        bk->s = ns;
        bk->cap = nc;
    }
    bk->s[bk->n].key = k;
    bk->s[bk->n].val = v;
    bk->s[bk->n].live = OM_LIVE;
    bk->n++;
    return 1;
}

/* DELETE(k): mark as deleted; the spot stays occupied (unique keys) or becomes empty
   (duplicates allowed). */
int om_delete(om_table *t, uint32_t k)
{
    if (k == OM_RESERVED) {
        t->err |= OM_ERR_RESERVED;
        return 0;
    }
    om_bucket *bk = &t->bk[om_bucket_of(t, k)];
    int64_t i = find_live(bk, k);
    if (i < 0)
        return 0;
    bk->s[i].live = t->dup ? OM_HOLE : OM_DELETED;
    return 1;
}

/* DELETEALL(k): every live element with key k, as DELETE does each. Returns how many. */
uint32_t om_delete_all(om_table *t, uint32_t k)
{
    if (k == OM_RESERVED) {
        t->err |= OM_ERR_RESERVED;
        return 0;
    }
    om_bucket *bk = &t->bk[om_bucket_of(t, k)];
    uint32_t c = 0;
    for (uint32_t i = 0; i < bk->n; i++)
        if (bk->s[i].live == OM_LIVE && bk->s[i].key == k) {
            bk->s[i].live = t->dup ? OM_HOLE : OM_DELETED;
            c++;
        }
    return c;
}

/* SEARCHALL(k): the values of every live element with key k, in list order. Returns how many
   there are (writes at most cap). */
uint32_t om_search_all(const om_table *t, uint32_t k, uint32_t *vals, uint32_t cap)
{
    if (k == OM_RESERVED) {
        ((om_table *)t)->err |= OM_ERR_RESERVED;
        return 0;
    }
    const om_bucket *bk = &t->bk[om_bucket_of(t, k)];
    uint32_t c = 0;
    for (uint32_t i = 0; i < bk->n; i++)
        if (bk->s[i].live == OM_LIVE && bk->s[i].key == k) {
            if (c < cap)
                vals[c] = bk->s[i].val;
            c++;
        }
    return c;
}

/* SEARCH(k). *slabs_visited (if not NULL) receives the number of slabs a head-to-tail walk
   reads: the slab holding the element, or every slab of the list on a miss. */
int om_search(const om_table *t, uint32_t k, uint32_t *val, uint32_t *slabs_visited)
{
    if (k == OM_RESERVED) {
        ((om_table *)t)->err |= OM_ERR_RESERVED;
        *val = OM_RESERVED;
        if (slabs_visited)
            *slabs_visited = 0;
        return 0;
    }
    const om_bucket *bk = &t->bk[om_bucket_of(t, k)];
    int64_t i = find_live(bk, k);
    if (i < 0) {
        *val = OM_RESERVED;
        if (slabs_visited)
            *slabs_visited = slabs_for(bk->n, t->M);
        return 0;
    }
    *val = bk->s[i].val;
    if (slabs_visited)
        *slabs_visited = (uint32_t)(i / t->M) + 1;
    return 1;
}

/* FLUSH of buckets first .. first + count - 1 (those below B): drop deleted elements and
   release the slabs no longer needed ("Flush" subsection). Live elements keep their relative
   order. */
void om_flush_buckets(om_table *t, uint32_t first, uint32_t count)
{
    for (uint64_t i = first; i < (uint64_t)first + count && i < t->B; i++) {
        om_bucket *bk = &t->bk[i];
        uint32_t before = slabs_for(bk->n, t->M), w = 0;
        for (uint32_t r = 0; r < bk->n; r++)
            if (bk->s[r].live == OM_LIVE)
                bk->s[w++] = bk->s[r];
        bk->n = w;
        t->pool_used -= before - slabs_for(bk->n, t->M);
    }
}

/* FLUSH of every bucket. */
void om_flush_all(om_table *t)
{
    om_flush_buckets(t, 0, t->B);
}

/* ---- batched drivers: apply ops one after another in array order ---- */

/* REPLACE (INSERT with duplicates allowed) of each pair in order. */
void om_replace_batch(om_table *t, const uint32_t *keys, const uint32_t *vals, uint64_t n,
                      uint8_t *status)
{
    for (uint64_t i = 0; i < n; i++) {
        int s = t->dup ? om_insert(t, keys[i], vals[i]) : om_replace(t, keys[i], vals[i]);
        if (status)
            status[i] = (uint8_t)s;
    }
}

void om_delete_batch(om_table *t, const uint32_t *keys, uint64_t n, uint8_t *status)
{
    for (uint64_t i = 0; i < n; i++) {
        int s = om_delete(t, keys[i]);
        if (status)
            status[i] = (uint8_t)s;
    }
}

void om_search_batch(const om_table *t, const uint32_t *keys, uint64_t n, uint32_t *vals,
                     uint8_t *found, uint32_t *visits)
{
    for (uint64_t i = 0; i < n; i++) {
        uint32_t v, sv;
        int f = om_search(t, keys[i], &v, &sv);
        vals[i] = v;
        if (found)
            found[i] = (uint8_t)f;
        if (visits)
            visits[i] = sv;
    }
}

/* ops: 0 = search, 1 = replace (INSERT with duplicates allowed), 2 = delete. vals_out gets the search result (0xFFFFFFFF for
   non-search ops and misses); status gets found / replace / delete status. */
void om_mixed_batch(om_table *t, const uint8_t *ops, const uint32_t *keys,
                    const uint32_t *vals_in, uint64_t n, uint32_t *vals_out, uint8_t *status)
{
    for (uint64_t i = 0; i < n; i++) {
        uint32_t v = OM_RESERVED;
        int s;
        switch (ops[i]) {
        case 0:
            s = om_search(t, keys[i], &v, NULL);
            break;
        case 1:
            s = t->dup ? om_insert(t, keys[i], vals_in[i]) : om_replace(t, keys[i], vals_in[i]);
            break;
        case 2:
            s = om_delete(t, keys[i]);
            break;
        default:
            s = 0;
            break;
        }
        vals_out[i] = v;
        status[i] = (uint8_t)s;
    }
}

/* ---- structure accounting ---- */

/* Per-bucket live, deleted and slab counts (arrays of length B, any may be NULL); empty spots
   left by deletions with duplicates allowed count as neither. Returns the total live count. */
uint64_t om_bucket_stats(const om_table *t, uint32_t *live, uint32_t *tomb, uint32_t *slabs)
{
    uint64_t total = 0;
    for (uint32_t i = 0; i < t->B; i++) {
        const om_bucket *bk = &t->bk[i];
        uint32_t l = 0, d = 0;
        for (uint32_t r = 0; r < bk->n; r++) {
            l += bk->s[r].live == OM_LIVE;
            d += bk->s[r].live == OM_DELETED;
        }
        total += l;
        if (live)
            live[i] = l;
        if (tomb)
            tomb[i] = d;
        if (slabs)
            slabs[i] = slabs_for(bk->n, t->M);
    }
    return total;
}

uint64_t om_total_slabs(const om_table *t)
{
    uint64_t s = 0;
    for (uint32_t i = 0; i < t->B; i++)
        s += slabs_for(t->bk[i].n, t->M);
    return s;
}

uint64_t om_pool_used(const om_table *t) { return t->pool_used; }

/* Memory utilisation with element size x bytes and per-slab overhead y bytes. */
double om_utilisation(const om_table *t, double x, double y)
{
    uint64_t live = om_bucket_stats(t, NULL, NULL, NULL);
    uint64_t slabs = om_total_slabs(t);
    return (x / ((double)t->M * x + y)) * ((double)live / (double)slabs);
}

/* Live (bucket, key, value) triples, bucket-major then insertion order. Returns the count
   (writes at most cap). */
uint64_t om_dump(const om_table *t, uint32_t *bucket, uint32_t *key, uint32_t *val,
                 uint64_t cap)
{
    uint64_t c = 0;
    for (uint32_t i = 0; i < t->B; i++) {
        const om_bucket *bk = &t->bk[i];
        for (uint32_t r = 0; r < bk->n; r++) {
            if (bk->s[r].live != OM_LIVE)
                continue;
            if (c < cap) {
                bucket[c] = i;
                key[c] = bk->s[r].key;
                val[c] = bk->s[r].val;
            }
            c++;
        }
    }
    return c;
}

void om_delete_all_batch(om_table *t, const uint32_t *keys, uint64_t n, uint32_t *counts)
{
    for (uint64_t i = 0; i < n; i++)
        counts[i] = om_delete_all(t, keys[i]);
}

/* SEARCHALL of each key in order: counts[i] values of query i go to vals[offsets[i] ...] when
   vals is not NULL (offsets from a previous counting call). */
void om_search_all_batch(const om_table *t, const uint32_t *keys, uint64_t n, uint32_t *counts,
                         const uint64_t *offsets, uint32_t *vals)
{
    for (uint64_t i = 0; i < n; i++)
        counts[i] = om_search_all(t, keys[i], vals ? vals + offsets[i] : NULL,
                                  vals ? 0xFFFFFFFFu : 0u);
}

void om_bucket_of_batch(const om_table *t, const uint32_t *keys, uint64_t n, uint32_t *out)
{
    for (uint64_t i = 0; i < n; i++)
        out[i] = om_bucket_of(t, keys[i]);
}
