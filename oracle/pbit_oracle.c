/*
 * Pbit oracle: a plain, sequential, deliberately slow CPU implementation of
 * the Pbit list sort (Planeta, "Pbit and other list sorting algorithms",
 * arXiv cs/0511020).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the HIP
 * path.
 *
 * What is computed (paper Sec. 3 "The idea of sorting using Pbit", Sec. 5
 * "Implementation in C++", Sec. 6 "Differences between sorting in descending
 * and ascending order"):
 *   - the list starting at `head` is split by the K-bit pattern taken at the
 *     top of the not-yet-examined bits (bit offset m after m := m - K, digit
 *     (key >> m) & (Omega - 1), Sec. 4 "Cutting bits off");
 *   - each non-empty group is split again on the next K bits (recursion, Sec. 5
 *     item 8), empty groups are skipped (Sec. 3, "empty lists are omitted");
 *   - once all M bits are consumed, each final group is concatenated in front
 *     of the already-sorted tail P by walking it to its end (the merge of
 *     Sec. 5.1), groups taken from the highest pattern to the lowest for
 *     ascending order and the other way round for descending order (Sec. 6).
 *
 * Readings taken where the paper is silent or contradicts itself:
 *   - groups are first-in-first-out lists (a head and a tail per group, the
 *     "first group" of roots in Sec. 5.1), so that equal keys keep their list
 *     order for every M/K.  The printed listings push each node on the front
 *     of its group, which reverses equal keys once per level; that behaviour
 *     is kept behind ORACLE_FLAG_LIFO so tests can show the difference.
 *   - signed keys (Sec. 7-8): the list is split into negative and
 *     non-negative keys keeping list order, each part is sorted as unsigned
 *     and the parts are concatenated (negatives first when ascending).
 *   - floating-point keys (Sec. 14): the stored M bits are an IEEE-754 style
 *     sign-magnitude number (sign, then characteristic, then mantissa).  The
 *     paper sorts on the mantissa first and then, stably, on the
 *     characteristic; for non-negative numbers that is one sort on the whole
 *     bit pattern, done here.  The paper does not treat negative numbers: they
 *     are split off by the sign bit as in Sec. 8, and since a larger
 *     magnitude means a smaller value, the negative part is sorted on its
 *     pattern in the opposite direction before the parts are joined.  So -0
 *     comes before +0, and NaNs go to the ends by their sign bit.
 *   - M is the storage width of a key in bits (8, 16, 32 or 64); K must
 *     divide M.  An empty list returns NIL and writes nothing.
 *
 * Extra memory is O(Omega * M/K) group roots (Sec. 3, the bound T), never
 * proportional to n.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define ORACLE_NIL 0xFFFFFFFFu

enum {
    ORACLE_OK = 0,
    ORACLE_EINVAL = -1,
    ORACLE_EMALFORMED = -2,
    ORACLE_ENOMEM = -3
};

enum {
    ORACLE_FLAG_LIFO = 1,       /* push-front groups, as in the printed listings */
    ORACLE_FLAG_DESCENDING = 2, /* Sec. 6: largest key first                      */
    ORACLE_FLAG_SIGNED = 4,     /* Sec. 7-8: two's-complement keys               */
    ORACLE_FLAG_FLOAT = 8       /* Sec. 14: sign-magnitude floating-point keys   */
};

typedef struct {
    uint32_t *next;
    const void *keys;
    uint32_t width;   /* M, bits per stored key */
    uint32_t K;       /* bits per pattern       */
    uint32_t omega;   /* 2^K groups             */
    int lifo;
    int descending;
    uint32_t *roots;  /* (M/K) levels x 2 x omega slots: heads then tails */
    uint64_t merge_steps;
    uint64_t split_visits;
    uint64_t calls;
    uint32_t depth;
    uint32_t max_depth;
} pbit_oracle_ctx;

/* Key of node i widened to 64 bits (the value, never its bytes: Sec. 15). */
static uint64_t oracle_key(const pbit_oracle_ctx *c, uint32_t i)
{
    switch (c->width) {
    case 8: return ((const uint8_t *)c->keys)[i];
    case 16: return ((const uint16_t *)c->keys)[i];
    case 32: return ((const uint32_t *)c->keys)[i];
    default: return ((const uint64_t *)c->keys)[i];
    }
}

/* The merge of Sec. 5.1: walk A to its last node, hang B behind it, return A.
 * Every node walked is counted; over a whole sort the count equals n. */
static uint32_t oracle_merge(pbit_oracle_ctx *c, uint32_t A, uint32_t B)
{
    if (A == ORACLE_NIL)
        return B;
    uint32_t t = A;
    c->merge_steps++;
    while (c->next[t] != ORACLE_NIL) {
        t = c->next[t];
        c->merge_steps++;
    }
    c->next[t] = B;
    return A;
}

/* Sort the NIL-terminated sub-list L on the bits below offset m and return it
 * followed by the already sorted list P (Sec. 5, with the direction of Sec. 6). */
static uint32_t oracle_pbit(pbit_oracle_ctx *c, uint32_t L, uint32_t m, uint32_t P)
{
    if (L == ORACLE_NIL)
        return P;
    c->calls++;
    m -= c->K;
    uint32_t level = c->depth;
    c->depth++;
    if (c->depth > c->max_depth)
        c->max_depth = c->depth;

    uint32_t *head = c->roots + (size_t)level * 2u * c->omega;
    uint32_t *tail = head + c->omega;
    for (uint32_t g = 0; g < c->omega; g++)
        head[g] = tail[g] = ORACLE_NIL;

    /* Split: each node goes to the group named by its pattern at offset m. */
    uint32_t i = L;
    while (i != ORACLE_NIL) {
        uint32_t following = c->next[i];
        uint32_t g = (uint32_t)((oracle_key(c, i) >> m) & (uint64_t)(c->omega - 1u));
        c->split_visits++;
        if (c->lifo) {
            c->next[i] = head[g];
            head[g] = i;
        } else {
            c->next[i] = ORACLE_NIL;
            if (head[g] == ORACLE_NIL)
                head[g] = i;
            else
                c->next[tail[g]] = i;
            tail[g] = i;
        }
        i = following;
    }

    /* Groups are prepended to P, so the group that must come last is handled
     * first: the highest pattern for ascending order, the lowest for descending. */
    for (uint32_t s = 0; s < c->omega; s++) {
        uint32_t g = c->descending ? s : (c->omega - 1u - s);
        if (m > 0)
            P = oracle_pbit(c, head[g], m, P);
        else
            P = oracle_merge(c, head[g], P);
    }
    c->depth--;
    return P;
}

static int oracle_valid_shape(uint32_t M, uint32_t K)
{
    if (M != 8 && M != 16 && M != 32 && M != 64)
        return 0;
    if (K == 0 || K > 16 || K > M || (M % K) != 0)
        return 0;
    return 1;
}

/* Walk from head: the list must hold exactly n nodes, every index below n,
 * and end in NIL.  Nothing is written. */
static int oracle_walk_check(uint32_t head, const uint32_t *next, uint64_t n,
                             uint32_t lo, uint32_t hi)
{
    uint64_t steps = 0;
    uint32_t i = head;
    while (i != ORACLE_NIL) {
        if (i < lo || i >= hi)
            return ORACLE_EMALFORMED;
        if (++steps > n)
            return ORACLE_EMALFORMED; /* cycle */
        i = next[i];
    }
    return steps == n ? ORACLE_OK : ORACLE_EMALFORMED;
}

/*
 * Sort the list (head, next[0..n)) by keys[0..n) of M bits, K bits per
 * pattern.  next[] is relinked in place.  Returns the new head (NIL for an
 * empty list) or a negative status.  counters, when not NULL, receives
 * {merge steps, split visits, recursive calls, deepest level}.
 */
int64_t pbit_oracle_sort(uint32_t head, uint32_t *next, const void *keys, uint64_t n,
                         uint32_t M, uint32_t K, uint32_t flags, uint64_t *counters)
{
    if (counters)
        memset(counters, 0, 4 * sizeof(uint64_t));
    if (!oracle_valid_shape(M, K))
        return ORACLE_EINVAL;
    if (n >= (uint64_t)ORACLE_NIL)
        return ORACLE_EINVAL;
    if (n == 0 || head == ORACLE_NIL)
        return (n == 0 && head == ORACLE_NIL) ? (int64_t)ORACLE_NIL : ORACLE_EINVAL;
    if (!next || !keys || head >= n)
        return ORACLE_EINVAL;
    int st = oracle_walk_check(head, next, n, 0, (uint32_t)n);
    if (st != ORACLE_OK)
        return st;

    pbit_oracle_ctx c;
    memset(&c, 0, sizeof c);
    c.next = next;
    c.keys = keys;
    c.width = M;
    c.K = K;
    c.omega = 1u << K;
    c.lifo = (flags & ORACLE_FLAG_LIFO) != 0;
    c.descending = (flags & ORACLE_FLAG_DESCENDING) != 0;
    c.roots = (uint32_t *)malloc((size_t)(M / K) * 2u * c.omega * sizeof(uint32_t));
    if (!c.roots)
        return ORACLE_ENOMEM;

    uint32_t P;
    if ((flags & ORACLE_FLAG_SIGNED) && (flags & ORACLE_FLAG_FLOAT)) {
        free(c.roots);
        return ORACLE_EINVAL;
    }
    if (flags & (ORACLE_FLAG_SIGNED | ORACLE_FLAG_FLOAT)) {
        /* Sec. 8: split by sign (list order kept), sort each part unsigned,
         * then join: negatives before non-negatives when ascending. */
        uint32_t nh = ORACLE_NIL, nt = ORACLE_NIL, ph = ORACLE_NIL, pt = ORACLE_NIL;
        uint32_t i = head;
        while (i != ORACLE_NIL) {
            uint32_t following = next[i];
            int negative = (int)((oracle_key(&c, i) >> (M - 1u)) & 1u);
            next[i] = ORACLE_NIL;
            if (negative) {
                if (nh == ORACLE_NIL) nh = i; else next[nt] = i;
                nt = i;
            } else {
                if (ph == ORACLE_NIL) ph = i; else next[pt] = i;
                pt = i;
            }
            i = following;
        }
        /* A negative float's pattern grows with its magnitude, so its part
         * runs in the direction opposite to the requested one. */
        int flip = (flags & ORACLE_FLAG_FLOAT) != 0;
        int desc = c.descending;
        if (!desc) {
            c.descending = 0;
            P = oracle_pbit(&c, ph, M, ORACLE_NIL);
            c.descending = flip;
            P = oracle_pbit(&c, nh, M, P);
        } else {
            c.descending = !flip;
            P = oracle_pbit(&c, nh, M, ORACLE_NIL);
            c.descending = 1;
            P = oracle_pbit(&c, ph, M, P);
        }
    } else {
        P = oracle_pbit(&c, head, M, ORACLE_NIL);
    }
    free(c.roots);
    if (counters) {
        counters[0] = c.merge_steps;
        counters[1] = c.split_visits;
        counters[2] = c.calls;
        counters[3] = c.max_depth;
    }
    return (int64_t)P;
}

/*
 * Many independent lists sharing next[] and keys[]: list l owns the node slab
 * [offsets[l], offsets[l+1]) and its next[] entries are global indices inside
 * that slab.  Each list is checked and sorted on its own.  new_heads[l]
 * receives the sorted head (NIL for an empty slab).  Returns 0 or the first
 * negative status (lists before it are already sorted).
 */
int pbit_oracle_sort_lists(const uint32_t *heads, const uint64_t *offsets, uint32_t num_lists,
                           uint32_t *next, const void *keys, uint32_t M, uint32_t K,
                           uint32_t flags, uint32_t *new_heads)
{
    if (!oracle_valid_shape(M, K) || !heads || !offsets || !new_heads)
        return ORACLE_EINVAL;
    for (uint32_t l = 0; l < num_lists; l++) {
        uint64_t lo = offsets[l], hi = offsets[l + 1];
        if (hi < lo || hi >= (uint64_t)ORACLE_NIL)
            return ORACLE_EINVAL;
        uint64_t len = hi - lo;
        if (len == 0) {
            if (heads[l] != ORACLE_NIL)
                return ORACLE_EINVAL;
            new_heads[l] = ORACLE_NIL;
            continue;
        }
        if (heads[l] < lo || heads[l] >= hi)
            return ORACLE_EINVAL;
        int st = oracle_walk_check(heads[l], next, len, (uint32_t)lo, (uint32_t)hi);
        if (st != ORACLE_OK)
            return st;
        /* Sort the slab as a list of its own: shift indices to slab-local. */
        uint32_t *local = (uint32_t *)malloc((size_t)len * sizeof(uint32_t));
        if (!local)
            return ORACLE_ENOMEM;
        for (uint64_t j = 0; j < len; j++)
            local[j] = next[lo + j] == ORACLE_NIL ? ORACLE_NIL : next[lo + j] - (uint32_t)lo;
        const char *kbase = (const char *)keys + (size_t)lo * (M / 8u);
        int64_t h = pbit_oracle_sort(heads[l] - (uint32_t)lo, local, kbase, len, M, K, flags, NULL);
        if (h < 0) {
            free(local);
            return (int)h;
        }
        for (uint64_t j = 0; j < len; j++)
            next[lo + j] = local[j] == ORACLE_NIL ? ORACLE_NIL : local[j] + (uint32_t)lo;
        new_heads[l] = (uint32_t)h + (uint32_t)lo;
        free(local);
    }
    return ORACLE_OK;
}

/* List order: order[t] = the t-th node met walking from head (the positions a
 * parallel ranking must reproduce).  Returns the number of nodes or a
 * negative status. */
int64_t pbit_oracle_list_order(uint32_t head, const uint32_t *next, uint64_t n, uint32_t *order)
{
    if (n == 0 || head == ORACLE_NIL)
        return 0;
    if (head >= n)
        return ORACLE_EINVAL;
    int st = oracle_walk_check(head, next, n, 0, (uint32_t)n);
    if (st != ORACLE_OK)
        return st;
    uint64_t t = 0;
    for (uint32_t i = head; i != ORACLE_NIL; i = next[i])
        order[t++] = i;
    return (int64_t)t;
}

/* Sec. 13, doubly-linked lists: the sort relinks only next[]; afterwards a
 * repair walks the list from its head and points each node's backward link at
 * the node met just before it (NIL for the head).  prev[] entries of nodes not
 * on the list are left alone.  Returns the number of nodes walked or a
 * negative status (nothing is written then). */
int64_t pbit_oracle_repair_prev(uint32_t head, const uint32_t *next, uint64_t n, uint32_t *prev)
{
    if (head == ORACLE_NIL)
        return 0;
    if (n == 0 || head >= n)
        return ORACLE_EINVAL;
    uint64_t steps = 0;
    for (uint32_t i = head; i != ORACLE_NIL; i = next[i]) {
        if (i >= n || ++steps > n)
            return ORACLE_EMALFORMED;
    }
    uint32_t behind = ORACLE_NIL;
    for (uint32_t i = head; i != ORACLE_NIL; i = next[i]) {
        prev[i] = behind;
        behind = i;
    }
    return (int64_t)steps;
}

/*
 * The same sort on several host threads (a CPU baseline, not a pin).  The top
 * levels of the recursion run as in pbit_oracle_sort: the list is split into
 * first-in-first-out groups on the top pattern, and, while fewer than 256
 * groups exist and bits remain, each group again on the next pattern.  The
 * groups are independent sub-lists (Sec. 3), so each is sorted by the
 * recursion of Sec. 5 on its own thread, which then walks its result to the
 * end (the walk of the merge of Sec. 5.1) so that the groups can be joined in
 * pattern order without a second walk.  Unsigned keys only; flags 0 or
 * ORACLE_FLAG_DESCENDING.  threads = 0 uses every online core.  Returns the
 * new head or a negative status.
 */
typedef struct {
    uint32_t head, tail;  /* sorted sub-list, or NIL */
    uint32_t m;           /* bits still to split below */
} oracle_task;

typedef struct {
    pbit_oracle_ctx proto;
    oracle_task *tasks;
    uint32_t n_tasks;
    uint32_t next_task;
    pthread_mutex_t mu;
    int failed;
} oracle_pool;

static void *oracle_worker(void *arg)
{
    oracle_pool *pool = (oracle_pool *)arg;
    pbit_oracle_ctx c = pool->proto;
    c.roots = (uint32_t *)malloc((size_t)(c.width / c.K) * 2u * c.omega * sizeof(uint32_t));
    if (!c.roots) {
        pthread_mutex_lock(&pool->mu);
        pool->failed = 1;
        pthread_mutex_unlock(&pool->mu);
        return NULL;
    }
    for (;;) {
        pthread_mutex_lock(&pool->mu);
        uint32_t t = pool->next_task++;
        pthread_mutex_unlock(&pool->mu);
        if (t >= pool->n_tasks)
            break;
        oracle_task *tk = &pool->tasks[t];
        if (tk->head == ORACLE_NIL)
            continue;
        uint32_t h = tk->m > 0 ? oracle_pbit(&c, tk->head, tk->m, ORACLE_NIL) : tk->head;
        uint32_t last = h;
        while (c.next[last] != ORACLE_NIL)
            last = c.next[last];
        tk->head = h;
        tk->tail = last;
    }
    free(c.roots);
    return NULL;
}

/* One split level over every task: task i becomes omega tasks in pattern
 * order, each a first-in-first-out group. */
static oracle_task *oracle_split_tasks(const pbit_oracle_ctx *c, const oracle_task *in,
                                       uint32_t n_in)
{
    oracle_task *out = (oracle_task *)malloc((size_t)n_in * c->omega * sizeof(oracle_task));
    if (!out)
        return NULL;
    for (uint32_t t = 0; t < n_in; t++) {
        oracle_task *g = out + (size_t)t * c->omega;
        uint32_t m = in[t].m - c->K;
        for (uint32_t d = 0; d < c->omega; d++) {
            g[d].head = g[d].tail = ORACLE_NIL;
            g[d].m = m;
        }
        for (uint32_t i = in[t].head; i != ORACLE_NIL;) {
            uint32_t following = c->next[i];
            uint32_t d = (uint32_t)((oracle_key(c, i) >> m) & (uint64_t)(c->omega - 1u));
            c->next[i] = ORACLE_NIL;
            if (g[d].head == ORACLE_NIL)
                g[d].head = i;
            else
                c->next[g[d].tail] = i;
            g[d].tail = i;
            i = following;
        }
    }
    return out;
}

int64_t pbit_oracle_sort_threads(uint32_t head, uint32_t *next, const void *keys, uint64_t n,
                                 uint32_t M, uint32_t K, uint32_t flags, uint32_t threads)
{
    if (!oracle_valid_shape(M, K) || (flags & ~(uint32_t)ORACLE_FLAG_DESCENDING))
        return ORACLE_EINVAL;
    if (n >= (uint64_t)ORACLE_NIL)
        return ORACLE_EINVAL;
    if (n == 0 || head == ORACLE_NIL)
        return (n == 0 && head == ORACLE_NIL) ? (int64_t)ORACLE_NIL : ORACLE_EINVAL;
    if (!next || !keys || head >= n)
        return ORACLE_EINVAL;
    int st = oracle_walk_check(head, next, n, 0, (uint32_t)n);
    if (st != ORACLE_OK)
        return st;
    if (threads == 0) {
        long p = sysconf(_SC_NPROCESSORS_ONLN);
        threads = p > 0 ? (uint32_t)p : 1u;
    }
    oracle_pool pool;
    memset(&pool, 0, sizeof pool);
    pool.proto.next = next;
    pool.proto.keys = keys;
    pool.proto.width = M;
    pool.proto.K = K;
    pool.proto.omega = 1u << K;
    pool.proto.descending = (flags & ORACLE_FLAG_DESCENDING) != 0;

    oracle_task *tasks = (oracle_task *)malloc(sizeof(oracle_task));
    if (!tasks)
        return ORACLE_ENOMEM;
    tasks[0].head = head;
    tasks[0].m = M;
    uint32_t n_tasks = 1;
    do {
        oracle_task *split = oracle_split_tasks(&pool.proto, tasks, n_tasks);
        free(tasks);
        if (!split)
            return ORACLE_ENOMEM;
        tasks = split;
        n_tasks *= pool.proto.omega;
    } while (n_tasks < 256u && tasks[0].m > 0);

    pool.tasks = tasks;
    pool.n_tasks = n_tasks;
    pthread_mutex_init(&pool.mu, NULL);
    pthread_t *tid = (pthread_t *)malloc((size_t)threads * sizeof(pthread_t));
    uint32_t started = 0;
    if (tid)
        for (; started < threads; started++)
            if (pthread_create(&tid[started], NULL, oracle_worker, &pool) != 0)
                break;
    if (started == 0)
        oracle_worker(&pool);
    for (uint32_t t = 0; t < started; t++)
        pthread_join(tid[t], NULL);
    free(tid);
    pthread_mutex_destroy(&pool.mu);
    if (pool.failed) {
        free(tasks);
        return ORACLE_ENOMEM;
    }
    /* join the sorted groups in pattern order (Sec. 6 for the direction) */
    uint32_t first = ORACLE_NIL, last = ORACLE_NIL;
    for (uint32_t s = 0; s < n_tasks; s++) {
        const oracle_task *tk = &tasks[pool.proto.descending ? n_tasks - 1u - s : s];
        if (tk->head == ORACLE_NIL)
            continue;
        if (first == ORACLE_NIL)
            first = tk->head;
        else
            next[last] = tk->head;
        last = tk->tail;
    }
    free(tasks);
    return (int64_t)first;
}
