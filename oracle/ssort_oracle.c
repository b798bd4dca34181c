/*
 * CPU oracle for the string sorter.  TEST INFRASTRUCTURE ONLY: nothing in the
 * product path links, loads or calls it; only the tests, the smoke check and
 * the benchmark's CPU-baseline leg do.  It shares no code, header or table
 * with the HIP library.
 *
 * What it computes (Preliminaries): the input is n strings s_0..s_{n-1}; the
 * order is the canonical lexicographic one over unsigned bytes in which a
 * proper prefix precedes its extensions (the zero terminator lies outside the
 * alphabet, and the empty string is the smallest string).  The result is the
 * permutation perm with (s_perm[i], perm[i]) strictly increasing, i.e. identical
 * strings in ascending input index, and the LCP array H with H[0] = 0 (the
 * undefined first entry, read as lcp(empty, s) = 0) and H[i] = lcp(s_perm[i-1],
 * s_perm[i]).
 *
 * Sorting follows multikey quicksort (Basic sequential algorithms): a ternary
 * partition on the character at the common depth d, recursion on "<" and ">"
 * at d and on "=" at d+1, and an insertion sort for small ranges.  The LCP
 * array is the plain definition, a byte loop over adjacent outputs.
 *
 * With threads > 1 the same sequential multikey quicksort runs on several
 * threads: a subproblem of more than 2^16 strings goes to a shared job queue
 * guarded by a mutex instead of the thread's own stack (the job-queue pattern
 * of the practical parallelisation of S5, Section 4.5).  The subproblems are
 * disjoint ranges and each is partitioned deterministically, so the result
 * does not depend on the thread count or the schedule.  This exists to time
 * the oracle on every host core; it is the same algorithm.
 *
 * The single-step helpers restate one step of super scalar string sample sort
 * (Algorithm 1, Fig. 1, Implementation details) in its plain form: the 8-byte
 * big-endian key with zero padding, the lower-bound bucket number with
 * equality buckets, the level order of a perfect search tree, and the
 * splitter LCPs by a byte loop.  They check intermediate results.
 *
 * The LCP algorithms of Section 5 at the end (LCP-insertion sort, Algorithm
 * 5; binary LCP-compare and LCP-merge, Algorithms 2 and 3; K-way LCP-merge
 * with an LCP-aware tournament tree, Algorithm 4) are written out with a
 * counter of character comparisons, so that the tests can hold them to the
 * bounds of the section's theorems and to the plain definition above.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_TO_END 1u

typedef struct {
    const uint8_t *chars;
    uint64_t nchars;
    uint64_t *st;   /* start offset of each string */
    uint64_t *ln;   /* length of each string */
    uint32_t n;
} strs_t;

static int load_strs(strs_t *S, const uint8_t *chars, uint64_t nchars, const uint64_t *off,
                     const uint32_t *len, uint32_t n, uint32_t flags)
{
    S->chars = chars;
    S->nchars = nchars;
    S->n = n;
    S->st = (uint64_t *)malloc(sizeof(uint64_t) * (n ? n : 1));
    S->ln = (uint64_t *)malloc(sizeof(uint64_t) * (n ? n : 1));
    if (!S->st || !S->ln) return -1;
    for (uint32_t i = 0; i < n; ++i) {
        S->st[i] = off[i];
        if (flags & ORACLE_TO_END) S->ln[i] = nchars - off[i];
        else if (len) S->ln[i] = len[i];
        else S->ln[i] = off[i + 1] - off[i];
        if (S->st[i] > nchars || S->ln[i] > nchars - S->st[i]) return -2;
    }
    return 0;
}

static void free_strs(strs_t *S)
{
    free(S->st);
    free(S->ln);
}

/* character at depth d as an int: 1 + byte while inside the string, 0 at its end */
static inline int ch(const strs_t *S, uint32_t i, uint64_t d)
{
    return d < S->ln[i] ? 1 + (int)S->chars[S->st[i] + d] : 0;
}

/* full comparison from depth d on (both strings agree before d), ties by index */
static int cmp_from(const strs_t *S, uint32_t a, uint32_t b, uint64_t d)
{
    for (;; ++d) {
        int ca = ch(S, a, d), cb = ch(S, b, d);
        if (ca != cb) return ca < cb ? -1 : 1;
        if (ca == 0) break;
    }
    return a < b ? -1 : (a > b ? 1 : 0);
}

static int cmp_u32(const void *x, const void *y)
{
    uint32_t a = *(const uint32_t *)x, b = *(const uint32_t *)y;
    return a < b ? -1 : (a > b);
}

typedef struct { uint64_t lo, hi, d; } frame_t;

/* Shared job queue of the multi-threaded run (NULL: one thread). */
#define POOL_SPLIT (1u << 16)
typedef struct {
    pthread_mutex_t mu;
    pthread_cond_t cv;
    frame_t *q;
    uint64_t qn, qcap;
    int active;          /* threads working on a job */
    int failed;          /* an allocation failed */
} pool_t;

static void pool_push(pool_t *P, frame_t f)
{
    pthread_mutex_lock(&P->mu);
    if (P->qn == P->qcap) {
        uint64_t nc = P->qcap ? 2 * P->qcap : 64;
        frame_t *nq = (frame_t *)realloc(P->q, sizeof(frame_t) * nc);
        if (!nq) {
            P->failed = 1;
            pthread_mutex_unlock(&P->mu);
            return;
        }
        P->q = nq;
        P->qcap = nc;
    }
    P->q[P->qn++] = f;
    pthread_cond_signal(&P->cv);
    pthread_mutex_unlock(&P->mu);
}

/* Multikey quicksort of the frame f with the thread's own stack; frames of
 * more than POOL_SPLIT strings go to the shared queue when there is one. */
static int mkqs_frame(const strs_t *S, uint32_t *a, frame_t f0, pool_t *pool)
{
    uint64_t cap = 1024, top = 0;
    frame_t *stk = (frame_t *)malloc(sizeof(frame_t) * cap);
    if (!stk) return -1;
    stk[top++] = f0;
    while (top) {
        frame_t f = stk[--top];
        uint64_t m = f.hi - f.lo;
        if (m < 2) continue;
        if (m < 16) {                         /* insertion sort base case */
            for (uint64_t i = f.lo + 1; i < f.hi; ++i) {
                uint32_t x = a[i];
                uint64_t j = i;
                while (j > f.lo && cmp_from(S, a[j - 1], x, f.d) > 0) {
                    a[j] = a[j - 1];
                    --j;
                }
                a[j] = x;
            }
            continue;
        }
        /* pivot character: median of three */
        int c0 = ch(S, a[f.lo], f.d), c1 = ch(S, a[f.lo + m / 2], f.d), c2 = ch(S, a[f.hi - 1], f.d);
        int pv = c0 < c1 ? (c1 < c2 ? c1 : (c0 < c2 ? c2 : c0)) : (c0 < c2 ? c0 : (c1 < c2 ? c2 : c1));
        /* ternary partition: [lo,lt) <, [lt,gt) =, [gt,hi) > */
        uint64_t lt = f.lo, i = f.lo, gt = f.hi;
        while (i < gt) {
            int c = ch(S, a[i], f.d);
            if (c < pv) {
                uint32_t t = a[lt]; a[lt] = a[i]; a[i] = t;
                ++lt; ++i;
            } else if (c > pv) {
                --gt;
                uint32_t t = a[gt]; a[gt] = a[i]; a[i] = t;
            } else {
                ++i;
            }
        }
        if (top + 3 > cap) {
            frame_t *grown = (frame_t *)realloc(stk, sizeof(frame_t) * cap * 2);
            if (!grown) {
                free(stk);
                return -1;
            }
            stk = grown;
            cap *= 2;
        }
        frame_t sub[3];
        int ns = 0;
        sub[ns++] = (frame_t){f.lo, lt, f.d};
        sub[ns++] = (frame_t){gt, f.hi, f.d};
        if (pv == 0)        /* every string of the "=" group ended: identical strings */
            qsort(a + lt, gt - lt, sizeof(uint32_t), cmp_u32);
        else
            sub[ns++] = (frame_t){lt, gt, f.d + 1};
        for (int k = 0; k < ns; ++k) {
            if (pool && sub[k].hi - sub[k].lo > POOL_SPLIT) pool_push(pool, sub[k]);
            else stk[top++] = sub[k];
        }
    }
    free(stk);
    return 0;
}

typedef struct {
    const strs_t *S;
    uint32_t *a;
    pool_t *pool;
} worker_arg_t;

/* A thread of the multi-threaded run: take jobs until the queue is empty and
 * no other thread can add one. */
static void *pool_worker(void *arg)
{
    worker_arg_t *W = (worker_arg_t *)arg;
    pool_t *P = W->pool;
    for (;;) {
        pthread_mutex_lock(&P->mu);
        while (P->qn == 0 && P->active > 0) pthread_cond_wait(&P->cv, &P->mu);
        if (P->qn == 0) {
            pthread_cond_broadcast(&P->cv);
            pthread_mutex_unlock(&P->mu);
            return NULL;
        }
        frame_t f = P->q[--P->qn];
        P->active++;
        pthread_mutex_unlock(&P->mu);
        int rc = mkqs_frame(W->S, W->a, f, P);
        pthread_mutex_lock(&P->mu);
        if (rc) P->failed = 1;
        P->active--;
        if (P->qn == 0 && P->active == 0) pthread_cond_broadcast(&P->cv);
        pthread_mutex_unlock(&P->mu);
    }
}

static int mkqs(const strs_t *S, uint32_t *a, uint64_t n, int threads)
{
    if (threads <= 1 || n <= POOL_SPLIT) return mkqs_frame(S, a, (frame_t){0, n, 0}, NULL);
    pool_t P;
    memset(&P, 0, sizeof(P));
    pthread_mutex_init(&P.mu, NULL);
    pthread_cond_init(&P.cv, NULL);
    pool_push(&P, (frame_t){0, n, 0});
    worker_arg_t W = {S, a, &P};
    pthread_t *tid = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)threads);
    int started = 0;
    if (tid)
        for (int t = 1; t < threads; ++t)
            if (pthread_create(&tid[started], NULL, pool_worker, &W) == 0) ++started;
    pool_worker(&W);
    for (int t = 0; t < started; ++t) pthread_join(tid[t], NULL);
    free(tid);
    free(P.q);
    pthread_cond_destroy(&P.cv);
    pthread_mutex_destroy(&P.mu);
    return P.failed ? -1 : 0;
}

static uint64_t lcp_pair(const strs_t *S, uint32_t a, uint32_t b)
{
    uint64_t m = S->ln[a] < S->ln[b] ? S->ln[a] : S->ln[b];
    const uint8_t *pa = S->chars + S->st[a], *pb = S->chars + S->st[b];
    uint64_t h = 0;
    while (h < m && pa[h] == pb[h]) ++h;
    return h;
}

typedef struct {
    const strs_t *S;
    const uint32_t *perm;
    uint32_t *lcp;
    uint32_t lo, hi;
} lcp_arg_t;

static void *lcp_range(void *arg)
{
    lcp_arg_t *A = (lcp_arg_t *)arg;
    for (uint32_t i = A->lo; i < A->hi; ++i)
        A->lcp[i] = i ? (uint32_t)lcp_pair(A->S, A->perm[i - 1], A->perm[i]) : 0;
    return NULL;
}

/* Sort; perm and lcp (nullable) are host arrays of n entries; threads <= 1
 * runs on the calling thread only.  Returns 0 on success, <0 on bad input
 * (-1: out of memory).  lcp values are clamped to 32 bits (strings longer
 * than 4 GiB are outside the library's contract). */
int ssort_oracle_sort(const uint8_t *chars, uint64_t nchars, const uint64_t *offsets,
                      const uint32_t *lengths, uint32_t n, uint32_t flags,
                      uint32_t *perm, uint32_t *lcp, int threads)
{
    strs_t S;
    int rc = load_strs(&S, chars, nchars, offsets, lengths, n, flags);
    if (rc) { free_strs(&S); return rc; }
    for (uint32_t i = 0; i < n; ++i) perm[i] = i;
    if (mkqs(&S, perm, n, threads)) { free_strs(&S); return -1; }
    if (lcp) {
        /* the LCP array: the byte loop over neighbours, in ranges per thread */
        int T = threads > 1 ? threads : 1;
        if ((uint64_t)T > (uint64_t)n / 65536 + 1) T = (int)((uint64_t)n / 65536 + 1);
        lcp_arg_t *A = (lcp_arg_t *)malloc(sizeof(lcp_arg_t) * (size_t)T);
        pthread_t *tid = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)T);
        if (!A || !tid) {
            free(A);
            free(tid);
            free_strs(&S);
            return -1;
        }
        /* thread t > 0 computes range t; a thread that cannot start leaves
         * its range to the calling thread */
        uint8_t *run = (uint8_t *)calloc((size_t)T, 1);
        for (int t = 0; t < T; ++t)
            A[t] = (lcp_arg_t){&S, perm, lcp, (uint32_t)((uint64_t)n * t / T), (uint32_t)((uint64_t)n * (t + 1) / T)};
        for (int t = 1; t < T; ++t)
            if (run && pthread_create(&tid[t], NULL, lcp_range, &A[t]) == 0) run[t] = 1;
        lcp_range(&A[0]);
        for (int t = 1; t < T; ++t) {
            if (run && run[t]) pthread_join(tid[t], NULL);
            else lcp_range(&A[t]);
        }
        free(run);
        free(A);
        free(tid);
    }
    free_strs(&S);
    return 0;
}

/* Distinguishing prefix and LCP sum of a sorted result (Preliminaries).
 * out[0] = D (length-delimited: sum of min(|s|, 1 + max(H[i], H[i+1])))
 * out[1] = D with one terminator per string (the paper's convention)
 * out[2] = L = sum of H[1..n-1]
 * out[3] = N = total length;  out[4] = N plus n terminators */
int ssort_oracle_stats(const uint8_t *chars, uint64_t nchars, const uint64_t *offsets,
                       const uint32_t *lengths, uint32_t n, uint32_t flags,
                       const uint32_t *perm, const uint32_t *lcp, uint64_t *out)
{
    strs_t S;
    int rc = load_strs(&S, chars, nchars, offsets, lengths, n, flags);
    if (rc) { free_strs(&S); return rc; }
    uint64_t D = 0, Dp = 0, L = 0, N = 0;
    for (uint32_t i = 0; i < n; ++i) {
        uint64_t hl = i ? lcp[i] : 0, hr = (i + 1 < n) ? lcp[i + 1] : 0;
        uint64_t mx = 1 + (hl > hr ? hl : hr);
        uint64_t len = S.ln[perm[i]];
        D += mx < len ? mx : len;
        Dp += mx < len + 1 ? mx : len + 1;
        if (i) L += lcp[i];
        N += len;
    }
    out[0] = D; out[1] = Dp; out[2] = L; out[3] = N; out[4] = N + n;
    free_strs(&S);
    return 0;
}

/* Invariant checker, O(L + n): verifies that perm is a permutation, lcp[0]=0,
 * and for every i >= 1 with a = s_perm[i-1], b = s_perm[i], h = lcp[i]:
 * a[0..h) = b[0..h), and either h = |a| = |b| with perm[i-1] < perm[i], or
 * h = |a| < |b|, or h < min(|a|,|b|) with a[h] < b[h].  Together these fix the
 * sorted order and the LCP array exactly.  Returns -1 if everything holds,
 * else the first failing position (n for a permutation failure). */
int64_t ssort_oracle_check(const uint8_t *chars, uint64_t nchars, const uint64_t *offsets,
                           const uint32_t *lengths, uint32_t n, uint32_t flags,
                           const uint32_t *perm, const uint32_t *lcp)
{
    strs_t S;
    int rc = load_strs(&S, chars, nchars, offsets, lengths, n, flags);
    if (rc) { free_strs(&S); return -2; }
    int64_t bad = -1;
    uint8_t *seen = (uint8_t *)calloc(n ? n : 1, 1);
    for (uint32_t i = 0; i < n && bad < 0; ++i) {
        if (perm[i] >= n || seen[perm[i]]) bad = n;
        else seen[perm[i]] = 1;
    }
    if (bad < 0 && n && lcp[0] != 0) bad = 0;
    for (uint32_t i = 1; i < n && bad < 0; ++i) {
        uint32_t a = perm[i - 1], b = perm[i];
        uint64_t h = lcp[i], la = S.ln[a], lb = S.ln[b];
        uint64_t m = la < lb ? la : lb;
        if (h > m || memcmp(S.chars + S.st[a], S.chars + S.st[b], h) != 0) { bad = i; break; }
        int ok;
        if (h == la && h == lb) ok = a < b;
        else if (h == la) ok = 1;
        else if (h == lb) ok = 0;
        else ok = S.chars[S.st[a] + h] < S.chars[S.st[b] + h];
        if (!ok) bad = i;
    }
    free(seen);
    free_strs(&S);
    return bad;
}

/* ---- single-step helpers (one step of Algorithm 1, plain definitions) ---- */

/* 8 characters of string i from depth h, first character in the most
 * significant byte, zero past the end of the string. */
void ssort_oracle_keys(const uint8_t *chars, uint64_t nchars, const uint64_t *offsets,
                       const uint32_t *lengths, uint32_t n, uint32_t flags,
                       const uint32_t *idx, uint64_t m, const uint32_t *depth, uint64_t *keys)
{
    strs_t S;
    if (load_strs(&S, chars, nchars, offsets, lengths, n, flags)) { free_strs(&S); return; }
    for (uint64_t j = 0; j < m; ++j) {
        uint64_t k = 0;
        for (int t = 0; t < 8; ++t) {
            uint64_t p = (uint64_t)depth[j] + t;
            uint64_t b = p < S.ln[idx[j]] ? S.chars[S.st[idx[j]] + p] : 0;
            k = k * 256 + b;
        }
        keys[j] = k;
    }
    free_strs(&S);
}

/* Bucket of each key for sorted splitters x[0..v): with l the number of
 * splitters strictly below the key, bucket 2l, or 2l+1 if the key equals x[l]. */
void ssort_oracle_classify(const uint64_t *keys, uint64_t m, const uint64_t *x, uint32_t v,
                           uint32_t *bucket)
{
    for (uint64_t j = 0; j < m; ++j) {
        uint32_t l = 0;
        while (l < v && x[l] < keys[j]) ++l;
        bucket[j] = 2 * l + ((l < v && x[l] == keys[j]) ? 1 : 0);
    }
}

/* Level order of a perfect binary search tree over in-order ranks 0..v-1
 * (v = 2^d - 1): rank[j-1] is the in-order rank of level-order node j >= 1.
 * Built by recursion: the root is the middle rank, children cover halves. */
static void tree_rec(uint32_t lo, uint32_t hi, uint32_t j, uint32_t *rank)
{
    if (lo >= hi) return;
    uint32_t mid = lo + (hi - lo) / 2;
    rank[j - 1] = mid;
    tree_rec(lo, mid, 2 * j, rank);
    tree_rec(mid + 1, hi, 2 * j + 1, rank);
}

void ssort_oracle_tree_ranks(uint32_t v, uint32_t *rank)
{
    tree_rec(0, v, 1, rank);
}

/* LCP in bytes of adjacent splitters, h[0] = h[v] = 0, h[i] = lcp(x[i-1], x[i])
 * counted over the 8 key bytes from the most significant one. */
void ssort_oracle_splitter_lcp(const uint64_t *x, uint32_t v, uint32_t *h)
{
    h[0] = 0;
    h[v] = 0;
    for (uint32_t i = 1; i < v; ++i) {
        uint32_t l = 0;
        while (l < 8 && ((x[i - 1] >> (56 - 8 * l)) & 0xFF) == ((x[i] >> (56 - 8 * l)) & 0xFF)) ++l;
        h[i] = l;
    }
}

/* ---- Section 5: LCP-aware insertion sort and merging, with a counter of
 * character comparisons.  A character comparison is one evaluation of the
 * loop condition that compares the characters of two strings at the same
 * position (the final ordering test after the loop uses the same two
 * characters and is counted with the comparison that ended the loop, as the
 * proofs of the section do). ---- */

/* LCP-insertion sort (Algorithm 5) of the strings idx[0..m), which share the
 * common prefix hbar.  out_perm gets the sorted order (identical strings keep
 * their order in idx: x is placed after an equal string), out_lcp the LCP
 * array (out_lcp[0] = 0).  *ncmp counts character comparisons (bounded by
 * L + m(m-1)/2 by the theorem after Algorithm 5).  Returns 0, or <0 on bad
 * input. */
int ssort_oracle_lcp_insertion_sort(const uint8_t *chars, uint64_t nchars, const uint64_t *offsets,
                                    const uint32_t *lengths, uint32_t n, uint32_t flags,
                                    const uint32_t *idx, uint32_t m, uint32_t hbar,
                                    uint32_t *out_perm, uint32_t *out_lcp, uint64_t *ncmp)
{
    strs_t S;
    int rc = load_strs(&S, chars, nchars, offsets, lengths, n, flags);
    if (rc) { free_strs(&S); return rc; }
    for (uint32_t j = 0; j < m; ++j)
        if (idx[j] >= n) { free_strs(&S); return -3; }
    /* s[0..j) sorted, H[i] = lcp(s[i-1], s[i]) for 1 <= i < j */
    uint32_t *s = out_perm;
    uint64_t *H = (uint64_t *)calloc((size_t)m + 1, sizeof(uint64_t));
    if (!H) { free_strs(&S); return -1; }
    uint64_t cnt = 0;
    for (uint32_t j = 0; j < m; ++j) {
        uint32_t x = idx[j];
        uint64_t hp = hbar;          /* h': LCP of x with the string last passed */
        uint64_t i = j;
        H[j] = hbar;                 /* x shares hbar with every string */
        while (i > 0) {
            if (H[i] < hp) break;                   /* case 1: s[i-1] < x */
            if (H[i] == hp) {                       /* case 2: compare characters */
                uint64_t p = hp;
                for (;;) {
                    ++cnt;
                    int cx = ch(&S, x, hp), cy = ch(&S, s[i - 1], hp);
                    if (!(cx != 0 && cx == cy)) break;
                    ++hp;
                }
                if (ch(&S, x, hp) >= ch(&S, s[i - 1], hp)) {   /* x after s[i-1] */
                    H[i] = hp;
                    hp = p;
                    break;
                }
            }
            /* case 3 (or x smaller after comparing): move s[i-1] right */
            s[i] = s[i - 1];
            H[i + 1] = H[i];
            --i;
        }
        s[i] = x;
        H[i + 1] = hp;
    }
    if (out_lcp) {
        if (m) out_lcp[0] = 0;
        for (uint32_t i = 1; i < m; ++i) out_lcp[i] = (uint32_t)H[i];
    }
    if (ncmp) *ncmp = cnt;
    free(H);
    free_strs(&S);
    return 0;
}

/* Binary LCP-compare (Algorithm 2) of strings a and b with ha = lcp(p, s_a),
 * hb = lcp(p, s_b) for a common smaller string p.  Returns 1 when s_a comes
 * first (equal strings: the smaller input index first, the stable reading of
 * the algorithm's "a for s_a <= s_b"); *h gets lcp(s_a, s_b). */
static int lcp_compare(const strs_t *S, uint32_t a, uint64_t ha, uint32_t b, uint64_t hb, uint64_t *h, uint64_t *cnt)
{
    if (ha == hb) {                                  /* case 1 */
        uint64_t hh = ha;
        for (;;) {
            ++*cnt;
            int ca = ch(S, a, hh), cb = ch(S, b, hh);
            if (!(ca != 0 && ca == cb)) break;
            ++hh;
        }
        *h = hh;
        int ca = ch(S, a, hh), cb = ch(S, b, hh);
        if (ca != cb) return ca < cb;
        return a < b;                                /* both ended: identical strings */
    }
    if (ha < hb) {                                   /* case 2: s_b first */
        *h = ha;
        return 0;
    }
    *h = hb;                                         /* case 3: s_a first */
    return 1;
}

/* K-way LCP-merge (Algorithm 4) of the runs [rb[k], rb[k+1]) of (perm, lcp)
 * into (out_perm, out_lcp), with an LCP-aware loser tree over KP leaves (KP
 * the smallest power of two >= K; the extra leaves are empty runs). */
static int kway_merge(const strs_t *S, const uint32_t *rb, uint32_t K, const uint32_t *perm, const uint32_t *lcp,
                      uint32_t *out_perm, uint32_t *out_lcp, uint64_t *cnt)
{
    uint32_t KP = 1;
    while (KP < K) KP <<= 1;
    const uint32_t NONE = 0xFFFFFFFFu;   /* an exhausted run (the sentinel, larger than every string) */
    uint64_t *pos = (uint64_t *)malloc(sizeof(uint64_t) * KP);
    uint32_t *y = (uint32_t *)malloc(sizeof(uint32_t) * 2 * KP);    /* loser run of each game node */
    uint64_t *hy = (uint64_t *)malloc(sizeof(uint64_t) * 2 * KP);   /* its LCP with that game's winner */
    if (!pos || !y || !hy) { free(pos); free(y); free(hy); return -1; }
    for (uint32_t r = 0; r < KP; ++r) pos[r] = r < K ? rb[r] : 0;
    #define RUN_LIVE(r) ((r) != NONE && (r) < K && pos[r] < rb[(r) + 1])
    /* initial games bottom-up: node v's winner passes up, its loser stays;
     * wn/wh hold the winners of the level below */
    uint32_t *wn = (uint32_t *)malloc(sizeof(uint32_t) * 2 * KP);
    uint64_t *wh = (uint64_t *)malloc(sizeof(uint64_t) * 2 * KP);
    if (!wn || !wh) { free(pos); free(y); free(hy); free(wn); free(wh); return -1; }
    for (uint32_t r = 0; r < KP; ++r) {
        wn[KP + r] = RUN_LIVE(r) ? r : NONE;
        wh[KP + r] = 0;              /* LCP with the empty string */
    }
    for (uint32_t v = KP - 1; v >= 1; --v) {
        uint32_t a = wn[2 * v], b = wn[2 * v + 1];
        uint64_t ha = wh[2 * v], hb = wh[2 * v + 1];
        if (b == NONE) { wn[v] = a; wh[v] = ha; y[v] = b; hy[v] = hb; continue; }
        if (a == NONE) { wn[v] = b; wh[v] = hb; y[v] = a; hy[v] = ha; continue; }
        uint64_t h;
        int af = lcp_compare(S, perm[pos[a]], ha, perm[pos[b]], hb, &h, cnt);
        wn[v] = af ? a : b;
        wh[v] = af ? ha : hb;
        y[v] = af ? b : a;
        hy[v] = h;
    }
    uint32_t w = KP > 1 ? wn[1] : wn[KP];
    uint64_t hw = KP > 1 ? wh[1] : wh[KP];
    uint64_t j = 0;
    while (w != NONE) {
        out_perm[j] = perm[pos[w]];
        if (out_lcp) out_lcp[j] = j ? (uint32_t)hw : 0;
        ++j;
        /* the winner's run advances; its next string's LCP with the string
         * just written is the run's own LCP entry */
        ++pos[w];
        uint32_t x = RUN_LIVE(w) ? w : NONE;
        uint64_t hx = x != NONE ? lcp[pos[w]] : 0;
        for (uint32_t v = (KP + w) >> 1; v >= 1; v >>= 1) {
            uint32_t b = y[v];
            if (b == NONE) continue;                 /* x wins against an empty run */
            if (x == NONE) {                         /* the stored loser wins */
                y[v] = x; x = b;
                uint64_t t = hy[v]; hy[v] = hx; hx = t;
                continue;
            }
            uint64_t h;
            int xf = lcp_compare(S, perm[pos[x]], hx, perm[pos[b]], hy[v], &h, cnt);
            if (!xf) {
                y[v] = x;
                x = b;
                hx = hy[v];
            }
            hy[v] = h;
        }
        w = x;
        hw = hx;
    }
    #undef RUN_LIVE
    free(pos); free(y); free(hy); free(wn); free(wh);
    return 0;
}

/* Binary LCP-merge (Algorithm 3) of two runs of (perm, lcp). */
static void binary_merge(const strs_t *S, const uint32_t *pa, const uint32_t *la, uint64_t na,
                         const uint32_t *pb, const uint32_t *lb, uint64_t nb,
                         uint32_t *out_perm, uint32_t *out_lcp, uint64_t *cnt)
{
    uint64_t i = 0, k = 0, j = 0;
    uint64_t ha = 0, hb = 0;     /* LCPs of the candidates with the last output (first: the empty string) */
    while (i < na && k < nb) {
        uint64_t h;
        int af = lcp_compare(S, pa[i], ha, pb[k], hb, &h, cnt);
        if (af) {
            out_perm[j] = pa[i];
            out_lcp[j++] = (uint32_t)ha;
            ++i;
            hb = h;                               /* lcp(written s_a, s_b) */
            ha = i < na ? la[i] : 0;              /* lcp(written s_a, its successor) */
        } else {
            out_perm[j] = pb[k];
            out_lcp[j++] = (uint32_t)hb;
            ++k;
            ha = h;
            hb = k < nb ? lb[k] : 0;
        }
    }
    for (; i < na; ++i, ha = i < na ? la[i] : 0) { out_perm[j] = pa[i]; out_lcp[j++] = (uint32_t)ha; }
    for (; k < nb; ++k, hb = k < nb ? lb[k] : 0) { out_perm[j] = pb[k]; out_lcp[j++] = (uint32_t)hb; }
}

/* Merge K sorted runs of indices into `in` (Algorithm 4; with binary != 0 and
 * K = 2, Algorithm 3).  run_begin[0..K]; lcp_in[p] = LCP of the strings at
 * p-1 and p of the same run (ignored at a run's start).  out_lcp[0] = 0.
 * *ncmp counts character comparisons.  Returns 0, or <0 on bad input. */
int ssort_oracle_lcp_merge(const uint8_t *chars, uint64_t nchars, const uint64_t *offsets,
                           const uint32_t *lengths, uint32_t n, uint32_t flags,
                           const uint32_t *run_begin, uint32_t K, int binary,
                           const uint32_t *perm_in, const uint32_t *lcp_in,
                           uint32_t *out_perm, uint32_t *out_lcp, uint64_t *ncmp)
{
    if (K < 1 || run_begin[0] != 0 || (binary && K != 2)) return -3;
    for (uint32_t k = 0; k < K; ++k)
        if (run_begin[k + 1] < run_begin[k]) return -3;
    uint64_t total = run_begin[K];
    for (uint64_t p = 0; p < total; ++p)
        if (perm_in[p] >= n) return -3;
    strs_t S;
    int rc = load_strs(&S, chars, nchars, offsets, lengths, n, flags);
    if (rc) { free_strs(&S); return rc; }
    uint64_t cnt = 0;
    uint32_t *tmp = (uint32_t *)malloc(sizeof(uint32_t) * (total ? total : 1));
    if (!tmp) { free_strs(&S); return -1; }
    uint32_t *ol = out_lcp ? out_lcp : tmp;
    if (binary) {
        binary_merge(&S, perm_in, lcp_in, run_begin[1], perm_in + run_begin[1], lcp_in + run_begin[1],
                     run_begin[2] - run_begin[1], out_perm, ol, &cnt);
        if (total) ol[0] = 0;
    } else {
        rc = kway_merge(&S, run_begin, K, perm_in, lcp_in, out_perm, ol, &cnt);
    }
    if (ncmp) *ncmp = cnt;
    free(tmp);
    free_strs(&S);
    return rc;
}

/* LCP-mergesort of the strings a[0..m) into (out, hout) by halving (K = 2,
 * Algorithm 3) or K-way splitting (Algorithm 4); scratch buffers of m. */
static int mergesort_rec(const strs_t *S, uint32_t *a, uint32_t *h, uint64_t m, uint32_t K,
                         uint32_t *tp, uint32_t *th, uint64_t *cnt)
{
    if (m <= 1) {
        if (m) h[0] = 0;
        return 0;
    }
    const uint32_t parts = K;   /* K parts even when m < K (some empty) */
    uint32_t rb[65];
    for (uint32_t k = 0; k <= parts; ++k) rb[k] = (uint32_t)(m * k / parts);
    for (uint32_t k = 0; k < parts; ++k)
        if (mergesort_rec(S, a + rb[k], h + rb[k], rb[k + 1] - rb[k], K, tp + rb[k], th + rb[k], cnt)) return -1;
    if (K == 2) {
        binary_merge(S, a, h, rb[1], a + rb[1], h + rb[1], m - rb[1], tp, th, cnt);
    } else if (kway_merge(S, rb, parts, a, h, tp, th, cnt)) {
        return -1;
    }
    memcpy(a, tp, sizeof(uint32_t) * m);
    memcpy(h, th, sizeof(uint32_t) * m);
    h[0] = 0;
    return 0;
}

/* LCP-mergesort (the theorems after Algorithms 3 and 4) of all n strings:
 * perm and lcp as for ssort_oracle_sort; 2 <= K <= 64.  *ncmp counts
 * character comparisons.  Returns 0, or <0 on bad input. */
int ssort_oracle_lcp_mergesort(const uint8_t *chars, uint64_t nchars, const uint64_t *offsets,
                               const uint32_t *lengths, uint32_t n, uint32_t flags, uint32_t K,
                               uint32_t *perm, uint32_t *lcp, uint64_t *ncmp)
{
    if (K < 2 || K > 64) return -3;
    strs_t S;
    int rc = load_strs(&S, chars, nchars, offsets, lengths, n, flags);
    if (rc) { free_strs(&S); return rc; }
    uint32_t *tp = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint32_t *th = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    if (!tp || !th) { free(tp); free(th); free_strs(&S); return -1; }
    for (uint32_t i = 0; i < n; ++i) perm[i] = i;
    uint64_t cnt = 0;
    rc = mergesort_rec(&S, perm, lcp, n, K, tp, th, &cnt);
    if (ncmp) *ncmp = cnt;
    free(tp);
    free(th);
    free_strs(&S);
    return rc;
}
