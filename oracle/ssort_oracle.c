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
 * The single-step helpers at the end restate one step of super scalar string
 * sample sort (Algorithm 1, Fig. 1, Implementation details) in its plain
 * form: the 8-byte big-endian key with zero padding, the lower-bound bucket
 * number with equality buckets, the level order of a perfect search tree, and
 * the splitter LCPs by a byte loop.  They check intermediate results.
 */
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

static void mkqs(const strs_t *S, uint32_t *a, uint64_t n)
{
    uint64_t cap = 1024, top = 0;
    frame_t *stk = (frame_t *)malloc(sizeof(frame_t) * cap);
    stk[top++] = (frame_t){0, n, 0};
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
            cap *= 2;
            stk = (frame_t *)realloc(stk, sizeof(frame_t) * cap);
        }
        stk[top++] = (frame_t){f.lo, lt, f.d};
        stk[top++] = (frame_t){gt, f.hi, f.d};
        if (pv == 0)        /* every string of the "=" group ended: identical strings */
            qsort(a + lt, gt - lt, sizeof(uint32_t), cmp_u32);
        else
            stk[top++] = (frame_t){lt, gt, f.d + 1};
    }
    free(stk);
}

static uint64_t lcp_pair(const strs_t *S, uint32_t a, uint32_t b)
{
    uint64_t m = S->ln[a] < S->ln[b] ? S->ln[a] : S->ln[b];
    const uint8_t *pa = S->chars + S->st[a], *pb = S->chars + S->st[b];
    uint64_t h = 0;
    while (h < m && pa[h] == pb[h]) ++h;
    return h;
}

/* Sort; perm and lcp (nullable) are host arrays of n entries.  Returns 0 on
 * success, <0 on bad input.  lcp values are clamped to 32 bits (strings longer
 * than 4 GiB are outside the library's contract). */
int ssort_oracle_sort(const uint8_t *chars, uint64_t nchars, const uint64_t *offsets,
                      const uint32_t *lengths, uint32_t n, uint32_t flags,
                      uint32_t *perm, uint32_t *lcp)
{
    strs_t S;
    int rc = load_strs(&S, chars, nchars, offsets, lengths, n, flags);
    if (rc) { free_strs(&S); return rc; }
    for (uint32_t i = 0; i < n; ++i) perm[i] = i;
    mkqs(&S, perm, n);
    if (lcp) {
        if (n) lcp[0] = 0;
        for (uint32_t i = 1; i < n; ++i) lcp[i] = (uint32_t)lcp_pair(&S, perm[i - 1], perm[i]);
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
