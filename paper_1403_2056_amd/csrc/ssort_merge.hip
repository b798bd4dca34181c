// K-way LCP-merge of sorted string runs (Section 5: binary LCP-compare,
// Algorithm 2; K-way LCP-merge with an LCP-aware tournament tree, Algorithm
// 4; the caching variant of the implementation details), for gfx950.
//
// Input: K runs, each a sorted sequence of string indices with its LCP array.
// Output: the merged sequence (equal strings ordered by index) and its LCP
// array.  Parallel form: every g-th element of every run is a sample; a
// sample's cut (for every run, the number of its elements below the sample)
// comes from one LCP-accelerated binary search per run, and the cuts in
// sample order split the merge into independent jobs (a job: for each run
// the elements between two consecutive cuts).  One thread merges one job with
// an LCP-aware loser tree whose nodes cache the 8 characters of their string
// at the node's LCP (the paper caches the one distinguishing character; eight
// fit in the 64-bit word the comparisons use), so most games are decided
// without touching the strings.  A last pass computes the LCP across job
// boundaries.
#include "ssort_dev.h"
#include "ssort_kernels.h"

namespace ssm {

using ssd::Strs;
using ssd::key_at;

constexpr int MNT = 64;          // threads per merge workgroup
constexpr int MKMAX = 32;        // largest K
constexpr uint32_t SENT = 0xFFFFFFFFu;   // exhausted player
constexpr uint32_t WAITING = 0xFFFFFFFEu;   // tree build: no player has reached the node yet
// A player's LCP and the number of valid characters in its cached word share
// one 32-bit entry: LCPs up to HMASK - 8 (about 16 MiB) are supported.
constexpr uint32_t HMASK = 0xFFFFFFu;

struct MergeParams {
    Strs S;
    uint32_t rb[MKMAX + 1];  // run boundaries
    const uint32_t *pin;     // runs of string indices
    const uint32_t *hin;     // their LCP arrays (entry at a run's start ignored)
    uint32_t *pout, *hout;
    uint64_t *cache;         // 8 characters of each input string at its LCP
    uint32_t *cuts;          // (nsamp + 1) rows of K cuts, in sample order
    unsigned long long *err;
    unsigned long long *next_job;   // next merge job to claim
    uint32_t K, n, g, nsamp;
};

// Start and length of string id.
__device__ __forceinline__ void str_ref(const MergeParams &M, uint32_t id, uint64_t *st, uint32_t *ln) {
    const uint64_t s0 = M.S.off[id];
    uint64_t l;
    if (M.S.flags & ssd::TO_END) l = M.S.nchars - s0;
    else if (M.S.len) l = M.S.len[id];
    else l = M.S.off[id + 1] - s0;
    *st = s0;
    *ln = (uint32_t)l;
}

__device__ __forceinline__ uint64_t str_key(const MergeParams &M, uint32_t id, uint32_t h) {
    uint64_t st;
    uint32_t ln;
    str_ref(M, id, &st, &ln);
    return key_at(M.S.chars, M.S.nchars, st, ln, h);
}

// Compare strings a and b that agree on [0, d): returns their LCP and
// whether a < b (equal strings: by index), and in *lw the loser's characters
// at the LCP (the word's leading *lv of them valid), taken from the bytes
// just compared.  Both strings are located once, then compared 32 characters
// (four independent 8-byte loads each) a trip.
__device__ __forceinline__ uint32_t cmp_from(const MergeParams &M, uint32_t a, uint32_t b, uint32_t d, bool *a_less,
                                             uint64_t *lw, uint32_t *lv) {
    uint64_t sa, sb;
    uint32_t la, lb;
    str_ref(M, a, &sa, &la);
    str_ref(M, b, &sb, &lb);
    for (uint32_t l = d;; l += 32) {
        uint64_t ka[4], kb[4];
        ssd::keys32_at(M.S.chars, M.S.nchars, sa, la, l, ka);
        ssd::keys32_at(M.S.chars, M.S.nchars, sb, lb, l, kb);
        // the first word that differs or ends both strings (selects only:
        // no indexing of the word arrays by a computed index)
        uint32_t i = 4;
#pragma unroll
        for (int t = 3; t >= 0; --t)
            if (ka[t] != kb[t] || (ka[t] & 0xFF) == 0) i = (uint32_t)t;
        if (i == 4) continue;
        auto pick = [](const uint64_t *k, uint32_t j) -> uint64_t {
            return j == 0 ? k[0] : j == 1 ? k[1] : j == 2 ? k[2] : j == 3 ? k[3] : 0ull;
        };
        const uint64_t xa = pick(ka, i), xb = pick(kb, i);
        if (xa == xb) {   // both end in this word: equal strings
            *a_less = a < b;
            *lw = 0;   // past the end
            *lv = 8;
            return min(la, lb);
        }
        const bool al = xa < xb;
        *a_less = al;
        const uint32_t e = (uint32_t)(__clzll(xa ^ xb) >> 3);
        // the loser's 8 characters from the difference on
        const uint64_t w0 = al ? xb : xa;
        const uint64_t w1 = al ? pick(kb, i + 1) : pick(ka, i + 1);
        *lw = e ? (w0 << (8 * e)) | (w1 >> (64 - 8 * e)) : w0;
        *lv = (i + 1 < 4 || e == 0) ? 8u : 8u - e;
        return l + 8 * i + e;
    }
}

__device__ __forceinline__ uint32_t cmp_from(const MergeParams &M, uint32_t a, uint32_t b, uint32_t d, bool *a_less) {
    uint64_t w;
    uint32_t v;
    return cmp_from(M, a, b, d, a_less, &w, &v);
}

// 8 characters at the LCP position of every input element (the run's first
// element: at 0).
__global__ void k_mcache(MergeParams M) {
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < M.n; p += gridDim.x * blockDim.x) {
        bool first = false;
        for (uint32_t k = 0; k < M.K; ++k) first |= (M.rb[k] == p);
        // every later kernel reads strings through these indices: one outside
        // the set ends the merge with a device error (they check it first)
        if (M.pin[p] >= M.S.n || (!first && M.hin[p] > HMASK - 8)) {
            atomicOr(M.err, ssd::ERR_MERGE);
            M.cache[p] = 0;
            continue;
        }
        M.cache[p] = str_key(M, M.pin[p], first ? 0u : M.hin[p]);
    }
}

// Number of samples of run k below position c (samples sit at 0, g, 2g, ...).
__device__ __forceinline__ uint32_t samples_below(uint32_t c, uint32_t g) { return (c + g - 1) / g; }

// One lane per (sample, run): the lanes of a sample form a group of KP, the
// smallest power of two >= K, aligned inside the 64-wide wavefront.  Lane r
// finds the sample's cut in run r (lower bound of (string, index) with the
// LCP-accelerated binary search: the search keeps the LCPs of the sample with
// the elements just outside [lo, hi) and compares from their minimum); the
// group sums the samples below the cuts by shuffles into the sample's
// position in sample order, and lane r writes cut r of that row.
__global__ void k_msample(MergeParams M) {
    if (*M.err) return;
    uint32_t KP = 1;
    while (KP < M.K) KP <<= 1;
    const uint32_t gt = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t t = gt / KP;   // sample
    const uint32_t r = gt % KP;   // run this lane searches
    // which run and position: samples of run k are numbered from the
    // running total of earlier runs' samples
    bool live = t < M.nsamp;
    uint32_t k = 0, pos = 0, sid = 0;
    if (live) {
        uint32_t base = 0;
        for (; k < M.K; ++k) {
            const uint32_t c = samples_below(M.rb[k + 1] - M.rb[k], M.g);
            if (t < base + c) break;
            base += c;
        }
        live = k < M.K;
        if (live) {
            pos = (t - base) * M.g;
            sid = M.pin[M.rb[k] + pos];
        }
    }
    const bool mine = live && r < M.K;
    uint32_t c = 0;
    if (mine) {
        if (r == k) {
            c = pos;
        } else {
            const uint32_t *run = M.pin + M.rb[r];
            uint32_t lo = 0, hi = M.rb[r + 1] - M.rb[r], llo = 0, lhi = 0;
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                bool mid_less;
                const uint32_t l = cmp_from(M, run[mid], sid, min(llo, lhi), &mid_less);
                if (mid_less) {
                    lo = mid + 1;
                    llo = l;
                } else {
                    hi = mid;
                    lhi = l;
                }
            }
            c = lo;
        }
    }
    uint32_t order = mine ? samples_below(c, M.g) : 0u;
    for (uint32_t o = 1; o < KP; o <<= 1) order += (uint32_t)__shfl_xor((int)order, (int)o, 64);
    if (!mine) return;
    if (order >= M.nsamp) {
        atomicOr(M.err, ssd::ERR_MERGE);
        return;
    }
    M.cuts[(size_t)order * M.K + r] = c;
}

// Per-thread loser tree in LDS: node v (1..K-1) holds the loser's run, its
// string id, its LCP with the winner of that game, and its 8 characters at
// that LCP.  A loser's run does not advance while it sits in the tree, so the
// id stays valid there and the replay reads no run position from global
// memory.  KM, a power of two >= K, sizes the arrays: 28 * KM bytes per thread, so a
// tree sized for the launch's K (not the largest) keeps more workgroups
// resident per CU.
template <int KM>
struct MergeLDS {
    uint32_t y[KM][MNT];
    uint32_t yi[KM][MNT];   // string id of the loser's current element
    uint32_t h[KM][MNT];    // its LCP with the game's winner | valid cached characters << 24
    uint64_t c[KM][MNT];
    uint32_t pos[KM][MNT];   // next element of each run (absolute)
    uint32_t end[KM][MNT];
};

__device__ __forceinline__ uint32_t hv_pack(uint32_t h, uint32_t v) { return h | (v << 24); }

// One game (Algorithm 2 with cached characters): the candidate (x, hx, cx)
// against the node's loser (y, hy, cy), both with LCPs against the same
// smaller string p; hx and hy carry, above their LCP, how many of the cached
// characters (the word's leading bytes, taken at the LCP) are valid.  Returns
// true when the candidate wins; the loser's LCP with the winner (and its valid
// count) and its characters at that LCP end up in (lh, lc).  When the cached
// characters decide, the loser's word is shifted to its new LCP and keeps the
// rest of its valid characters, so the strings themselves are read only when
// every valid cached character is equal.
__device__ __forceinline__ bool game(const MergeParams &M, uint32_t x, uint32_t xid, uint32_t hx, uint64_t cx,
                                     uint32_t y, uint32_t yid, uint32_t hy, uint64_t cy, uint32_t *lh, uint64_t *lc) {
    if (y == SENT) {
        *lh = hy;
        *lc = cy;
        return true;
    }
    if (x == SENT) {
        *lh = hx;
        *lc = cx;
        return false;
    }
    const uint32_t lx = hx & HMASK, ly = hy & HMASK;
    if (lx > ly) {   // the candidate agrees longer with p: it is smaller
        *lh = hy;
        *lc = cy;
        return true;
    }
    if (lx < ly) {
        *lh = hx;
        *lc = cx;
        return false;
    }
    // equal LCPs: compare characters from there, the valid cached ones first
    const uint32_t m = min(hx >> 24, hy >> 24);   // characters valid in both words
    const uint64_t vm = m >= 8 ? ~0ull : ~(~0ull >> (8 * m));
    const uint64_t z = (cx ^ cy) & vm;
    bool x_less;
    uint32_t e;   // equal characters from the LCP on
    if (z) {
        x_less = (cx & vm) < (cy & vm);
        e = (uint32_t)(__clzll(z) >> 3);
    } else {
        // an end of string among the equal valid characters: identical strings
        uint32_t t = 0;
        while (t < m && ((cx >> (56 - 8 * t)) & 0xFF)) ++t;
        if (t < m) {
            x_less = xid < yid;
            e = t;
        } else {
            uint64_t lw;
            uint32_t lv;
            uint32_t l = cmp_from(M, xid, yid, lx + m, &x_less, &lw, &lv);
            if (l > HMASK - 8) {   // beyond the packed LCP range: a device error, never a wrong order
                atomicOr(M.err, ssd::ERR_MERGE);
                l = HMASK - 8;
            }
            *lh = hv_pack(l, lv);
            *lc = lw;
            return x_less;
        }
    }
    // the loser keeps its characters after the first e
    const uint64_t lold = x_less ? cy : cx;
    const uint32_t vold = (x_less ? hy : hx) >> 24;
    *lh = hv_pack(lx + e, vold - e);
    *lc = e ? lold << (8 * e) : lold;
    return x_less;
}

template <int KM>
__global__ __launch_bounds__(MNT) void k_mmerge(MergeParams M) {
    __shared__ MergeLDS<KM> L;
    if (*M.err) return;
    const int me = threadIdx.x;
    const uint32_t K = M.K;
    uint32_t KP = 1;
    while (KP < K) KP <<= 1;
    if (KP > (uint32_t)KM) {   // the host picked a tree too small for K
        atomicOr(M.err, ssd::ERR_MERGE);
        return;
    }
    // Jobs are claimed one at a time from a shared counter: their lengths
    // vary (about exponentially around g), and a wave that held one job per
    // lane would run as long as its longest job.
    for (;;) {
    const uint32_t j = (uint32_t)min(__hip_atomic_fetch_add(M.next_job, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                                     (unsigned long long)M.nsamp);
    if (j >= M.nsamp || *M.err) return;
    // this job: for each run, the elements between cut rows j and j+1; a
    // row the sample search left unwritten (two samples of the same rank:
    // runs that are not sorted by (string, index), or an index in two runs)
    // or cuts out of order end the merge with a device error, never an access
    uint32_t out = 0, len = 0;
    bool bad = false;
    for (uint32_t r = 0; r < KP; ++r) {
        if (r < K) {
            const uint32_t a = M.cuts[(size_t)j * K + r];
            const uint32_t b = (j + 1 < M.nsamp) ? M.cuts[(size_t)(j + 1) * K + r] : M.rb[r + 1] - M.rb[r];
            bad |= a == SENT || b == SENT || a > b || b > M.rb[r + 1] - M.rb[r];
            if (bad) break;
            L.pos[r][me] = M.rb[r] + a;
            L.end[r][me] = M.rb[r] + b;
            out += a;
            len += b - a;
        } else {
            L.pos[r][me] = L.end[r][me] = 0;
        }
    }
    // jobs tile the output: job 0 starts at 0 and job j+1 where job j ends,
    // so every output position is written once
    if (bad || (j == 0 && out != 0) || out > M.n || len > M.n - out) {
        atomicOr(M.err, ssd::ERR_MERGE);
        return;
    }
    // players: the runs' first elements of the job, LCP 0 against the empty
    // string.  The tree is built by inserting them one after the other: a
    // player climbs from its leaf, stops at the first node no player of the
    // other subtree has reached yet (it waits there), and otherwise plays
    // the waiting player, the loser staying at the node with its LCP against
    // the winner.  Inserted left to right, each subtree is complete when its
    // last player arrives, so every game is between the winners of two
    // subtrees, both with LCPs against the empty string; the player that
    // passes the root is the first winner.  Only the node arrays in LDS and
    // the climbing player's registers are used.
    for (uint32_t v = 1; v < KP; ++v) L.y[v][me] = WAITING;
    uint32_t w = SENT, hw = 0, wid = 0;
    for (uint32_t r = 0; r < KP; ++r) {
        uint32_t x = SENT, xid = 0, hx = 0;
        uint64_t cx = 0;
        if (r < K && L.pos[r][me] < L.end[r][me]) {
            x = r;
            xid = M.pin[L.pos[r][me]];
            hx = hv_pack(0, 8);
            cx = str_key(M, xid, 0);
        }
        bool waits = false;
        for (uint32_t v = (KP + r) >> 1; v >= 1; v >>= 1) {
            const uint32_t y = L.y[v][me];
            if (y == WAITING) {
                L.y[v][me] = x;
                L.yi[v][me] = xid;
                L.h[v][me] = hx;
                L.c[v][me] = cx;
                waits = true;
                break;
            }
            const uint32_t yid = L.yi[v][me];
            const uint32_t hy = L.h[v][me];
            const uint64_t cy = L.c[v][me];
            uint32_t lh;
            uint64_t lc;
            if (game(M, x, xid, hx, cx, y, yid, hy, cy, &lh, &lc)) {
                L.y[v][me] = y;
                L.yi[v][me] = yid;
            } else {
                L.y[v][me] = x;
                L.yi[v][me] = xid;
                x = y;
                xid = yid;
                hx = hy;
                cx = cy;
            }
            L.h[v][me] = lh;
            L.c[v][me] = lc;
        }
        if (!waits) {
            w = x;
            wid = xid;
            hw = hx;
        }
    }
    bool first = true;
    while (w != SENT) {
        const uint32_t p = L.pos[w][me];
        M.pout[out] = wid;
        if (!first && M.hout) M.hout[out] = hw & HMASK;
        first = false;
        ++out;
        // the winner's run advances; its next element's LCP with the string
        // just written is the run's own LCP entry, its cached characters too
        L.pos[w][me] = p + 1;
        uint32_t x = w, hx = 0;
        uint64_t cx = 0;
        uint32_t xid = 0;
        if (p + 1 < L.end[w][me]) {
            hx = hv_pack(M.hin[p + 1], 8);
            cx = M.cache[p + 1];
            xid = M.pin[p + 1];
        } else {
            x = SENT;
        }
        for (uint32_t v = (KP + w) >> 1; v >= 1; v >>= 1) {
            const uint32_t y = L.y[v][me];
            const uint32_t yid = L.yi[v][me];
            uint32_t lh;
            uint64_t lc;
            const bool xw = game(M, x, xid, hx, cx, y, yid, L.h[v][me], L.c[v][me], &lh, &lc);
            if (!xw) {
                L.y[v][me] = x;
                L.yi[v][me] = xid;
                x = y;
                xid = yid;
                hx = L.h[v][me];
                cx = L.c[v][me];
            } else {
                L.y[v][me] = y;
            }
            L.h[v][me] = lh;
            L.c[v][me] = lc;
        }
        w = x;
        wid = xid;
        hw = hx;
    }
    }
}

// LCP between the first output of each job and the string before it (after
// k_mmerge has checked every cut row: it runs only without a device error).
__global__ void k_mseam(MergeParams M) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M.nsamp || *M.err) return;
    uint32_t q = 0;
    for (uint32_t r = 0; r < M.K; ++r) q += M.cuts[(size_t)j * M.K + r];
    uint32_t qe = M.n;
    if (j + 1 < M.nsamp) {
        qe = 0;
        for (uint32_t r = 0; r < M.K; ++r) qe += M.cuts[(size_t)(j + 1) * M.K + r];
    }
    if (q >= qe || qe > M.n) return;
    if (q == 0) {
        M.hout[0] = 0;
        return;
    }
    bool less;
    M.hout[q] = cmp_from(M, M.pout[q - 1], M.pout[q], 0, &less);
}

// Clear the error word and mark every cut row unwritten (a kernel, not a
// memset, so that a captured graph holds no memset node).
__global__ void k_mreset(MergeParams M) {
    const size_t total = (size_t)(M.nsamp + 1) * M.K;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x)
        M.cuts[i] = SENT;
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *M.err = 0;
        *M.next_job = 0;
    }
}

}  // namespace ssm

