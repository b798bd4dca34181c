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
// the elements between two consecutive cuts); long jobs are split again at
// elements of their longest run.  A thread merges one job at a time with an
// LCP-aware loser tree whose nodes cache the 8 characters of their string at
// the node's LCP (the paper caches the one distinguishing character; eight
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
constexpr uint32_t NOREF = 0xFFFFFFFFu;   // a cut's LCP with its row's string is not available

__device__ __forceinline__ uint32_t hv_pack(uint32_t h, uint32_t v) { return h | (v << 24); }

// An input element as the merge reads it: its string (index, start,
// length), its LCP with the run's previous element and the 8 characters at
// that LCP, in one 32-byte entry, so that a lane advancing through K runs
// streams through K arrays instead of 3K.
struct __align__(32) MEnt {
    uint64_t c;              // 8 characters at the LCP (the run's first element: at 0)
    uint64_t st;
    uint32_t id, h, ln, pad;
};

struct MergeParams {
    Strs S;
    uint32_t rb[MKMAX + 1];  // run boundaries
    const uint32_t *pin;     // runs of string indices
    const uint32_t *hin;     // their LCP arrays (entry at a run's start ignored)
    uint32_t *pout, *hout;
    MEnt *ent;               // per input element, everything a merge step reads
    uint32_t *cuts;          // rows of K cuts: nsamp in sample order, the run ends, then the split rows
    // per cut: the LCP of the element at the cut with the row's string (the
    // sample or split element) and the valid count packed as in the tree, or
    // NOREF; and that element's characters at the LCP
    uint32_t *cuth;
    uint64_t *cutc;
    uint32_t *ja, *jb;       // merge jobs: from cut row ja[s] to cut row jb[s]
    uint32_t *xd;            // per split row: its job, the job's longest run, the split element's place there
    unsigned long long *err;
    unsigned long long *next_job;   // next merge job to claim
    unsigned long long *nsplit;     // split rows handed out
    uint32_t K, n, g, nsamp;
    uint32_t lcap;           // jobs longer than this are split
    uint32_t xcap;           // split rows the workspace holds (n / lcap + 1)
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

// 64 characters of a string from depth h as raw words (the first character
// in the low byte of w[0]), loaded from the at most nine aligned words that
// hold them; *rem: the characters the string has from h (bytes of w past
// them are not the string's).
__device__ __forceinline__ void raw64(const uint8_t *chars, uint64_t nchars, uint64_t st, uint32_t ln, uint32_t h,
                                      uint64_t w[8], uint32_t *rem) {
#pragma unroll
    for (int j = 0; j < 8; ++j) w[j] = 0;
    *rem = 0;
    if (h >= ln) return;
    const uint64_t p = st + h;
    if (p >= nchars) return;
    const uint32_t r = (uint32_t)min((uint64_t)(ln - h), nchars - p);
    *rem = r;
    const uint32_t sh = (uint32_t)((uintptr_t)(chars + p) & 7);
    const uint64_t *a0 = reinterpret_cast<const uint64_t *>(chars + (p - sh));
    const uint32_t nw = (sh + min(r, 64u) + 7) >> 3;   // words holding wanted bytes, 1..9
    uint64_t a[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) a[i] = (uint32_t)i < nw ? a0[i] : 0ull;
#pragma unroll
    for (int j = 0; j < 8; ++j) w[j] = sh ? (a[j] >> (8 * sh)) | (a[j + 1] << (64 - 8 * sh)) : a[j];
}

// Compare strings a and b (located at sa, sb with lengths la, lb) that agree
// on [0, d): returns their LCP and whether a < b (equal strings: by index),
// and in *lw the loser's characters at the LCP (the word's leading *lv of them
// valid), taken from the bytes just compared.  64 characters of each string a
// trip, compared as raw words (equality needs no byte order): only the first
// differing word and the loser's new word are put in character order.
__device__ __forceinline__ uint32_t cmp_at(const MergeParams &M, uint32_t a, uint64_t sa, uint32_t la, uint32_t b,
                                           uint64_t sb, uint32_t lb, uint32_t d, bool *a_less, uint64_t *lw,
                                           uint32_t *lv) {
    // word j of a window (selects only: no indexing of the word arrays by a
    // computed index); 0 past the window
    auto pick = [](const uint64_t *k, uint32_t j) -> uint64_t {
        uint64_t r = 0;
#pragma unroll
        for (int t = 0; t < 8; ++t) r = j == (uint32_t)t ? k[t] : r;
        return r;
    };
    for (uint32_t l = d;; l += 64) {
        uint64_t A[8], B[8];
        uint32_t ra, rb;
        raw64(M.S.chars, M.S.nchars, sa, la, l, A, &ra);
        raw64(M.S.chars, M.S.nchars, sb, lb, l, B, &rb);
        const uint32_t m = min(min(ra, rb), 64u);   // characters both have in the window
        // the first word with a difference among them
        uint32_t i = 8;
        uint64_t z = 0;
#pragma unroll
        for (int t = 7; t >= 0; --t) {
            const int r = (int)m - 8 * t;
            const uint64_t mk = r >= 8 ? ~0ull : r <= 0 ? 0ull : ~0ull >> (64 - 8 * r);
            const uint64_t zt = (A[t] ^ B[t]) & mk;
            if (zt) {
                i = (uint32_t)t;
                z = zt;
            }
        }
        uint32_t pos;
        bool al;
        if (i < 8) {
            const uint32_t bit = (uint32_t)__builtin_ctzll(z) & ~7u;
            pos = 8 * i + (bit >> 3);
            al = ((pick(A, i) >> bit) & 0xFF) < ((pick(B, i) >> bit) & 0xFF);
        } else if (m < 64) {
            // one string ends inside the window with no difference before
            if (ra == rb) {   // both: equal strings
                *a_less = a < b;
                *lw = 0;   // past the end
                *lv = 8;
                return l + m;
            }
            al = ra < rb;   // the shorter is a prefix of the longer
            pos = m;
        } else {
            continue;
        }
        *a_less = al;
        // the loser's 8 characters from pos (it has at least one there), zero
        // past its end; those past the window are unknown unless it ends
        // inside the window
        const uint32_t rl = al ? rb : ra;
        const uint32_t j0 = pos >> 3, o = pos & 7;
        const uint64_t u0 = al ? pick(B, j0) : pick(A, j0);
        const uint64_t u1 = al ? pick(B, j0 + 1) : pick(A, j0 + 1);
        uint64_t raw = o ? (u0 >> (8 * o)) | (u1 << (64 - 8 * o)) : u0;
        const uint32_t left = rl - pos;
        if (left < 8) raw &= ~0ull >> (64 - 8 * left);
        *lw = __builtin_bswap64(raw);
        *lv = (rl <= 64 || pos + 8 <= 64) ? 8u : 64u - pos;
        return l + pos;
    }
}

// LCP of the strings with indices a and b, compared 32 characters (four
// big-endian 8-byte keys, zero past the end) a trip.
__device__ __forceinline__ uint32_t lcp_of(const MergeParams &M, uint32_t a, uint32_t b) {
    uint64_t sa, sb;
    uint32_t la, lb;
    str_ref(M, a, &sa, &la);
    str_ref(M, b, &sb, &lb);
    for (uint32_t l = 0;; l += 32) {
        uint64_t ka[4], kb[4];
        ssd::keys32_at(M.S.chars, M.S.nchars, sa, la, l, ka);
        ssd::keys32_at(M.S.chars, M.S.nchars, sb, lb, l, kb);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (ka[t] != kb[t]) return l + 8 * t + (uint32_t)(__clzll(ka[t] ^ kb[t]) >> 3);
            if ((ka[t] & 0xFF) == 0) return min(la, lb);   // both end in this word: equal strings
        }
    }
}

// 8 characters at the LCP position of every input element (the run's first
// element: at 0), and its string's start, length and index.
__global__ void k_mcache(MergeParams M) {
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < M.n; p += gridDim.x * blockDim.x) {
        bool first = false;
        for (uint32_t k = 0; k < M.K; ++k) first |= (M.rb[k] == p);
        // every later kernel reads strings through these indices: one outside
        // the set ends the merge with a device error (they check it first)
        if (M.pin[p] >= M.S.n || (!first && M.hin[p] > HMASK - 8)) {
            atomicOr(M.err, ssd::ERR_MERGE);
            continue;
        }
        uint64_t st;
        uint32_t ln;
        const uint32_t id = M.pin[p], h = first ? 0u : M.hin[p];
        str_ref(M, id, &st, &ln);
        MEnt e;
        e.c = key_at(M.S.chars, M.S.nchars, st, ln, h);
        e.st = st;
        e.id = id;
        e.h = h;
        e.ln = ln;
        e.pad = 0;
        M.ent[p] = e;
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
    uint32_t k = 0, pos = 0;
    MEnt sr;
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
            sr = M.ent[M.rb[k] + pos];
        }
    }
    const bool mine = live && r < M.K;
    uint32_t c = 0, ch = NOREF;
    uint64_t cc = 0;
    if (mine) {
        if (r == k) {
            c = pos;
            if (sr.ln <= HMASK - 8) ch = hv_pack(sr.ln, 8);   // the sample itself: its whole length, then the end
        } else {
            // first among run r's own samples (every g-th element: few, and
            // shared by every search of the run, so they stay in the
            // caches), then inside the one sample interval that holds the
            // cut; the LCPs with the bracketing elements carry over
            const MEnt *run = M.ent + M.rb[r];
            const uint32_t len = M.rb[r + 1] - M.rb[r];
            uint32_t llo = 0, lhi = 0, vhi = 0;
            uint64_t whi = 0;
            uint32_t slo = 0, shi = samples_below(len, M.g);
            while (slo < shi) {
                const uint32_t mid = (slo + shi) >> 1;
                bool mid_less;
                const MEnt &rm = run[(size_t)mid * M.g];
                uint64_t lw;
                uint32_t lv;
                const uint32_t l = cmp_at(M, rm.id, rm.st, rm.ln, sr.id, sr.st, sr.ln, min(llo, lhi), &mid_less, &lw, &lv);
                if (mid_less) {
                    slo = mid + 1;
                    llo = l;
                } else {
                    shi = mid;
                    lhi = l;
                    whi = lw;
                    vhi = lv;
                }
            }
            // slo samples are below: the elements up to sample slo - 1 are,
            // sample slo (if any) is not
            uint32_t lo = slo ? (slo - 1) * M.g + 1 : 0u;
            uint32_t hi = min(slo * M.g, len);
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                bool mid_less;
                const MEnt &rm = run[mid];
                uint64_t lw;
                uint32_t lv;
                const uint32_t l = cmp_at(M, rm.id, rm.st, rm.ln, sr.id, sr.st, sr.ln, min(llo, lhi), &mid_less, &lw, &lv);
                if (mid_less) {
                    lo = mid + 1;
                    llo = l;
                } else {
                    // the element is the larger: its characters at the LCP
                    hi = mid;
                    lhi = l;
                    whi = lw;
                    vhi = lv;
                }
            }
            c = lo;
            // the element at the cut was compared last when hi came down to it
            if (c < M.rb[r + 1] - M.rb[r] && lhi <= HMASK - 8) {
                ch = hv_pack(lhi, vhi);
                cc = whi;
            }
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
    M.cuth[(size_t)order * M.K + r] = ch;
    M.cutc[(size_t)order * M.K + r] = cc;
}

// Jobs between consecutive samples vary in length (about exponentially
// around g, the longest several times g), and the merge takes about as long
// as its lanes' share of the work plus the longest job: a job longer than
// lcap is split into p = ceil(len / lcap)
// parts at elements of its longest run (evenly spaced in that run's range),
// each element's cut in every other run found by the same LCP-accelerated
// binary search as the samples', inside the job's range.  One lane group of
// KP lanes per job, lane r for run r.  The job list: job j is rows (j, j+1)
// unsplit, else (j, x_1), (x_1, x_2), ..., (x_{p-1}, j+1) with the split rows
// x_t taken from a shared counter; row nsamp holds the run ends.
constexpr int SPLIT_NT = 256;   // threads per k_msplit workgroup
// (No early exit on an earlier device error: every thread reaches the
// workgroup's barriers, and the rows it reads are in bounds whatever they
// hold; the merge does not run after an error.)
__global__ __launch_bounds__(SPLIT_NT) void k_msplit(MergeParams M) {
    uint32_t KP = 1;
    while (KP < M.K) KP <<= 1;
    const uint32_t gt = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t j = gt / KP, r = gt % KP;
    const bool live = j < M.nsamp;
    const bool mine = live && r < M.K;
    const uint32_t K = M.K;
    if (j == 0 && mine) M.cuts[(size_t)M.nsamp * K + r] = M.rb[r + 1] - M.rb[r];
    uint32_t a = 0, b = 0;
    bool bad = false;
    if (mine) {
        a = M.cuts[(size_t)j * K + r];
        b = (j + 1 < M.nsamp) ? M.cuts[(size_t)(j + 1) * K + r] : M.rb[r + 1] - M.rb[r];
        bad = a == SENT || b == SENT || a > b || b > M.rb[r + 1] - M.rb[r];
    }
    // the group's job length and its longest run (lowest run on ties)
    uint32_t d = (mine && !bad) ? min(b - a, 1u << 26) : 0u;
    uint32_t len = d;
    uint32_t best = (d << 5) | (31u - (r & 31u));
    for (uint32_t o = 1; o < KP; o <<= 1) {
        len += (uint32_t)__shfl_xor((int)len, (int)o, 64);
        best = max(best, (uint32_t)__shfl_xor((int)best, (int)o, 64));
    }
    uint32_t nbad = bad ? 1u : 0u;
    for (uint32_t o = 1; o < KP; o <<= 1) nbad += (uint32_t)__shfl_xor((int)nbad, (int)o, 64);
    const uint32_t rs = 31u - (best & 31u), ds = best >> 5;
    uint32_t parts = (len + M.lcap - 1) / M.lcap;
    parts = min(parts, ds);   // split elements distinct in the longest run
    if (!live || nbad) parts = 0;   // (a bad row is reported by the merge, which checks every row)
    // split rows for the workgroup's jobs with one atomic (one per job, or
    // per wave, serialise by the ten thousand on the counter): an exclusive
    // prefix sum of the group leaders' counts, per wave by shuffles, then
    // over the waves in LDS
    __shared__ uint32_t wsum[SPLIT_NT / 64];
    __shared__ unsigned long long bbase;
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    const uint32_t mycnt = (r == 0 && parts > 1) ? parts - 1 : 0u;
    uint32_t incl = mycnt;
    for (uint32_t o = 1; o < 64; o <<= 1) {
        const uint32_t v = (uint32_t)__shfl_up((int)incl, o, 64);
        if (lane >= o) incl += v;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    uint32_t before = 0, total = 0;
    for (uint32_t u = 0; u < SPLIT_NT / 64; ++u) {
        const uint32_t t = wsum[u];
        before += u < wv ? t : 0u;
        total += t;
    }
    if (threadIdx.x == 0)
        bbase = total ? __hip_atomic_fetch_add(M.nsplit, (unsigned long long)total, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT)
                      : 0ull;
    __syncthreads();
    const unsigned long long wbase = bbase + before;
    const uint32_t excl = (uint32_t)__shfl((int)(incl - mycnt), (int)(lane & ~(KP - 1)), 64);
    if (!live) return;
    if (parts <= 1) {
        // unsplit
        if (r == 0) {
            M.ja[j] = j;
            M.jb[j] = j + 1;
        }
        return;
    }
    const unsigned long long x0 = wbase + excl;
    if (x0 + parts - 1 > M.xcap) {
        if (r == 0) atomicOr(M.err, ssd::ERR_MERGE);
        return;
    }
    const uint32_t row0 = M.nsamp + 1 + (uint32_t)x0;   // split row of part 1
    const uint32_t a_s = __shfl((int)a, (int)((threadIdx.x & 63u & ~(KP - 1)) + rs), 64);
    // the split elements' places in run rs; their cuts are searched by
    // k_msplit_rows, one lane group per split row
    for (uint32_t t = 1 + r; t < parts; t += KP) {
        uint32_t *x = M.xd + 3 * (size_t)(x0 + t - 1);
        x[0] = j;
        x[1] = rs;
        x[2] = a_s + (uint32_t)(((uint64_t)t * ds) / parts);
    }
    if (r == 0) {
        M.ja[j] = j;
        M.jb[j] = row0;
        for (uint32_t t = 1; t < parts; ++t) {
            const uint32_t s = M.nsamp + (uint32_t)x0 + t - 1;   // job slot of part t + 1
            M.ja[s] = row0 + t - 1;
            M.jb[s] = t + 1 < parts ? row0 + t : j + 1;
        }
    }
}

// The cuts of every split row: lane r of the row's group finds, inside the
// row's job, the lower bound of the split element in run r (in run rs, the
// split element itself), with the element's LCP with it and its characters
// there, as the sample search does.
__global__ void k_msplit_rows(MergeParams M) {
    if (*M.err) return;
    uint32_t KP = 1;
    while (KP < M.K) KP <<= 1;
    const uint32_t gt = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t x = gt / KP, r = gt % KP;
    const uint32_t nx = (uint32_t)min(*M.nsplit, (unsigned long long)M.xcap);
    if (x >= nx || r >= M.K) return;
    const uint32_t K = M.K;
    const uint32_t j = M.xd[3 * (size_t)x], rs = M.xd[3 * (size_t)x + 1], sp = M.xd[3 * (size_t)x + 2];
    if (j >= M.nsamp || rs >= K || sp >= M.rb[rs + 1] - M.rb[rs]) {
        atomicOr(M.err, ssd::ERR_MERGE);
        return;
    }
    const uint32_t a = M.cuts[(size_t)j * K + r];
    const uint32_t b = (j + 1 < M.nsamp) ? M.cuts[(size_t)(j + 1) * K + r] : M.rb[r + 1] - M.rb[r];
    if (a == SENT || b == SENT || a > b || b > M.rb[r + 1] - M.rb[r]) {
        atomicOr(M.err, ssd::ERR_MERGE);
        return;
    }
    const MEnt sr = M.ent[M.rb[rs] + sp];
    uint32_t c, ch = NOREF;
    uint64_t cc = 0;
    if (r == rs) {
        c = sp;
        if (sr.ln <= HMASK - 8) ch = hv_pack(sr.ln, 8);
    } else {
        const MEnt *run = M.ent + M.rb[r];
        uint32_t lo = a, hi = b, llo = 0, lhi = 0, vhi = 0;
        uint64_t whi = 0;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            bool mid_less;
            const MEnt &rm = run[mid];
            uint64_t lw;
            uint32_t lv;
            const uint32_t l = cmp_at(M, rm.id, rm.st, rm.ln, sr.id, sr.st, sr.ln, min(llo, lhi), &mid_less, &lw, &lv);
            if (mid_less) {
                lo = mid + 1;
                llo = l;
            } else {
                hi = mid;
                lhi = l;
                whi = lw;
                vhi = lv;
            }
        }
        c = lo;
        // (below b the element at the cut was compared: hi came down to it)
        if (c < b && lhi <= HMASK - 8) {
            ch = hv_pack(lhi, vhi);
            cc = whi;
        }
    }
    const size_t q = (size_t)(M.nsamp + 1 + x) * K + r;
    M.cuts[q] = c;
    M.cuth[q] = ch;
    M.cutc[q] = cc;
}

// Per-thread loser tree in LDS: node v (1..K-1) holds the loser's run, its
// string index, its LCP with the winner of that game, and its 8 characters at
// that LCP; per run, the position of its element in the tree (or climbing).
// A loser's run does not advance while it sits in the tree, so its element
// is the entry at its run's position: the replay reads no run position from
// global memory, and a game that compares strings reads both strings'
// entries there.  The end of a run's part of the job comes from the job's
// upper cut row (a cached read beside the next entry's).  KM, a power of two
// >= K, sizes the arrays: 24 * KM bytes per thread, so that a tree sized for
// the launch's K (not the largest) keeps more workgroups resident per CU.
template <int KM>
struct MergeLDS {
    uint32_t y[KM][MNT];
    uint32_t yi[KM][MNT];   // string id of the loser's current element
    uint32_t h[KM][MNT];    // its LCP with the game's winner | valid cached characters << 24
    uint64_t c[KM][MNT];
    uint32_t pos[KM][MNT];   // each run's element in the tree (absolute position)
};

// One game (Algorithm 2 with cached characters): the candidate (x, hx, cx)
// against the node's loser (y, hy, cy), both with LCPs against the same
// smaller string p; hx and hy carry, above their LCP, how many of the cached
// characters (the word's leading bytes, taken at the LCP) are valid.  Returns
// true when the candidate wins; the loser's LCP with the winner (and its valid
// count) and its characters at that LCP end up in (lh, lc).  When the cached
// characters decide, the loser's word is shifted to its new LCP and keeps the
// rest of its valid characters, so the strings themselves are read only when
// every valid cached character is equal.
// The part of a game decided without reading the strings: returns 0 when
// the candidate wins, 1 when it loses (the loser's LCP and characters in
// (lh, lc)), 2 when every valid cached character is equal and the strings
// must be compared from *from on.
__device__ __forceinline__ int game_pre(uint32_t x, uint32_t xid, uint32_t hx, uint64_t cx, uint32_t y, uint32_t yid,
                                        uint32_t hy, uint64_t cy, uint32_t *lh, uint64_t *lc, uint32_t *from) {
    if (y == SENT) {
        *lh = hy;
        *lc = cy;
        return 0;
    }
    if (x == SENT) {
        *lh = hx;
        *lc = cx;
        return 1;
    }
    const uint32_t lx = hx & HMASK, ly = hy & HMASK;
    if (lx > ly) {   // the candidate agrees longer with p: it is smaller
        *lh = hy;
        *lc = cy;
        return 0;
    }
    if (lx < ly) {
        *lh = hx;
        *lc = cx;
        return 1;
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
            *from = lx + m;
            return 2;
        }
    }
    // the loser keeps its characters after the first e
    const uint64_t lold = x_less ? cy : cx;
    const uint32_t vold = (x_less ? hy : hx) >> 24;
    *lh = hv_pack(lx + e, vold - e);
    *lc = e ? lold << (8 * e) : lold;
    return x_less ? 0 : 1;
}

// The strings' part, for the elements at input positions px and py: compare
// from `from` on (Algorithm 2 with the LCP found).
__device__ __forceinline__ bool game_str(const MergeParams &M, uint32_t px, uint32_t py, uint32_t from, uint32_t *lh,
                                         uint64_t *lc) {
    const MEnt a = M.ent[px], b = M.ent[py];
    bool x_less;
    uint64_t lw;
    uint32_t lv;
    uint32_t l = cmp_at(M, a.id, a.st, a.ln, b.id, b.st, b.ln, from, &x_less, &lw, &lv);
    if (l > HMASK - 8) {   // beyond the packed LCP range: a device error, never a wrong order
        atomicOr(M.err, ssd::ERR_MERGE);
        l = HMASK - 8;
    }
    *lh = hv_pack(l, lv);
    *lc = lw;
    return x_less;
}

// A whole game between runs x and y (their elements at px, py): true when
// the candidate wins.
__device__ __forceinline__ bool game(const MergeParams &M, uint32_t x, uint32_t xid, uint32_t px, uint32_t hx,
                                     uint64_t cx, uint32_t y, uint32_t yid, uint32_t py, uint32_t hy, uint64_t cy,
                                     uint32_t *lh, uint64_t *lc) {
    uint32_t from = 0;
    const int d = game_pre(x, xid, hx, cx, y, yid, hy, cy, lh, lc, &from);
    if (d != 2) return d == 0;
    return game_str(M, px, py, from, lh, lc);
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
    // Jobs are claimed one at a time from a shared counter, and a lane that
    // finishes its job claims the next one inside the same loop (lanes that
    // merged their jobs in lockstep would hold their wave for its longest
    // job each time).  The candidate climbs the tree with the part of each
    // game that needs no string; a lane whose game needs the strings stops
    // at that node, and the comparison runs once per iteration for every
    // lane stopped (inside the climb it would run, for the few lanes that
    // need it, at every level, with the wave's other lanes waiting); the lane
    // goes on climbing in the next iteration.
    uint32_t out = 0;              // next output position of the lane's job
    // the candidate: its run x (SENT: exhausted), string, LCP with the last
    // output (and valid count) and cached characters; v: the node it plays
    // next, 0 once it has passed the root (it is the next output)
    uint32_t x = SENT, xid = 0, hx = 0, v = 0;
    uint64_t cx = 0;
    bool first = true;             // the next output is its job's first
    uint32_t jrow = 0;             // the job's upper cut row
    // end (absolute position) of run r's part of the job
    auto run_end = [&](uint32_t r) -> uint32_t { return M.rb[r] + M.cuts[(size_t)jrow * K + r]; };
    for (;;) {
    if (v == 0) {
    if (x == SENT) {
    // the job is done (or none was claimed yet): the next one
    const uint32_t njobs = M.nsamp + (uint32_t)min(*M.nsplit, (unsigned long long)M.xcap);
    // the lanes that need a job in this iteration claim consecutive ones
    // with one atomic (a counter that every lane hit on its own would
    // serialise over a hundred thousand of them at the start)
    const uint64_t need = __ballot(1);
    const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(need >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)need, 0u));
    const int lead = __builtin_ctzll(need);
    unsigned long long base = 0;
    if (rank == 0)
        base = __hip_atomic_fetch_add(M.next_job, (unsigned long long)__popcll(need), __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
    base = (unsigned long long)__shfl((long long)base, lead, 64);
    const uint32_t j = (uint32_t)min(base + rank, (unsigned long long)njobs);
    if (j >= njobs || *M.err) return;
    // this job: for each run, the elements between its two cut rows; a
    // row the sample search left unwritten (two samples of the same rank:
    // runs that are not sorted by (string, index), or an index in two runs)
    // or cuts out of order end the merge with a device error, never an access
    const uint32_t ra = M.ja[j], rb = M.jb[j];
    if (ra > M.nsamp + M.xcap || rb > M.nsamp + M.xcap) {
        atomicOr(M.err, ssd::ERR_MERGE);
        return;
    }
    uint32_t len = 0;
    out = 0;
    bool bad = false;
    for (uint32_t r = 0; r < KP; ++r) {
        if (r < K) {
            const uint32_t a = M.cuts[(size_t)ra * K + r];
            const uint32_t b = M.cuts[(size_t)rb * K + r];
            bad |= a == SENT || b == SENT || a > b || b > M.rb[r + 1] - M.rb[r];
            if (bad) break;
            L.pos[r][me] = M.rb[r] + a;
            out += a;
            len += b - a;
        } else {
            L.pos[r][me] = 0;
        }
    }
    jrow = rb;
    // jobs tile the output: job 0 starts at 0 and every other job where
    // another one ends, so every output position is written once
    if (bad || (j == 0 && out != 0) || out > M.n || len > M.n - out) {
        atomicOr(M.err, ssd::ERR_MERGE);
        return;
    }
    // players: the runs' first elements of the job, with their LCPs against
    // a string no larger than any of them (Algorithm 4 starts from the empty
    // string): the job's lower row's string (its sample or split element),
    // whose LCP with each cut element the search that placed the cut found,
    // with the element's characters there, so that the first games are
    // decided like the later ones, mostly without reading the strings; when
    // one of them is missing (a string too long for the packed LCP), the
    // empty string for every player.  The tree is built by inserting them
    // one after the other: a player climbs from its leaf, stops at the first
    // node no player of the other subtree has reached yet (it waits there),
    // and otherwise plays the waiting player, the loser staying at the node
    // with its LCP against the winner.  Inserted left to right, each subtree
    // is complete when its last player arrives, so every game is between the
    // winners of two subtrees, both with LCPs against the same string; the
    // player that passes the root is the first winner.  Only the node arrays
    // in LDS and the climbing player's registers are used.
    bool ref = true;
    for (uint32_t r = 0; r < K; ++r)
        if (L.pos[r][me] < run_end(r) && M.cuth[(size_t)ra * K + r] == NOREF) ref = false;
    for (uint32_t u = 1; u < KP; ++u) L.y[u][me] = WAITING;
    uint32_t wn = SENT, widn = 0, hwn = 0;   // the first winner
    for (uint32_t r = 0; r < KP; ++r) {
        uint32_t x = SENT, xid = 0, hx = 0;
        uint64_t cx = 0;
        if (r < K && L.pos[r][me] < run_end(r)) {
            const MEnt &e = M.ent[L.pos[r][me]];
            x = r;
            xid = e.id;
            if (ref) {
                hx = M.cuth[(size_t)ra * K + r];
                cx = M.cutc[(size_t)ra * K + r];
            } else {
                hx = hv_pack(0, 8);
                cx = key_at(M.S.chars, M.S.nchars, e.st, e.ln, 0);
            }
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
            // (a string comparison only between two live players: sentinels
            // are decided first)
            const uint32_t px = x < K ? L.pos[x][me] : 0u, py = y < K ? L.pos[y][me] : 0u;
            if (!game(M, x, xid, px, hx, cx, y, yid, py, hy, cy, &lh, &lc)) {
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
            wn = x;
            widn = xid;
            hwn = hx;
        }
    }
    x = wn;
    xid = widn;
    hx = hwn;
    first = true;
    continue;   // an empty job leaves x = SENT: claim the next
    }
    // output the candidate; its run's next element climbs from the leaf: its
    // LCP with the string just written is the run's own LCP entry, its
    // cached characters too
    const uint32_t run = x;
    const uint32_t p = L.pos[run][me];
    M.pout[out] = xid;
    if (!first && M.hout) M.hout[out] = hx & HMASK;
    first = false;
    ++out;
    L.pos[run][me] = p + 1;
    if (p + 1 < run_end(run)) {
        const MEnt e = M.ent[p + 1];
        xid = e.id;
        hx = hv_pack(e.h, 8);
        cx = e.c;
    } else {
        x = SENT;
    }
    v = (KP + run) >> 1;
    }
    // climb while the games need no string
    uint32_t from = 0;
    bool stop = false;
    while (v >= 1) {
        const uint32_t y = L.y[v][me], yid = L.yi[v][me];
        const uint32_t hy = L.h[v][me];
        const uint64_t cy = L.c[v][me];
        uint32_t lh;
        uint64_t lc;
        const int d = game_pre(x, xid, hx, cx, y, yid, hy, cy, &lh, &lc, &from);
        if (d == 2) {
            stop = true;
            break;
        }
        if (d == 1) {
            L.y[v][me] = x;
            L.yi[v][me] = xid;
            x = y;
            xid = yid;
            hx = hy;
            cx = cy;
        }
        L.h[v][me] = lh;
        L.c[v][me] = lc;
        v >>= 1;
    }
    if (stop) {
        // the game at node v compares the strings
        // (both runs live: a sentinel never needs the strings)
        const uint32_t y = L.y[v][me], yid = L.yi[v][me];
        const uint32_t hy = L.h[v][me];
        const uint64_t cy = L.c[v][me];
        uint32_t lh;
        uint64_t lc;
        if (!game_str(M, L.pos[x][me], L.pos[y][me], from, &lh, &lc)) {
            L.y[v][me] = x;
            L.yi[v][me] = xid;
            x = y;
            xid = yid;
            hx = hy;
            cx = cy;
        }
        L.h[v][me] = lh;
        L.c[v][me] = lc;
        v >>= 1;
    }
    }
}

// LCP between the first output of each job and the string before it (after
// k_mmerge has checked every job's cut rows: it runs only without a device
// error).
__global__ void k_mseam(MergeParams M) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (*M.err) return;
    const uint32_t njobs = M.nsamp + (uint32_t)min(*M.nsplit, (unsigned long long)M.xcap);
    if (j >= njobs) return;
    const uint32_t ra = M.ja[j], rb = M.jb[j];
    uint32_t q = 0, qe = 0;
    for (uint32_t r = 0; r < M.K; ++r) {
        q += M.cuts[(size_t)ra * M.K + r];
        qe += M.cuts[(size_t)rb * M.K + r];
    }
    if (q >= qe || qe > M.n) return;
    if (q == 0) {
        M.hout[0] = 0;
        return;
    }
    M.hout[q] = lcp_of(M, M.pout[q - 1], M.pout[q]);
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
        *M.nsplit = 0;
    }
}

}  // namespace ssm

