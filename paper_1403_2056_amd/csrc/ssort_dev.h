// Device-side building blocks of the string sample sorter (gfx950, wave64).
//
// Notation follows Algorithm 1 (one step of super scalar string sample sort):
// a segment of strings with common prefix h is classified by the 8 characters
// at depth h (w = 8), packed big-endian into one uint64 so that one unsigned
// compare orders 8 characters; v = 2^d - 1 splitters x_0 < ... < x_{v-1} form
// a perfect search tree held in LDS in level order; bucket 2l holds keys
// strictly between x_{l-1} and x_l, bucket 2l+1 keys equal to x_l.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ssd {

constexpr int NT = 256;                 // threads per workgroup
constexpr int NW = NT / 64;             // waves per workgroup
constexpr int VMAX = 255;               // largest splitter count (d = 8)
constexpr int DMAX = 8;
constexpr int NBMAX = 2 * VMAX + 1;     // 511 buckets
constexpr int NBPAD = 512;
constexpr int SAMPLE_MAX = 2 * (VMAX + 1) - 1;   // oversampling factor 2
constexpr int CH = 1024;                // base-case chunk (strings held in LDS)
#ifndef SSD_ROOT_CHUNKS
#define SSD_ROOT_CHUNKS 4
#endif
constexpr int ROOT_CHUNKS = SSD_ROOT_CHUNKS;   // chunks of NT*K strings per whole-GPU level tile
constexpr uint32_t SEAM = 0x80000000u;  // lcp slot still holds a separation depth
constexpr uint32_t TO_END = 1u;

// One string reference: start offset, length, input index.
struct __align__(16) Rec {
    uint64_t st;
    uint32_t ln;
    uint32_t id;
};

struct Strs {
    const uint8_t *chars;
    uint64_t nchars;
    const uint64_t *off;
    const uint32_t *len;
    uint32_t n;
    uint32_t flags;
};

__device__ __forceinline__ Rec make_rec(const Strs &S, uint32_t i) {
    Rec r;
    r.st = S.off[i];
    r.id = i;
    if (S.flags & TO_END) r.ln = (uint32_t)(S.nchars - r.st);
    else if (S.len) r.ln = S.len[i];
    else r.ln = (uint32_t)(S.off[i + 1] - r.st);
    return r;
}

// The 8 characters of a string from depth h, first character in the most
// significant byte, zero past the end of the string (the zero terminator is
// outside the alphabet, so the padding orders a proper prefix first).  Reads
// only the aligned 8-byte words that hold at least one byte of the string.
__device__ __forceinline__ uint64_t key_at(const uint8_t *chars, uint64_t nchars, uint64_t st, uint32_t ln,
                                           uint32_t h) {
    if (h >= ln) return 0;
    const uint64_t p = st + h;
    if (p >= nchars) return 0;   // never read outside the buffer (valid inputs never get here)
    const uint32_t rem = (uint32_t)min((uint64_t)(ln - h), nchars - p);
    // the aligned words by pointer arithmetic from `chars` (not through an
    // integer), so that the loads stay global-memory loads: a generic (flat)
    // load would also count against the LDS wait counter and every later LDS
    // wait would wait for it
    const uint32_t sh = (uint32_t)((uintptr_t)(chars + p) & 7);
    const uint64_t *a0 = reinterpret_cast<const uint64_t *>(chars + (p - sh));
    uint64_t w = a0[0] >> (8 * sh);
    if (sh != 0 && rem > 8 - sh) w |= a0[1] << (64 - 8 * sh);
    uint64_t k = __builtin_bswap64(w);
    if (rem < 8) k &= ~0ull << (8 * (8 - rem));
    return k;
}

// Keys of a classification step, base-case round or seam: the next q
// characters of a string from depth h in one uint64, first character in the
// most significant bits, zero past the end, so that one unsigned compare
// orders q characters and a zero last character means the string ends inside
// the key.  ByteKey: q = 8 characters of 8 bits (the word of Algorithm 1).
struct ByteKey {
    __device__ __forceinline__ uint32_t q() const { return 8u; }
    __device__ __forceinline__ uint64_t key(const Strs &S, uint64_t st, uint32_t ln, uint32_t h) const {
        return key_at(S.chars, S.nchars, st, ln, h);
    }
    __device__ __forceinline__ bool ends(uint64_t k) const { return (k & 0xFF) == 0; }
    // equal leading characters of two different keys (z = their xor != 0)
    __device__ __forceinline__ uint32_t eqc(uint64_t z) const { return (uint32_t)(__clzll(z) >> 3); }
};

// Alphabet compression (the alphabet-compression idea of the paper's
// outlook): when only sigma' < 256 byte values occur, character c gets the
// order-preserving code 1 + (number of occurring values below c), the end of
// the string code 0, so b = ceil(log2(sigma' + 1)) bits hold a character and
// one key holds q = min(64 / b, 32) characters (21 for DNA instead of 8).
// Keys compare exactly as the strings do; depths and LCPs stay in characters.
struct Alphabet {
    uint32_t b, q, sigma, pad;
    uint32_t present[8];      // bitmap of the byte values that occur
    uint8_t code[256];        // 0 for the value 0 and absent values, 1..sigma' in byte order
};

struct PackedKey {
    const uint8_t *code;      // Alphabet::code in device memory (256 bytes: L1 hits)
    uint32_t b, nq;
    __device__ __forceinline__ uint32_t q() const { return nq; }
    __device__ __forceinline__ uint64_t key(const Strs &S, uint64_t st, uint32_t ln, uint32_t h) const {
        if (h >= ln) return 0;
        const uint64_t p = st + h;
        if (p >= S.nchars) return 0;
        const uint32_t r = (uint32_t)min((uint64_t)min(ln - h, nq), S.nchars - p);
        const uint32_t sh = (uint32_t)((uintptr_t)(S.chars + p) & 7);
        const uint64_t *a0 = reinterpret_cast<const uint64_t *>(S.chars + (p - sh));
        const uint32_t nw = (sh + r + 7) >> 3;   // aligned words holding the r characters, 1..5
        uint64_t w[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) w[i] = (uint32_t)i < nw ? a0[i] : 0ull;
        // u0..u3: characters p + 8i .. p + 8i + 7 in little-endian byte order
        const uint64_t u0 = sh ? (w[0] >> (8 * sh)) | (w[1] << (64 - 8 * sh)) : w[0];
        const uint64_t u1 = sh ? (w[1] >> (8 * sh)) | (w[2] << (64 - 8 * sh)) : w[1];
        const uint64_t u2 = sh ? (w[2] >> (8 * sh)) | (w[3] << (64 - 8 * sh)) : w[2];
        const uint64_t u3 = sh ? (w[3] >> (8 * sh)) | (w[4] << (64 - 8 * sh)) : w[3];
        uint64_t k = 0;
        uint32_t at = 64;
        // eight independent code loads per word, so that their latencies overlap
#pragma unroll 1
        for (uint32_t i = 0; 8 * i < r; ++i) {
            const uint64_t x = i == 0 ? u0 : i == 1 ? u1 : i == 2 ? u2 : u3;
            const uint32_t m = min(r - 8 * i, 8u);
            uint32_t c8[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) c8[t] = (uint32_t)t < m ? code[(x >> (8 * t)) & 0xFF] : 0u;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                if ((uint32_t)t < m) {
                    at -= b;
                    k |= (uint64_t)c8[t] << at;
                }
            }
        }
        return k;
    }
    __device__ __forceinline__ bool ends(uint64_t k) const { return ((k >> (64 - nq * b)) & ((1ull << b) - 1)) == 0; }
    __device__ __forceinline__ uint32_t eqc(uint64_t z) const { return (uint32_t)__clzll(z) / b; }
};

// The 32 characters of a string from depth h as four keys (key_at at h,
// h + 8, h + 16, h + 24), from the at most five aligned words that hold them.
__device__ __forceinline__ void keys32_at(const uint8_t *chars, uint64_t nchars, uint64_t st, uint32_t ln, uint32_t h,
                                          uint64_t k[4]) {
#pragma unroll
    for (int j = 0; j < 4; ++j) k[j] = 0;
    if (h >= ln) return;
    const uint64_t p = st + h;
    if (p >= nchars) return;
    const uint32_t rem = (uint32_t)min((uint64_t)(ln - h), nchars - p);
    const uint32_t sh = (uint32_t)((uintptr_t)(chars + p) & 7);
    const uint64_t *a0 = reinterpret_cast<const uint64_t *>(chars + (p - sh));
    const uint32_t nw = (sh + min(rem, 32u) + 7) >> 3;   // words holding wanted bytes, 1..5
    uint64_t w[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) w[i] = (uint32_t)i < nw ? a0[i] : 0ull;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint64_t lo = sh ? (w[j] >> (8 * sh)) | (w[j + 1] << (64 - 8 * sh)) : w[j];
        uint64_t kj = __builtin_bswap64(lo);
        const int r = (int)rem - 8 * j;
        if (r <= 0) kj = 0;
        else if (r < 8) kj &= ~0ull << (8 * (8 - r));
        k[j] = kj;
    }
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// threadIdx.x behind an empty asm statement, so that the optimiser cannot
// hoist what is derived from it (per-thread LDS addresses) out of the phase
// that uses it: hoisted to the start of the persistent kernel, dozens of
// such addresses stay live across its whole loop and push other values into
// scratch.  Every phase of the worker takes its thread index from here.
#ifndef SSD_OPAQUE
#define SSD_OPAQUE(x) asm volatile("" : "+v"(x))
#endif
__device__ __forceinline__ int tid_here() {
    int t = (int)threadIdx.x;
    SSD_OPAQUE(t);
    return t;
}

// Broadcast a value that is equal in every thread (read from LDS after a
// barrier) so that the compiler treats it as uniform.  Every branch or loop
// that contains a barrier must be controlled by such values: with a
// condition the compiler cannot prove uniform it may lower the region as an
// exec-masked divergent loop, where the lanes of one wave no longer reach a
// barrier together.
__device__ __forceinline__ uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Lanes of the wave holding the same bucket number (wave64 has no match
// instruction: one ballot per bit of the bucket number).
__device__ __forceinline__ uint64_t match_any(uint32_t m, int nbits) {
    uint64_t mask = ~0ull;
#pragma unroll 1
    for (int b = 0; b < nbits; ++b) {
        const bool bit = (m >> b) & 1u;
        const uint64_t bal = __ballot(bit);
        mask &= bit ? bal : ~bal;
    }
    return mask;
}

// Inclusive scan within a wave.
template <typename T, typename Op>
__device__ __forceinline__ T wave_incl_scan(T x, Op op) {
    const uint32_t l = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(x, o, 64);
        if (l >= (uint32_t)o) x = op(x, y);
    }
    return x;
}

struct AddOp { __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a + b; } };
struct MaxOp { __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a > b ? a : b; } };

// Exclusive (or inclusive) scan of a[0..len) in LDS by the whole workgroup;
// each thread owns a run of consecutive entries.  tmp needs NW entries.
// Returns the total.  Must be called by all threads; includes barriers.
template <typename Op>
__device__ __forceinline__ uint32_t block_scan(uint32_t *a, int len, uint32_t *tmp, bool exclusive, Op op, uint32_t ident) {
    const int tid = tid_here();
    const int per = (len + NT - 1) / NT;
    const int lo = tid * per;
    const int hi = min(len, lo + per);
    uint32_t acc = ident;
    for (int i = lo; i < hi; ++i) acc = op(acc, a[i]);
    uint32_t inc = wave_incl_scan(acc, op);
    const int w = tid >> 6;
    if ((tid & 63) == 63) tmp[w] = inc;
    __syncthreads();
    uint32_t wpre = ident;
    for (int j = 0; j < w; ++j) wpre = op(wpre, tmp[j]);
    uint32_t total = ident;
    for (int j = 0; j < NW; ++j) total = op(total, tmp[j]);
    total = uni(total);
    uint32_t run = op(wpre, __shfl_up(inc, 1, 64));
    if ((tid & 63) == 0) run = wpre;
    for (int i = lo; i < hi; ++i) {
        const uint32_t x = a[i];
        const uint32_t nx = op(run, x);
        a[i] = exclusive ? run : nx;
        run = nx;
    }
    __syncthreads();
    return total;
}

// Splitter set of one classification step (LDS or global copy).
struct Split {
    uint64_t tree[VMAX + 1];   // level order, tree[1..v]
    uint8_t hl[VMAX + 1];      // hl[l] = lcp(x[l-1], x[l]) in characters, hl[0] = hl[v] = 0
    uint8_t zr[VMAX + 1];      // zr[l] = x[l] ends its string (last character zero)
    uint32_t v, d, nb, nbits, ndistinct;
    uint32_t ulast;            // ranks >= ulast repeat x[ulast] (tree padded with the largest key)
    uint32_t equal;            // classify with an equality test at every node (S5-Equal)
    uint32_t q;                // characters per key (8, or more with alphabet compression)
};

// Level-order node of the splitter with in-order rank r in a perfect tree of
// depth d: with r+1 = (2p+1)·2^k the node sits k levels above the leaves, at
// position p of its level (the rank-to-tree conversion of the second
// equality-check variant in the implementation details of S5).
__device__ __forceinline__ uint32_t node_of_rank(uint32_t r, uint32_t d) {
    const uint32_t k = __builtin_ctz(r + 1);
    return (1u << (d - 1 - k)) + ((r + 1) >> (k + 1));
}

template <typename SP>
__device__ __forceinline__ uint64_t splitter(const SP &sp, uint32_t r) { return sp.tree[node_of_rank(r, sp.d)]; }

// Bucket of key c: descend the level-order tree going right when c > t_i,
// then l = i - (v+1) counts the splitters below c; bucket 2l, plus one when
// the key equals x_l (the last bucket 2v has no equality test).
__device__ __forceinline__ uint32_t classify(uint64_t c, const Split &sp) {
    uint32_t i = 1;
#pragma unroll
    for (int l = 0; l < DMAX; ++l)
        if (l < (int)sp.d) i = 2 * i + (c > sp.tree[i] ? 1u : 0u);
    const uint32_t l = i - (sp.v + 1);
    return 2 * l + ((l < sp.v && splitter(sp, l) == c) ? 1u : 0u);
}

// S5-Equal (fourth variant of the implementation details): test equality at
// every node and stop at the first equal splitter; its in-order rank r gives
// the equality bucket 2r+1 (the first copy when the tree is padded, so the
// bucket is the same as above).  Without a match the descent ends at a leaf.
__device__ __forceinline__ uint32_t classify_equal(uint64_t c, const Split &sp) {
    uint32_t i = 1;
    for (uint32_t l = 0; l < sp.d; ++l) {
        const uint64_t t = sp.tree[i];
        if (c == t) {
            const uint32_t delta = 31 - __clz(i);
            const uint32_t p = i - (1u << delta);
            const uint32_t r = ((2 * p + 1) << (sp.d - 1 - delta)) - 1;
            return 2 * min(r, sp.ulast) + 1;
        }
        i = 2 * i + (c > t ? 1u : 0u);
    }
    return 2 * (i - (sp.v + 1));
}

__device__ __forceinline__ uint32_t classify_any(uint64_t c, const Split &sp) {
    return sp.equal ? classify_equal(c, sp) : classify(c, sp);
}

__device__ __forceinline__ uint32_t hash32(uint32_t x) {
    x ^= x >> 16; x *= 0x7feb352dU; x ^= x >> 15; x *= 0x846ca68bU; x ^= x >> 16;
    return x;
}

// Position of sample t of a (< size) in a segment of `size` strings: one
// pseudo-random pick in each of a strata of size / a strings (every string
// when the segment holds at most a; the last size mod a strings are never
// picked).  32-bit arithmetic only.
__device__ __forceinline__ uint32_t sample_pos(uint32_t t, uint32_t a, uint32_t size, uint32_t seed) {
    if (size <= a) return t;
    const uint32_t stride = size / a;
    return t * stride + hash32(seed ^ (t * 0x9E3779B9u)) % stride;
}

// Sample size for a segment of `size` strings: ovs (v + 1) - 1, at most size.
__device__ __forceinline__ uint32_t sample_count(uint32_t size, uint32_t vmax, uint32_t ovs) {
    const uint32_t amax = ovs * (vmax + 1) - 1;
    return size < amax ? size : amax;
}

// Sample keys and splitters for a segment of `size` strings at depth h, read
// through `load(e)` (0 <= e < size).  Sample of up to ovs(v+1)-1 keys
// (oversampling factor ovs; all strings when the segment is that small, else
// one pseudo-random pick per stratum), sorted in LDS; the distinct sample keys become
// the splitters when they fit into the tree (the smallest tree 2^d'-1 >= their
// number, padded by the largest), else v equidistant distinct keys, so that no
// splitter repeats (cf. the skip-duplicates selection).  Then the level-order
// tree, the splitter LCPs (xor + count leading zeros) and the end-of-string
// flags.  `samp`, `srt` need ovs(vmax+1) entries (a power of two: the sort
// pads to one), `fl` as many, tmp NW.  SP is Split, or the wide level's
// WSplit (same fields, larger arrays).  UNR: sample loads issued together per
// thread (the persistent worker keeps 1 for its code size).
template <int UNR = 1, typename SP, typename Load, typename KC>
__device__ __forceinline__ void select_splitters(SP &sp, uint32_t size, uint32_t h, uint32_t seed, uint32_t vmax,
                                                 uint32_t equal, uint64_t *samp, uint64_t *srt, uint32_t *fl,
                                                 uint32_t *tmp, Load load, const KC &kc, uint32_t ovs = 2) {
    const int tid = tid_here();
    const uint32_t a = sample_count(size, vmax, ovs);
#pragma unroll UNR
    for (uint32_t t = tid; t < a; t += NT) samp[t] = load(sample_pos(t, a, size, seed), h);
    // sort the sample: bitonic network over the next power of two, padded
    // with the largest key (padding sorts last, so srt[0..a) holds the sample)
    uint32_t a2 = 1;
    while (a2 < a) a2 <<= 1;
    a2 = uni(a2);
    for (uint32_t t = tid; t < a2; t += NT) srt[t] = t < a ? samp[t] : ~0ull;
    __syncthreads();
    for (uint32_t kk = 2; kk <= a2; kk <<= 1) {
        for (uint32_t jj = kk >> 1; jj > 0; jj >>= 1) {
            for (uint32_t t = tid; t < a2 / 2; t += NT) {
                const uint32_t i = 2 * t - (t & (jj - 1));   // lower element of the pair
                const uint32_t k2 = i + jj;
                const uint64_t x = srt[i], y = srt[k2];
                const bool up = (i & kk) == 0;
                if ((x > y) == up) {
                    srt[i] = y;
                    srt[k2] = x;
                }
            }
            __syncthreads();
        }
    }
    for (uint32_t t = tid; t < a; t += NT) fl[t] = (t == 0 || srt[t] != srt[t - 1]) ? 1u : 0u;
    __syncthreads();
    const uint32_t U = uni(block_scan(fl, (int)a, tmp, true, AddOp(), 0u));
    // compact the distinct keys into samp[0..U)
    for (uint32_t t = tid; t < a; t += NT)
        if (t == 0 || srt[t] != srt[t - 1]) samp[fl[t]] = srt[t];
    __syncthreads();
    uint32_t d, v;
    if (U <= vmax) {
        d = 1;
        while ((1u << d) - 1 < U) ++d;
        v = (1u << d) - 1;
    } else {
        v = vmax;
        d = 31 - __clz(vmax + 1);
    }
    // splitter of in-order rank j: samp[xsrc(j)]
    auto xsrc = [&](uint32_t j) -> uint32_t {
        if (U <= vmax) return j < U ? j : U - 1;
        return (uint32_t)(((uint64_t)(j + 1) * U) / (v + 1));
    };
    if (tid == 0) {
        sp.v = v;
        sp.d = d;
        sp.nb = 2 * v + 1;
        uint32_t nbits = 1;
        while ((1u << nbits) < 2 * v + 2) ++nbits;
        sp.nbits = nbits;
        sp.ndistinct = U;
        sp.ulast = U <= vmax ? U - 1 : v;
        sp.equal = equal;
        sp.q = kc.q();
    }
    __syncthreads();
    for (uint32_t j = 1 + tid; j <= v; j += NT) {
        const uint32_t delta = 31 - __clz(j);
        const uint32_t p = j - (1u << delta);
        const uint32_t r = ((2 * p + 1) << (d - 1 - delta)) - 1;
        sp.tree[j] = samp[xsrc(r)];
    }
    for (uint32_t l = tid; l <= v; l += NT) {
        uint32_t hl = 0;
        if (l > 0 && l < v) {
            const uint64_t z = samp[xsrc(l - 1)] ^ samp[xsrc(l)];
            hl = z ? kc.eqc(z) : kc.q();
        }
        sp.hl[l] = (uint8_t)hl;
        sp.zr[l] = (l < v && kc.ends(samp[xsrc(l)])) ? 1 : 0;
    }
    __syncthreads();
}

}  // namespace ssd
