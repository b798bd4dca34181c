// Wide whole-GPU level for gfx950: level 0 classified against up to 4095
// splitters (8191 buckets) instead of 255.
//
// The paper sizes the classification tree for the cache that holds it
// (v = 8191 for a 256 KiB L2, in the implementation details of S5) and, in
// its refinements, proposes two ways to afford large trees: distributing the
// strings in several passes, as an LSD radix sort whose keys are the bucket
// numbers ("oracles") computed once, and a jump table indexed by a key's most
// significant bits that replaces the top of the descent.  Here the tree and
// its jump table live in LDS (up to 40 KB per workgroup), and the
// distribution takes two stable passes: by the low WLO bits of the bucket
// number, then by the rest, so that each pass scatters into at most 128
// destinations per tile (whole cache lines) instead of up to 8191.
//
// Launch sequence for level 0 when the tuning asks for v > 255 (all grids
// sized for the level's capacity, as for the narrow levels):
//   k_wsample       one workgroup per segment: sample, sort, splitters,
//                   level-order tree, splitter LCPs, end flags, jump table;
//                   clears the segment's bucket bounds
//   k_wclassify     tiles: key gather, jump-table lookup, rest of the descent,
//                   bucket number per string, histogram of its low digit
//   k_lvl_colscan   offsets of every (tile, low digit)
//   k_wscatter<1>   tiles: stable redistribution by the low digit (records
//                   and bucket numbers into the other buffers)
//   k_whist2        tiles: histogram of the high digit, in pass-1 order
//   k_lvl_colscan   offsets of every (tile, high digit)
//   k_wscatter<2>   tiles: stable redistribution by the high digit: records
//                   now in bucket order, stable within each bucket
//   k_wbounds       tiles: first and one-past-last position of each bucket
//   k_wschedule     one workgroup per segment: children, as for a narrow level
#include "ssort_kernels.h"

namespace ssd {

// Jump table: for every value p of a key's top JA bits, descend from the root
// while p alone decides each comparison (p above or below the top JA bits of
// the node's splitter) and keep the node where that stops: a tree node whose
// comparison needs the whole key, or a leaf (> v) when p decides the whole
// path.  Keys with top bits p continue their descent from jump[p].
template <typename SP>
__device__ void build_jump(SP &sp) {
    const uint32_t v = sp.v;
    for (uint32_t p = tid_here(); p < (1u << JA); p += NT) {
        uint32_t i = 1;
        while (i <= v) {
            const uint32_t tp = (uint32_t)(sp.tree[i] >> (64 - JA));
            if (p == tp) break;
            i = 2 * i + (p > tp ? 1u : 0u);
        }
        sp.jump[p] = (uint16_t)i;
    }
    __syncthreads();
}

struct WSampleLDS {
    WSplit sp;
    uint64_t samp[WVMAX + 1];
    uint64_t srt[WVMAX + 1];
    uint32_t fl[WVMAX + 1];
    uint32_t tmp[NW];
};

// Splitters of a wide segment: a sample of v keys (oversampling 1: the sample
// arrays are the LDS budget here), the same selection as the narrow steps.
template <bool Z>
__global__ __launch_bounds__(NT) void k_wsample(Params P) {
    __shared__ WSampleLDS L;
    if (P.ctl->error || blockIdx.x >= lvl_count(P, 0, 0)) return;
    const LvlSeg g = P.lseg[0][blockIdx.x];
    uint32_t *ws = P.wst + (size_t)blockIdx.x * WNBPAD, *we = P.wen + (size_t)blockIdx.x * WNBPAD;
    for (uint32_t b = threadIdx.x; b < (uint32_t)WNBPAD; b += NT) {
        ws[b] = 0;
        we[b] = 0;
    }
    const auto kc = KeyOf<Z>::make(P);
    auto kload = [&](uint32_t e, uint32_t hh) -> uint64_t {
        const Rec r = seg_rec(P, g.meta, g.begin + e);
        return kc.key(P.S, r.st, r.ln, hh);
    };
    select_splitters<8>(L.sp, g.size, g.depth, hash32(g.begin * 0x85EBCA6Bu ^ g.depth * 0xC2B2AE35u ^ g.size), P.wv,
                        0u, L.samp, L.srt, L.fl, L.tmp, kload, kc, 1u);
    build_jump(L.sp);
    const uint32_t *src = (const uint32_t *)&L.sp;
    uint32_t *dst = (uint32_t *)&P.wsplit[blockIdx.x];
    for (uint32_t i = threadIdx.x; i < sizeof(WSplit) / 4; i += NT) dst[i] = src[i];
}

// The segment and tile of a wide-level tile workgroup (false: nothing to do,
// or an inconsistent table, reported).
__device__ __forceinline__ bool wide_tile(const Params &P, uint32_t &seg, LvlSeg &g) {
    if (P.ctl->error || blockIdx.x >= lvl_count(P, 0, 1)) return false;
    seg = P.tile2seg[0][blockIdx.x];
    if (seg >= lvl_count(P, 0, 0)) {
        if (threadIdx.x == 0) atomicOr(&P.ctl->error, ERR_LEVEL);
        return false;
    }
    g = P.lseg[0][seg];
    // level 0 reads its records from the input (the first pass writes R0)
    if (g.begin > P.S.n || g.size > P.S.n - g.begin || blockIdx.x < g.tile0 || blockIdx.x - g.tile0 >= g.ntile ||
        !(g.meta & M_IDENT_SRC)) {
        if (threadIdx.x == 0) atomicOr(&P.ctl->error, ERR_LEVEL);
        return false;
    }
    return true;
}

// Classification against the wide tree.  LDS (dynamic): tree[0..wv], the
// jump table, the low-digit histogram.  Each key starts at jump[top bits] and
// finishes the descent (i <- 2i + [c > t_i]) from there; K keys per thread
// descend together, the loop ending once every lane's keys reached a leaf.
template <int K, bool Z>
__global__ __launch_bounds__(NT) void k_wclassify(Params P) {
    extern __shared__ uint64_t wlds[];
    uint32_t seg;
    LvlSeg g;
    if (!wide_tile(P, seg, g)) return;
    const WSplit *gs = &P.wsplit[seg];
    uint64_t *tree = wlds;
    uint16_t *jump = reinterpret_cast<uint16_t *>(wlds + (P.wv + 1));
    uint32_t *hist = reinterpret_cast<uint32_t *>(jump + (1u << JA));
    const uint32_t v = uni(gs->v), d = uni(gs->d);
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    for (uint32_t i = tid; i <= v; i += NT) tree[i] = gs->tree[i];
    {
        const uint32_t *js = reinterpret_cast<const uint32_t *>(gs->jump);
        uint32_t *jd = reinterpret_cast<uint32_t *>(jump);
        for (uint32_t i = tid; i < (1u << JA) / 2; i += NT) jd[i] = js[i];
    }
    for (uint32_t b = tid; b < (1u << WLO); b += NT) hist[b] = 0;
    __syncthreads();
    const auto kc = KeyOf<Z>::make(P);
    const uint32_t nd = 1u << WLO;
    const uint32_t lt = blockIdx.x - g.tile0;
    for (uint32_t ch = 0; ch < ROOT_CHUNKS; ++ch) {
        const uint32_t c0 = (lt * ROOT_CHUNKS + ch) * (uint32_t)(NT * K);
        if (c0 >= g.size) break;
        Rec r[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const uint32_t e = c0 + (uint32_t)(w * 64 * K + j * 64 + lane);
            if (e < g.size) r[j] = seg_rec(P, g.meta, g.begin + e);
        }
        uint64_t k[K];
        uint32_t node[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const uint32_t e = c0 + (uint32_t)(w * 64 * K + j * 64 + lane);
            k[j] = e < g.size ? kc.key(P.S, r[j].st, r[j].ln, g.depth) : 0;
            node[j] = e < g.size ? (uint32_t)jump[k[j] >> (64 - JA)] : v + 1;
        }
        for (int lv = 0; lv < WDMAX; ++lv) {
            bool live = false;
#pragma unroll
            for (int j = 0; j < K; ++j) {
                if (node[j] <= v) node[j] = 2 * node[j] + (k[j] > tree[node[j]] ? 1u : 0u);
                live |= node[j] <= v;
            }
            if (__ballot(live) == 0) break;
        }
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const uint32_t e = c0 + (uint32_t)(w * 64 * K + j * 64 + lane);
            const bool valid = e < g.size;
            const uint32_t l = node[j] - (v + 1);
            const uint32_t m = 2 * l + ((l < v && tree[node_of_rank(l, d)] == k[j]) ? 1u : 0u);
            const uint32_t dg = valid ? (m & (nd - 1)) : nd;
            const uint64_t mask = match_any(dg, WLO + 1);
            if (valid && lane == 63 - (int)__clzll(mask)) atomicAdd(&hist[dg], (uint32_t)__popcll(mask));
            if (valid) P.bkt[g.begin + e] = (uint16_t)m;
        }
    }
    __syncthreads();
    for (uint32_t b = tid; b < nd; b += NT) P.hist[(size_t)blockIdx.x * NBPAD + b] = hist[b];
}

// Histogram of the high digit (bucket number >> WLO) per tile of the pass-1
// order.
__global__ __launch_bounds__(NT) void k_whist2(Params P, uint32_t hbits) {
    __shared__ uint32_t hist[NBPAD];
    uint32_t seg;
    LvlSeg g;
    if (!wide_tile(P, seg, g)) return;
    const int tid = threadIdx.x, lane = tid & 63;
    const uint32_t nd = 1u << hbits;
    for (uint32_t b = tid; b < nd; b += NT) hist[b] = 0;
    __syncthreads();
    const uint32_t lt = blockIdx.x - g.tile0;
    const uint32_t e0 = lt * P.tile, e1 = min(g.size, e0 + P.tile);
    for (uint32_t b0 = e0; b0 < e1; b0 += NT) {
        const uint32_t e = b0 + tid;
        const bool valid = e < e1;
        const uint32_t dg = valid ? (uint32_t)(P.btmp[g.begin + e] >> WLO) : nd;
        const uint64_t mask = match_any(dg, (int)hbits + 1);
        if (valid && dg < nd && lane == 63 - (int)__clzll(mask)) atomicAdd(&hist[dg], (uint32_t)__popcll(mask));
        if (valid && dg >= nd) atomicOr(&P.ctl->error, ERR_LEVEL);
    }
    __syncthreads();
    for (uint32_t b = tid; b < nd; b += NT) P.hist[(size_t)blockIdx.x * NBPAD + b] = hist[b];
}

template <int K>
struct WScatterLDS {
    uint32_t run[NBPAD];
    uint32_t tmp[NW];
    ScatterLDS<K, true> sc;
};

// One stable distribution pass of a wide level: PASS 1 by the low digit, from
// the input records (and bkt) into R0 (and btmp); PASS 2 by the high digit,
// from R0 (and btmp) into R1 (and bkt).  Offsets: the segment start, the
// exclusive sum over the digit totals, the tile's column-scan offset.
template <int K, int PASS>
__global__ __launch_bounds__(NT) void k_wscatter(Params P, uint32_t hbits) {
    __shared__ WScatterLDS<K> L;
    uint32_t seg;
    LvlSeg g;
    if (!wide_tile(P, seg, g)) return;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const uint32_t dbits = PASS == 1 ? (uint32_t)WLO : hbits;
    const uint32_t nd = 1u << dbits;
    const uint32_t *tot = &P.ltot[0][(size_t)seg * NBPAD];
    for (uint32_t b = tid; b < NBPAD; b += NT) L.run[b] = b < nd ? tot[b] : 0u;
    __syncthreads();
    block_scan(L.run, (int)nd, L.tmp, true, AddOp(), 0u);
    for (uint32_t b = tid; b < nd; b += NT) L.run[b] += g.begin + P.hist[(size_t)blockIdx.x * NBPAD + b];
    __syncthreads();
    Rec *out = PASS == 1 ? P.R0 : P.R1;
    const uint16_t *bin = PASS == 1 ? P.bkt : P.btmp;
    uint16_t *bout = PASS == 1 ? P.btmp : P.bkt;
    const uint32_t lt = blockIdx.x - g.tile0;
    for (uint32_t ch = 0; ch < ROOT_CHUNKS; ++ch) {
        const uint32_t c0 = (lt * ROOT_CHUNKS + ch) * (uint32_t)(NT * K);
        if (c0 >= g.size) break;
        Rec r[K];
        uint32_t m[K];
        uint16_t pb[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const uint32_t e = c0 + (uint32_t)(w * 64 * K + j * 64 + lane);
            pb[j] = 0;
            m[j] = nd;
            if (e < g.size) {
                r[j] = PASS == 1 ? seg_rec(P, g.meta, g.begin + e) : P.R0[g.begin + e];
                pb[j] = bin[g.begin + e];
                // a bucket number is below 2^(WLO + hbits), so the digit is in
                // range; the mask keeps every LDS slot inside its array anyway
                m[j] = (PASS == 1 ? (uint32_t)pb[j] : (uint32_t)(pb[j] >> WLO)) & (nd - 1);
            }
        }
        scatter_chunk<K, true>(L.sc, L.tmp, nd, (int)dbits + 1, m, r, pb, min((uint32_t)(NT * K), g.size - c0), L.run,
                               out, bout, P.S.n, &P.ctl->error);
    }
}

// Bucket bounds from the bucket numbers in their final (bucket) order.
__global__ __launch_bounds__(NT) void k_wbounds(Params P) {
    uint32_t seg;
    LvlSeg g;
    if (!wide_tile(P, seg, g)) return;
    const uint32_t nb = P.wsplit[seg].nb;
    uint32_t *ws = P.wst + (size_t)seg * WNBPAD, *we = P.wen + (size_t)seg * WNBPAD;
    const uint32_t lt = blockIdx.x - g.tile0;
    const uint32_t e0 = lt * P.tile, e1 = min(g.size, e0 + P.tile);
    const uint16_t *bk = P.bkt + g.begin;
    for (uint32_t e = e0 + threadIdx.x; e < e1; e += NT) {
        const uint32_t b = bk[e];
        if (b >= nb) {
            atomicOr(&P.ctl->error, ERR_LEVEL);
            continue;
        }
        if (e == 0 || bk[e - 1] != b) ws[b] = e;
        if (e + 1 == g.size || bk[e + 1] != b) we[b] = e + 1;
    }
}

// Children of a wide segment: bucket sizes and starts from the bounds, one
// workgroup per NBPAD buckets (their chunks of small buckets stay inside the
// workgroup's buckets; queue slots and descriptors are reserved per
// workgroup).
constexpr uint32_t WSCHED_G = WNBPAD / NBPAD;
__global__ __launch_bounds__(NT) void k_wschedule(Params P) {
    __shared__ SchedLDS<NBPAD> L;
    const uint32_t seg = blockIdx.x / WSCHED_G, grp = blockIdx.x % WSCHED_G;
    if (P.ctl->error || seg >= lvl_count(P, 0, 0)) return;
    const LvlSeg g = P.lseg[0][seg];
    const WSplit &sp = P.wsplit[seg];
    const uint32_t nbs = uni(sp.nb);
    const uint32_t b0 = grp * NBPAD;
    if (b0 >= nbs) return;
    const uint32_t nb = min((uint32_t)NBPAD, nbs - b0);
    const uint32_t *ws = P.wst + (size_t)seg * WNBPAD + b0, *we = P.wen + (size_t)seg * WNBPAD + b0;
    for (uint32_t b = threadIdx.x; b < (uint32_t)NBPAD; b += NT) {
        const uint32_t a = b < nb ? ws[b] : 0u, e = b < nb ? we[b] : 0u;
        L.cnt[b] = e > a ? e - a : 0u;
        L.bst[b] = a;
    }
    __syncthreads();
    schedule_buckets<NBPAD>(P, 0, g, b0, nb, sp, L);
}

// Debug dump of one wide step (the whole input as one segment): keys, the
// splitters in order, the tree, the jump table, bucket numbers in input order,
// bucket sizes, the redistributed permutation.
__global__ void k_wdebug_dump(Params P, uint32_t depth, uint64_t *keys, uint64_t *split, uint64_t *tree,
                              uint16_t *jump, uint32_t *info, uint16_t *bucket, uint32_t *hist, uint32_t *perm) {
    const WSplit *sp = &P.wsplit[0];
    const uint32_t n = P.S.n;
    for (uint32_t i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT) {
        const Rec r = make_rec(P.S, i);
        keys[i] = key_at(P.S.chars, P.S.nchars, r.st, r.ln, depth);
        const uint32_t id = P.R1[i].id;
        perm[i] = id;
        if (id < n) bucket[id] = P.bkt[i];
    }
    if (blockIdx.x == 0) {
        for (uint32_t j = threadIdx.x; j < (uint32_t)(WVMAX + 1); j += NT) {
            split[j] = j < sp->v ? splitter(*sp, j) : 0;
            tree[j] = (j < sp->v) ? sp->tree[j + 1] : 0;
        }
        if (jump)
            for (uint32_t j = threadIdx.x; j < (1u << JA); j += NT) jump[j] = sp->jump[j];
        for (uint32_t b = threadIdx.x; b < (uint32_t)WNBPAD; b += NT)
            hist[b] = b < sp->nb ? P.wen[b] - P.wst[b] : 0;
        if (threadIdx.x == 0) {
            info[0] = sp->v;
            info[1] = sp->d;
            info[2] = sp->ndistinct;
            info[3] = JA;
        }
    }
}

template __global__ void k_wsample<false>(Params);
template __global__ void k_wsample<true>(Params);
template __global__ void k_wclassify<4, false>(Params);
template __global__ void k_wclassify<8, false>(Params);
template __global__ void k_wclassify<4, true>(Params);
template __global__ void k_wclassify<8, true>(Params);
template __global__ void k_wscatter<4, 1>(Params, uint32_t);
template __global__ void k_wscatter<4, 2>(Params, uint32_t);
template __global__ void k_wscatter<8, 1>(Params, uint32_t);
template __global__ void k_wscatter<8, 2>(Params, uint32_t);

}  // namespace ssd
