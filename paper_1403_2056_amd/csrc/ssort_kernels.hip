// HIP kernels of the string sample sorter for gfx950.
//
// Control flow of one sort (all enqueued on one stream, no host round trip):
//   k_init            queue ring, control block
//   k_seed            the input (or each batched set): a segment of the first
//                     whole-GPU level when large, else a worker task
//   [levels 0, 1]     large segments are classified by the whole GPU:
//                     k_lvl_sample (a workgroup per segment), k_lvl_classify
//                     (tiles), k_lvl_colscan (per segment and bucket),
//                     k_lvl_scatter (tiles), k_lvl_schedule (a workgroup per
//                     segment: next-level segments, worker tasks, base-case
//                     chunk tasks)
//   k_worker          persistent workgroups drain a device-side work queue of
//                     segments and base-case chunks; each segment step
//                     (sample, tree, classify, count, prefix sum, stable
//                     redistribution) is done by one workgroup, its large
//                     children are queued (one is kept), its small buckets go
//                     to the LCP-aware base case in chunks, queued as well
//   k_seam            LCPs at bucket boundaries from the separation depth
//                     recorded when the boundary was created
#include "ssort_kernels.h"

namespace ssd {

struct Task {
    uint32_t begin, size, depth, meta, setbase;
};

// Data another workgroup wrote during this launch (a task's records, a
// group descriptor, a queue slot) is read with device-coherent loads: on this
// chip a die's L2 can still hold a line of it from before the writer's
// release (a neighbouring range read earlier, or the previous sort in the same
// memory), and the acquire does not drop such lines.  A workgroup's own
// writes (the child it goes on with, its own chunks) use ordinary loads.
__device__ __forceinline__ uint32_t ld_coh32(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_coh64(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coh32(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coh64(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// A group descriptor handed to other workgroups: device-coherent stores.
__device__ __forceinline__ void st_desc(GroupDesc *d, uint32_t start, uint32_t size, uint32_t depth) {
    uint64_t *q = reinterpret_cast<uint64_t *>(d);
    st_coh64(q, (uint64_t)start | ((uint64_t)size << 32));
    st_coh64(q + 1, (uint64_t)depth);
}
__device__ __forceinline__ Rec ld_rec(const Rec *p, bool coh) {
    if (!coh) return *p;
    const uint64_t *q = reinterpret_cast<const uint64_t *>(p);
    const uint64_t a = ld_coh64(q), b = ld_coh64(q + 1);
    Rec r;
    r.st = a;
    r.ln = (uint32_t)b;
    r.id = (uint32_t)(b >> 32);
    return r;
}

__device__ __forceinline__ Rec load_rec(const Params &P, uint32_t meta, uint32_t pos, bool coh) {
    if (meta & M_IDENT_SRC) return make_rec(P.S, pos);
    return ld_rec(((meta & M_PARITY) ? P.R1 : P.R0) + pos, coh);
}

// A step writes its redistribution into the other record buffer.
__device__ __forceinline__ bool out_is_r1(uint32_t meta) {
    return (meta & M_IDENT_SRC) ? true : !(meta & M_PARITY);
}

__device__ __forceinline__ unsigned long long ld_rlx(unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rlx(unsigned long long *p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// queue counters carry no data: relaxed
__device__ __forceinline__ unsigned long long add_agent(unsigned long long *p, unsigned long long v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Make the workgroup's global writes visible to every workgroup of the
// device.  The L2 caches of the chip's dies are not coherent with each other
// for this memory, so an agent-scope release writes the die's L2 back; that
// is costly, so each wave first waits until its own stores have reached the
// L2 and then a single wave releases (instead of every wave).  Whatever is
// stored after this (queue slot sequence numbers) can be relaxed: a reader
// that sees it and then acquires sees the data.
//
// The fence alone compiles to the L2 write-back without a wait for it: the
// compiler leaves that wait to this wave's next store, but the publishing
// stores that follow the barrier come from every wave.  So the releasing wave
// waits for the write-back itself before the barrier; without that wait a
// sequence number could become visible before the data it publishes.
__device__ __forceinline__ void release_wg() {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __builtin_amdgcn_s_waitcnt(0);
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Stable redistribution of one chunk (Algorithm 1, redistribution; parallel
// form of the theorem's proof: per-workgroup counters and an interleaved
// prefix sum).  The chunk holds up to NT*K elements laid out wave-contiguous:
// element e = w*64*K + j*64 + lane.  Ranks inside a wave come from bucket
// matching by ballots, waves are ordered through per-wave counters, and the
// records are regrouped by bucket in LDS so that each bucket's run is written
// contiguously.  run[b] is the output position of the chunk's first element
// of bucket b and is advanced past the chunk.  With PAY, a 16-bit payload per
// element (the full bucket number, when the buckets here are digits of it)
// moves with its record into pout.
template <int K, bool PAY = false>
struct ScatterLDS {
    uint16_t wcnt[NW][NBPAD];   // per wave and bucket, at most 64*K per chunk
    uint16_t tot[NBPAD];        // per bucket in the chunk, at most NT*K
    uint32_t cs[NBPAD];
    Rec rec[NT * K];
    uint16_t b[NT * K];
    uint16_t pay[PAY ? NT * K : 1];
    uint32_t run[NBPAD];        // next output position per bucket (a step's own)
};

template <int K, bool PAY = false>
__device__ __forceinline__ void scatter_chunk(ScatterLDS<K, PAY> &L, uint32_t *tmp, uint32_t nb, int nbits,
                              const uint32_t (&m)[K], const Rec (&r)[K], const uint16_t *pay, uint32_t cnt,
                              uint32_t *run, Rec *out, uint16_t *pout, uint32_t nlim, unsigned long long *err) {
    const int tid = tid_here(), w = tid >> 6, lane = tid & 63;
    uint32_t *wc = (uint32_t *)&L.wcnt[0][0];
    for (int i = tid; i < NW * NBPAD / 2; i += NT) wc[i] = 0;
    __syncthreads();
    uint32_t rk[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const uint32_t mj = m[j];
        const uint64_t mask = match_any(mj, nbits);
        // wave-synchronous: every lane reads the wave's count before the
        // bucket's last lane advances it
        const uint32_t base = L.wcnt[w][mj];
        rk[j] = base + mbcnt(mask);
        __builtin_amdgcn_wave_barrier();
        if (lane == 63 - (int)__clzll(mask)) L.wcnt[w][mj] = (uint16_t)(base + (uint32_t)__popcll(mask));
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    for (uint32_t b = tid; b < nb; b += NT) {
        uint32_t c = 0;
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) {
            const uint32_t t = L.wcnt[ww][b];
            L.wcnt[ww][b] = (uint16_t)c;
            c += t;
        }
        L.tot[b] = (uint16_t)c;
        L.cs[b] = c;
    }
    __syncthreads();
    block_scan(L.cs, (int)nb, tmp, true, AddOp(), 0u);
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const uint32_t e = (uint32_t)(w * 64 * K + j * 64 + lane);
        if (e < cnt) {
            const uint32_t mj = m[j];
            const uint32_t slot = L.cs[mj] + L.wcnt[w][mj] + rk[j];
            L.rec[slot] = r[j];
            L.b[slot] = (uint16_t)mj;
            if constexpr (PAY) L.pay[slot] = pay[j];
        }
    }
    __syncthreads();
    for (uint32_t s = tid; s < cnt; s += NT) {
        const uint32_t mb = L.b[s];
        const uint32_t gp = run[mb] + (s - L.cs[mb]);
        if (gp < nlim) {
            out[gp] = L.rec[s];
            if constexpr (PAY) pout[gp] = L.pay[s];
        } else {
            atomicOr(err, ERR_SCATTER);
        }
    }
    __syncthreads();
    for (uint32_t b = tid; b < nb; b += NT) run[b] += L.tot[b];
    __syncthreads();
}

// A running minimum kept in LDS and lowered by other lanes, read afresh: an
// LDS load (through a generic pointer it would be a flat load, which also
// waits behind every global load in flight).
typedef uint32_t __attribute__((address_space(3))) lds_u32;
__device__ __forceinline__ uint32_t ld_stop(const uint32_t *p) { return *(volatile const lds_u32 *)p; }

// Length of the common prefix of strings a and b, known to agree on [0, from),
// compared 32 bytes (four independent 8-byte loads per string) at a time and
// given up once it reaches `stop` (the caller only needs values below it).
// Equal words that end both strings mean the strings are identical.
__device__ __forceinline__ uint32_t lcp_from(const Params &P, uint64_t sta, uint32_t lna, uint64_t stb, uint32_t lnb,
                                             uint32_t from, const uint32_t *stop) {
    uint32_t l = from;
    for (;;) {
        if (l >= ld_stop(stop)) return l;
        uint64_t ka[4], kb[4];
        keys32_at(P.S.chars, P.S.nchars, sta, lna, l, ka);
        keys32_at(P.S.chars, P.S.nchars, stb, lnb, l, kb);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (ka[i] != kb[i]) return l + 8 * i + (uint32_t)(__clzll(ka[i] ^ kb[i]) >> 3);
            if ((ka[i] & 0xFF) == 0) return min(lna, lnb);
        }
        l += 32;
    }
}

// Lanes per comparison for n pending long comparisons: the whole wave (512
// bytes a trip) for a few, halving down to 8 lanes (64 bytes a trip); 0 when
// there are more than a workgroup's lanes can cover 8 at a time (then every
// thread compares its own pairs).
__device__ __forceinline__ uint32_t group_width(uint32_t n) {
    if (n > (uint32_t)NT / 8) return 0;
    uint32_t g = 64;
    while (g > 8 && n * g > (uint32_t)NT) g >>= 1;
    return g;
}

// Length of the common prefix of strings a and b, known to agree on [0, from),
// computed by a group of G consecutive lanes (G a power of two, 8..64; the
// group's lanes pass the same arguments): lane j compares the 8 bytes at
// l + 8j, one ballot finds the first lane that sees a difference or the end,
// so one trip covers 8G bytes.  A lane whose position is at or beyond *stop
// (read by each lane; the caller only needs values below it, and *stop only
// decreases) ends the comparison there and the result is that position,
// which every earlier lane has verified to be a common prefix.  Called by all
// 64 lanes of the wave together (groups with on == false take part without a
// pair); the wave loops until its last group is done.
__device__ __forceinline__ uint32_t group_lcp(const Params &P, uint32_t G, bool on, uint64_t sta, uint32_t lna,
                                              uint64_t stb, uint32_t lnb, uint32_t from, const uint32_t *stop) {
    const uint32_t lane = lane_id();
    const uint32_t gl = lane & (G - 1), gb = lane & ~(G - 1);
    const uint64_t gmask = G >= 64 ? ~0ull : ((1ull << G) - 1) << gb;
    uint32_t res = 0;
    bool live = on;
    for (uint32_t l = from; __ballot(live) != 0; l += 8 * G) {
        bool f = false;
        uint32_t v = 0;
        if (live) {
            const uint32_t pos = l + 8 * gl;
            const bool cut = pos >= ld_stop(stop);
            uint64_t ka = 0, kb = 0;
            if (!cut) {
                ka = key_at(P.S.chars, P.S.nchars, sta, lna, pos);
                kb = key_at(P.S.chars, P.S.nchars, stb, lnb, pos);
            }
            f = cut || ka != kb || (ka & 0xFF) == 0;
            v = cut ? pos : (ka != kb ? pos + (uint32_t)(__clzll(ka ^ kb) >> 3) : min(lna, lnb));
        }
        const uint64_t m = __ballot(f) & gmask;
        const uint32_t got = __shfl(v, m ? (int)__builtin_ctzll(m) : (int)lane, 64);
        if (live && m) {
            res = got;
            live = false;
        }
    }
    return res;
}

// ---------------------------------------------------------------------------
// LCP-aware base case (semantics of LCP insertion sort, Algorithm 5: sorted
// order, stable by input index, and the adjacent LCPs).  A chunk of up to C
// strings from several groups; each group is sorted independently from its
// common depth.  Elements live at positions; a class is a run of positions
// [start, end) whose strings agree up to the class depth.  Rounds: gather the
// 8-byte key at the class depth, rank every element inside its class by
// (key, position) — positions inside a class follow input order, because
// every redistribution before the base case and every round is stable — and
// split classes at key changes: an element that starts a run of equal keys
// gets lcp = depth + equal leading bytes with the largest smaller key of its
// class, equal keys ending their strings are identical strings (lcp =
// length), runs of at least two equal keys without an end stay active at
// depth + 8.  An element whose depth is DONE needs no more rounds.
constexpr uint32_t DONE = 0xFFFFFFFFu;

template <int C>
struct BaseLDS {
    uint64_t st[C];
    uint64_t kq[C];          // keys by position (also the extension's pair list)
    uint32_t ln[C];
    uint32_t id[C];
    uint32_t d[C];           // per element: class depth, or DONE
    uint32_t scr[C];
    uint32_t cls[C];         // per position: class start | class end << 16
    uint32_t gp[C];          // per position: its place in the output arrays
    uint16_t ord[2][C];      // element at each position
    uint32_t any;
    uint32_t nlist;
};

// Adds to r, for the class keys a0 at position j + T and a1 at j + T + 1,
// whether each comes before key k at position q (qd = q - j): the borrow out
// of a - k - [j + T < q] is 1 exactly when a < k, or a = k at an earlier
// position.  One compare and a three-step carry chain per key (left to
// itself the compiler emits two 64-bit compares and mask logic per key).
template <int T>
__device__ __forceinline__ void rank_pair(uint32_t &r, uint64_t a0, uint64_t a1, uint64_t k, int qd) {
    uint32_t x;
    asm("v_cmp_lt_i32_e32 vcc, %[t0], %[qd]\n\t"
        "v_subb_co_u32_e32 %[x], vcc, %[a0l], %[kl], vcc\n\t"
        "v_subb_co_u32_e32 %[x], vcc, %[a0h], %[kh], vcc\n\t"
        "v_addc_co_u32_e32 %[r], vcc, 0, %[r], vcc\n\t"
        "v_cmp_lt_i32_e32 vcc, %[t1], %[qd]\n\t"
        "v_subb_co_u32_e32 %[x], vcc, %[a1l], %[kl], vcc\n\t"
        "v_subb_co_u32_e32 %[x], vcc, %[a1h], %[kh], vcc\n\t"
        "v_addc_co_u32_e32 %[r], vcc, 0, %[r], vcc"
        : [r] "+v"(r), [x] "=&v"(x)
        : [t0] "n"(T), [t1] "n"(T + 1), [qd] "v"(qd), [a0l] "v"((uint32_t)a0), [a0h] "v"((uint32_t)(a0 >> 32)),
          [a1l] "v"((uint32_t)a1), [a1h] "v"((uint32_t)(a1 >> 32)), [kl] "v"((uint32_t)k),
          [kh] "v"((uint32_t)(k >> 32))
        : "vcc");
}

// Group accessor: group g of the chunk has global start gstart(g), size
// gsize(g), common depth gdepth(g) and chunk-local exclusive prefix gpre(g).
template <int C, typename G, typename Mark, typename KC>
__device__ __forceinline__ void base_chunk(const Params &P, BaseLDS<C> &B, uint32_t *tmp, const Rec *src, uint32_t setbase,
                           uint32_t ng, uint32_t M, const G &grp, Mark mk, unsigned long long *st, const KC &kc,
                           bool coh) {
    const int tid = tid_here();
    auto find = [&](uint32_t q) -> uint32_t {
        uint32_t lo = 0, hi = ng;           // largest g with gpre(g) <= q
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (grp.gpre(mid) <= q) lo = mid; else hi = mid;
        }
        return lo;
    };
    constexpr int PER = (C + NT - 1) / NT;   // positions per thread
    const unsigned long long t_start = wall_clock64();
    {
        uint32_t gg[PER];
        Rec rr[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const uint32_t q = tid + u * NT;
            if (q < M) {
                gg[u] = find(q);
                rr[u] = ld_rec(&src[grp.gstart(gg[u]) + (q - grp.gpre(gg[u]))], coh);
            }
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const uint32_t q = tid + u * NT;
            if (q >= M) continue;
            const uint32_t g = gg[u];
            const uint32_t c0 = grp.gpre(g), sz = grp.gsize(g);
            B.st[q] = rr[u].st;
            B.ln[q] = rr[u].ln;
            B.id[q] = rr[u].id;
            B.d[q] = sz >= 2 ? grp.gdepth(g) : DONE;
            B.cls[q] = c0 | ((c0 + sz) << 16);
            B.gp[q] = grp.gstart(g) + (q - c0);
            B.ord[0][q] = (uint16_t)q;
        }
    }
    if (tid == 0) B.any = 0;
    __syncthreads();
    mk(PH_BASE);
    int cur = 0;
    uint32_t rounds = 0;
    bool more = true, first = true;
    while (more) {
        ++rounds;
        // after the first round every active class holds equal keys: it first
        // jumps to its exact common prefix, each member compared with the
        // class's first member from the class depth on (instead of one round
        // per 8 equal bytes)
        if (!first) {
        // (each active class's running minimum at its head and the list
        // count were reset when the classes were split)
        // first 32 bytes of every member against its class head; the pairs
        // still equal go to a list (kept where the keys go: they are gathered
        // again after the extension)
        uint32_t *list = reinterpret_cast<uint32_t *>(B.kq);
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const uint32_t q = tid + u * NT;
            if (q >= M) continue;
            const uint32_t c0 = B.cls[q] & 0xFFFF, e = B.ord[cur][q];
            if (q == c0 || B.d[e] == DONE) continue;
            const uint32_t f = B.ord[cur][c0], de = B.d[e];
            uint64_t ka[4], kb[4];
            keys32_at(P.S.chars, P.S.nchars, B.st[f], B.ln[f], de, ka);
            keys32_at(P.S.chars, P.S.nchars, B.st[e], B.ln[e], de, kb);
            uint32_t l = 0xFFFFFFFFu;
#pragma unroll
            for (int i = 3; i >= 0; --i) {
                if (ka[i] != kb[i]) l = de + 8 * i + (uint32_t)(__clzll(ka[i] ^ kb[i]) >> 3);
                else if ((ka[i] & 0xFF) == 0) l = min(B.ln[f], B.ln[e]);
            }
            if (l != 0xFFFFFFFFu) atomicMin(&B.scr[c0], l);
            else list[atomicAdd(&B.nlist, 1u)] = q;
        }
        __syncthreads();
        // the rest: by groups of lanes when few, by single threads when many
        {
            const uint32_t n = uni(B.nlist);
            const uint32_t gw = group_width(n);
            if (gw) {
                for (uint32_t i0 = 0; i0 < n; i0 += NT / gw) {
                    const uint32_t i = i0 + tid / gw;
                    const bool on = i < n;
                    const uint32_t q = on ? list[i] : 0u, c0 = B.cls[q] & 0xFFFF;
                    const uint32_t e = B.ord[cur][q], f = B.ord[cur][c0];
                    const uint32_t l = group_lcp(P, gw, on, B.st[f], B.ln[f], B.st[e], B.ln[e], B.d[e] + 32, &B.scr[c0]);
                    if (on && (tid & (gw - 1)) == 0) atomicMin(&B.scr[c0], l);
                }
            } else {
                for (uint32_t i = tid; i < n; i += NT) {
                    const uint32_t q = list[i], c0 = B.cls[q] & 0xFFFF;
                    const uint32_t e = B.ord[cur][q], f = B.ord[cur][c0];
                    const uint32_t l = lcp_from(P, B.st[f], B.ln[f], B.st[e], B.ln[e], B.d[e] + 32, &B.scr[c0]);
                    atomicMin(&B.scr[c0], l);
                }
            }
        }
        __syncthreads();
        mk(PH_BEXT);
        // the new depths: each thread writes those of the elements at its own
        // positions, which only it reads (for their keys, below)
        for (uint32_t q = tid; q < M; q += NT) {
            const uint32_t e = B.ord[cur][q];
            if (B.d[e] != DONE) B.d[e] = B.scr[B.cls[q] & 0xFFFF];
        }
        }
        first = false;
        {
            uint64_t kk[PER];
            bool on[PER];
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const uint32_t q = tid + u * NT;
                on[u] = false;
                if (q < M) {
                    const uint32_t e = B.ord[cur][q];
                    const uint32_t de = B.d[e];
                    on[u] = de != DONE;
                    if (on[u]) kk[u] = kc.key(P.S, B.st[e], B.ln[e], de);
                }
            }
#pragma unroll
            for (int u = 0; u < PER; ++u)
                if (on[u]) B.kq[tid + u * NT] = kk[u];
        }
        __syncthreads();
        mk(PH_BKEY);
        // rank inside the class by (key, position): the keys below, plus the
        // equal keys at earlier positions (positions inside a class follow
        // input order: every redistribution and round is stable)
        {
            uint32_t np[PER];
            uint64_t kk[PER];
            bool on[PER];
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const uint32_t q = tid + u * NT;
                on[u] = false;
                np[u] = q;
                if (q >= M) continue;
                if (B.d[B.ord[cur][q]] == DONE) continue;
                on[u] = true;
                const uint32_t cl = B.cls[q], c0 = cl & 0xFFFF, c1 = cl >> 16;
                const uint64_t k = B.kq[q];
                kk[u] = k;
                // eight, then four keys a trip: their LDS reads are issued
                // together (one at a time, each waited for its read)
                uint32_t r = 0;
                uint32_t j = c0;
                for (; j + 8 <= c1; j += 8) {
                    uint64_t a[8];
#pragma unroll
                    for (int t = 0; t < 8; ++t) a[t] = B.kq[j + t];
                    const int qd = (int)q - (int)j;
                    rank_pair<0>(r, a[0], a[1], k, qd);
                    rank_pair<2>(r, a[2], a[3], k, qd);
                    rank_pair<4>(r, a[4], a[5], k, qd);
                    rank_pair<6>(r, a[6], a[7], k, qd);
                }
                for (; j + 4 <= c1; j += 4) {
                    const uint64_t a0 = B.kq[j], a1 = B.kq[j + 1], a2 = B.kq[j + 2], a3 = B.kq[j + 3];
                    const int qd = (int)q - (int)j;
                    rank_pair<0>(r, a0, a1, k, qd);
                    rank_pair<2>(r, a2, a3, k, qd);
                }
                for (; j < c1; ++j) {
                    const uint64_t kj = B.kq[j];
                    r += (j < q ? kj <= k : kj < k) ? 1u : 0u;
                }
                np[u] = c0 + r;
            }
            __syncthreads();
            // keys and elements at their new positions (a class keeps its
            // positions; finished elements stay where they are)
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const uint32_t q = tid + u * NT;
                if (q >= M) continue;
                B.ord[cur ^ 1][np[u]] = B.ord[cur][q];
                if (on[u]) B.kq[np[u]] = kk[u];
            }
        }
        __syncthreads();
        // runs of equal keys in the new order: a run's first element gets its
        // lcp with the largest smaller key of its class (its new predecessor),
        // equal keys that end their strings are identical strings (lcp =
        // length), runs of two or more without an end stay active 8
        // characters deeper; each run start begins a class
        for (uint32_t p = tid; p < M; p += NT) {
            const uint32_t e = B.ord[cur ^ 1][p];
            const uint32_t de = B.d[e];
            if (de == DONE) {
                B.scr[p] = p;
                continue;
            }
            const uint32_t cl = B.cls[p], c0 = cl & 0xFFFF, c1 = cl >> 16;
            const uint64_t k = B.kq[p];
            const bool first = p == c0 || B.kq[p - 1] != k;
            const bool last = p + 1 == c1 || B.kq[p + 1] != k;
            if (first) {
                if (p > c0 && P.lcp) P.lcp[B.gp[p]] = de + kc.eqc(k ^ B.kq[p - 1]);
            } else if (kc.ends(k)) {
                if (P.lcp) P.lcp[B.gp[p]] = B.ln[e];
            }
            const bool go = !(first && last) && !kc.ends(k);
            B.d[e] = go ? de + kc.q() : DONE;
            if (go) B.any = 1;
            B.scr[p] = first ? p : 0u;
        }
        __syncthreads();
        mk(PH_BRANK);
        cur ^= 1;
        more = uni(B.any) != 0;
        if (more) {
            // class starts by a max-scan over the run starts, class ends at
            // each class's last position (kept in the key array meanwhile)
            block_scan(B.scr, (int)M, tmp, false, MaxOp(), 0u);
            uint32_t *cend = reinterpret_cast<uint32_t *>(B.kq);
            for (uint32_t q = tid; q < M; q += NT)
                if (q + 1 == M || B.scr[q + 1] != B.scr[q]) cend[B.scr[q]] = q + 1;
            __syncthreads();
            // and the next round's running minimum of each active class
            // starts at its head (only the head's thread reads that slot here)
            for (uint32_t q = tid; q < M; q += NT) {
                const uint32_t c0 = B.scr[q];
                B.cls[q] = c0 | (cend[c0] << 16);
                if (c0 == q && B.d[B.ord[cur][q]] != DONE) B.scr[q] = 0xFFFFFFFFu;
            }
            if (tid == 0) B.nlist = 0;
        }
        __syncthreads();
        if (tid == 0) B.any = 0;
        mk(PH_BSPLIT);
    }
    for (uint32_t q = tid; q < M; q += NT) P.perm[B.gp[q]] = B.id[B.ord[cur][q]] - setbase;
    if (tid == 0) {
        const unsigned long long dt = wall_clock64() - t_start;
        st[ST_CHUNKS] += 1;
        st[ST_ROUNDS] += rounds;
        st[ST_MAX_CHUNK] = max(st[ST_MAX_CHUNK], (dt << 24) | ((unsigned long long)min(rounds, 4095u) << 12) | M);
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Per-workgroup state of the persistent worker.
template <int K, int C>
struct StepLDS {
    Split sp;
    uint32_t hist[NBPAD];     // strings per bucket
    uint32_t bst[NBPAD];      // bucket start, relative to the segment
    uint32_t psz[NBPAD + 1];  // exclusive size prefix over the small buckets
    uint16_t lsmall[NBPAD];
    union {
        struct {
            uint16_t llarge[NBPAD];
            uint16_t lident[NBPAD];   // identical buckets, later the publish rank of each chunk
        };
        uint32_t gdep[NBPAD];         // a published chunk's group depths
    };
    uint16_t cfirst[NBPAD + 1];       // first small bucket of each chunk (bit 15: published)
    uint32_t nsmall, nlarge, nident, nchunk, npub, qfail;
    unsigned long long dbase, qpos2;
    unsigned long long best;
    unsigned long long qpos;
    unsigned long long ph[NPH];   // this workgroup's time per phase (thread 0)
    unsigned long long st[NST];   // this workgroup's statistics (thread 0)
    unsigned long long ph_last;
    uint32_t ext_min, nlist;
    uint32_t hstep;               // depth of the last step's classification (after any extension)
    uint32_t tmp[NW];
    union {
        struct {
            uint64_t samp[SAMPLE_MAX + 1];
            uint64_t srt[SAMPLE_MAX + 1];
            uint32_t fl[SAMPLE_MAX + 1];
        } s;
        ScatterLDS<K> sc;
        BaseLDS<C> base;
    } u;
};

// Charge the time since the last mark to phase i (thread 0 only; called
// right after a barrier, so it measures the workgroup's progress).
template <typename LDS>
__device__ __forceinline__ void mark(LDS &L, int i) {
    if (threadIdx.x == 0) {
        const unsigned long long now = wall_clock64();
        L.ph[i] += now - L.ph_last;
        L.ph_last = now;
    }
}

// Common depth of bucket b's strings after a step at depth h (Algorithm 1's
// output): h for the outer buckets b_0 and b_2v, h plus the splitter LCP for
// the other range buckets, h + q (8 characters, or more with alphabet
// compression) for equality buckets.
template <typename SP>
__device__ __forceinline__ uint32_t child_depth(const SP &sp, uint32_t h, uint32_t b) {
    if (b & 1) return h + sp.q;
    if (b == 0 || b == sp.nb - 1) return h;
    return h + sp.hl[b >> 1];
}

struct DescGroups {   // a chunk's groups, unpacked from their descriptors into LDS
    const uint32_t *start, *size, *depth, *pre;
    __device__ uint32_t gstart(uint32_t g) const { return start[g]; }
    __device__ uint32_t gsize(uint32_t g) const { return size[g]; }
    __device__ uint32_t gdepth(uint32_t g) const { return depth[g]; }
    __device__ uint32_t gpre(uint32_t g) const { return pre[g]; }
};

__device__ __forceinline__ unsigned long long uni64(unsigned long long x) {
    return ((unsigned long long)uni((uint32_t)(x >> 32)) << 32) | uni((uint32_t)x);
}

// Wait until queue position `pos` holds a task.  Executed by every lane of one
// wave with wave-uniform values only (no loop inside a lane-divergent region:
// a spin loop run by one lane next to barriers can be lowered so that the
// other lanes pass a barrier without it).  Polls with relaxed agent-scope
// loads (no cache invalidation per poll), sleeps between polls with a growing
// pause (up to about 4000 cycles), and issues one acquire fence when the task
// is there.  Returns 1 (task ready), 0 (queue drained:
// nothing pending, so nothing can be enqueued any more) or -1 (device error or
// the wait limit, by wall clock or by poll count).
__device__ __forceinline__ int poll_slot(const Params &P, Slot *s, unsigned long long pos) {
    const unsigned long long t0 = wall_clock64();
    uint32_t nap = 1;
    for (unsigned long long it = 0;; ++it) {
        if (uni64(ld_rlx(&s->seq)) == pos + 1) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            return 1;
        }
        // the shared counters only every 8th poll (the slot is this
        // workgroup's own line; the counters are everybody's)
        if ((it & 7) == 7) {
            if (uni64(ld_rlx(&P.ctl->pending)) == 0) return 0;
            if (uni64(ld_rlx(&P.ctl->error)) != 0) return -1;
        }
        if (wall_clock64() - t0 > P.limit_ticks || it > P.limit_iters) {
            if (lane_id() == 0)
                __hip_atomic_fetch_or(&P.ctl->error, ERR_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return -1;
        }
        for (uint32_t k = 0; k < nap; ++k) __builtin_amdgcn_s_sleep(8);
        nap = min(2 * nap, 8u);
    }
}

// Publishing a task (already counted in `pending`) at queue position pos takes
// two steps: stage() writes the slot's fields, and after the workgroup has
// released its writes (release_wg: records, descriptors, slot fields),
// commit() sets the slot's sequence number with a relaxed store.  One
// attempt, no waiting: the ring is sized so that the slot's previous occupant
// (pos - capacity) has long been consumed; if it has not, the sort fails with
// a device error (and *fail is set, so that nothing is committed) instead of
// overwriting it.
__device__ __forceinline__ void stage(const Params &P, unsigned long long pos, const Task &t, uint32_t *fail) {
    Slot *s = &P.ring[pos & P.ring_mask];
    if (ld_rlx(&s->seq) != pos) {
        __hip_atomic_fetch_or(&P.ctl->error, ERR_QUEUE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        *fail = 1;
        return;
    }
    st_coh32(&s->begin, t.begin);
    st_coh32(&s->size, t.size);
    st_coh32(&s->depth, t.depth);
    st_coh32(&s->meta, t.meta);
    st_coh32(&s->setbase, t.setbase);
}
__device__ __forceinline__ void commit(const Params &P, unsigned long long pos) {
    st_rlx(&P.ring[pos & P.ring_mask].seq, pos + 1);
}

// Identical strings (an equality bucket whose splitter ends the string):
// already in input-index order; lcp between them is their length.
__device__ __forceinline__ void finish_ident(const Params &P, const Rec *src, uint32_t start, uint32_t cnt, uint32_t setbase) {
    for (uint32_t i = tid_here(); i < cnt; i += NT) {
        const Rec r = src[start + i];
        P.perm[start + i] = r.id - setbase;
        if (P.lcp && i > 0) P.lcp[start + i] = r.ln;
    }
}

// One classification step of a segment by one workgroup.  Returns true when
// `t` has been replaced by a child segment this workgroup continues with.
template <int K, int C, typename KC>
__device__ __forceinline__ bool seg_step(const Params &P, Task &t, StepLDS<K, C> &L, const KC &kc, bool coh) {
    const int tid = tid_here(), w = tid >> 6, lane = tid & 63;
    const uint32_t begin = t.begin, S = t.size, meta = t.meta;
    uint32_t h = t.depth;
    auto kload = [&](uint32_t e, uint32_t hh) -> uint64_t {
        const Rec r = load_rec(P, meta, begin + e, coh);
        return kc.key(P.S, r.st, r.ln, hh);
    };
    // at most two samples: the second after a common-prefix extension (one
    // call site keeps the persistent kernel's code small)
#pragma nounroll
    for (uint32_t pass = 0;; ++pass) {
    select_splitters(L.sp, S, h, hash32(begin * 0x85EBCA6Bu ^ h * 0xC2B2AE35u ^ S), P.vmax, P.equal, L.u.s.samp,
                     L.u.s.srt, L.u.s.fl, L.tmp, kload, kc);
    mark(L, PH_SAMPLE);
    if (pass != 0 || uni(L.sp.ndistinct) != 1 || uni((uint32_t)L.sp.zr[0]) != 0) break;
    {
        // Every sampled string has the same next 8 bytes: an equality chain.
        // Instead of one classification step per 8 equal bytes, find the
        // segment's exact common prefix (the minimum over its strings of the
        // LCP with its first string) and classify there.
        if (tid == 0) {
            L.ext_min = 0xFFFFFFFFu;
            L.nlist = 0;
        }
        __syncthreads();
        const Rec f = load_rec(P, meta, begin, coh);
        uint64_t fk[4];
        keys32_at(P.S.chars, P.S.nchars, f.st, f.ln, h, fk);
        uint32_t *list = reinterpret_cast<uint32_t *>(L.u.s.samp);   // 4 * NT entries
        // four strings per thread at a time: their records, then their first
        // 32 bytes (16 independent loads), then the comparisons; the strings
        // equal to the first one on all 32 bytes go on in a list
        for (uint32_t b0 = 1; b0 < S; b0 += 4 * NT) {
            const uint32_t e0 = b0 + tid;
            Rec r[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (e0 + u * NT < S) r[u] = load_rec(P, meta, begin + e0 + u * NT, coh);
            uint64_t k[4][4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (e0 + u * NT < S) keys32_at(P.S.chars, P.S.nchars, r[u].st, r[u].ln, h, k[u]);
                else k[u][0] = k[u][1] = k[u][2] = k[u][3] = 0;
            }
            uint32_t res = 0xFFFFFFFFu;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                bool done = e0 + u * NT >= S;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    if (done) continue;
                    if (k[u][i] != fk[i]) {
                        res = min(res, h + 8 * i + (uint32_t)(__clzll(k[u][i] ^ fk[i]) >> 3));
                        done = true;
                    } else if ((fk[i] & 0xFF) == 0) {
                        res = min(res, min(f.ln, r[u].ln));
                        done = true;
                    }
                }
                if (!done) list[atomicAdd(&L.nlist, 1u)] = e0 + u * NT;
            }
            if (res != 0xFFFFFFFFu) atomicMin(&L.ext_min, res);
            __syncthreads();
            const uint32_t n = uni(L.nlist);
            __syncthreads();
            if (tid == 0) L.nlist = 0;
            const uint32_t gw = group_width(n);
            if (gw) {
                for (uint32_t i0 = 0; i0 < n; i0 += NT / gw) {
                    const uint32_t i = i0 + tid / gw;
                    const bool on = i < n;
                    const Rec q = load_rec(P, meta, begin + (on ? list[i] : 0u), coh);
                    const uint32_t l = group_lcp(P, gw, on, f.st, f.ln, q.st, q.ln, h + 32, &L.ext_min);
                    if (on && (tid & (gw - 1)) == 0) atomicMin(&L.ext_min, l);
                }
            } else {
                for (uint32_t i = tid; i < n; i += NT) {
                    const Rec q = load_rec(P, meta, begin + list[i], coh);
                    atomicMin(&L.ext_min, lcp_from(P, f.st, f.ln, q.st, q.ln, h + 32, &L.ext_min));
                }
            }
            __syncthreads();
        }
        h = uni(L.ext_min);
        mark(L, PH_EXTEND);
    }
    }
    for (int b = tid; b < NBPAD; b += NT) L.hist[b] = 0;
    if (tid == 0) {
        L.st[ST_SEGMENTS] += 1;
        L.st[ST_STRINGS] += S;
        L.st[ST_MAX_DEPTH] = max(L.st[ST_MAX_DEPTH], (unsigned long long)h);
        L.hstep = h;
    }
    __syncthreads();
    const uint32_t nb = uni(L.sp.nb);
    const int nbits = (int)uni(L.sp.nbits);
    const uint32_t CK = NT * K;
    // classify and count
    for (uint32_t c0 = 0; c0 < S; c0 += CK) {
        Rec r[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const uint32_t e = c0 + (uint32_t)(w * 64 * K + j * 64 + lane);
            if (e < S) r[j] = load_rec(P, meta, begin + e, coh);
        }
        uint64_t k[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const uint32_t e = c0 + (uint32_t)(w * 64 * K + j * 64 + lane);
            k[j] = (e < S) ? kc.key(P.S, r[j].st, r[j].ln, h) : 0;
        }
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const uint32_t e = c0 + (uint32_t)(w * 64 * K + j * 64 + lane);
            const bool valid = e < S;
            const uint32_t m = valid ? classify_any(k[j], L.sp) : nb;
            const uint64_t mask = match_any(m, nbits);
            if (valid && lane == 63 - (int)__clzll(mask)) atomicAdd(&L.hist[m], (uint32_t)__popcll(mask));
            if (valid) P.bkt[begin + e] = (uint16_t)m;
        }
    }
    __syncthreads();
    mark(L, PH_CLASSIFY);
    for (int b = tid; b < NBPAD; b += NT) L.bst[b] = (uint32_t)b < nb ? L.hist[b] : 0u;
    __syncthreads();
    block_scan(L.bst, (int)nb, L.tmp, true, AddOp(), 0u);
    for (int b = tid; b < NBPAD; b += NT) L.u.sc.run[b] = begin + L.bst[b];
    __syncthreads();
    const bool to1 = out_is_r1(meta);
    Rec *out = to1 ? P.R1 : P.R0;
    for (uint32_t c0 = 0; c0 < S; c0 += CK) {
        Rec r[K];
        uint32_t m[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const uint32_t e = c0 + (uint32_t)(w * 64 * K + j * 64 + lane);
            if (e < S) {
                r[j] = load_rec(P, meta, begin + e, coh);
                m[j] = P.bkt[begin + e];
            } else {
                m[j] = nb;
            }
        }
        scatter_chunk<K>(L.u.sc, L.tmp, nb, nbits, m, r, nullptr, min(CK, S - c0), L.u.sc.run, out, nullptr, P.S.n,
                         &P.ctl->error);
    }
    // the redistributed records are visible to this workgroup now; to the
    // others with the one release before the tasks are committed
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    mark(L, PH_SCATTER);

    // ---- children (Algorithm 1 output: bucket i has common prefix h + h'_{i/2}
    // for even i, except the outer buckets which keep h, and h + 8 for odd i) ----
    const uint32_t cpar = to1 ? M_PARITY : 0u;
    if (tid == 0) {
        L.nlarge = 0;
        L.nident = 0;
        L.best = 0;
        L.qfail = 0;
        L.npub = 0;
    }
    __syncthreads();
    for (uint32_t b = tid; b < nb; b += NT) {
        const uint32_t cnt = L.hist[b], st = L.bst[b];
        uint32_t small = 0;
        if (cnt) {
            const uint32_t l = b >> 1;
            const bool odd = b & 1;
            if (P.lcp && st > 0) P.lcp[begin + st] = SEAM | h;
            if (odd && L.sp.zr[l]) {
                L.lident[atomicAdd(&L.nident, 1u)] = (uint16_t)b;
            } else if (cnt <= P.tbase) {
                small = 1;
            } else {
                const uint32_t k = atomicAdd(&L.nlarge, 1u);
                L.llarge[k] = (uint16_t)b;
                atomicMax(&L.best, ((unsigned long long)cnt << 16) | k);
            }
        }
        L.psz[b] = small;
    }
    __syncthreads();
    const uint32_t nsmall = uni(block_scan(L.psz, (int)nb, L.tmp, true, AddOp(), 0u));
    for (uint32_t b = tid; b < nb; b += NT) {
        const uint32_t cnt = L.hist[b];
        if (cnt && cnt <= P.tbase && !((b & 1) && L.sp.zr[b >> 1])) L.lsmall[L.psz[b]] = (uint16_t)b;
    }
    __syncthreads();
    // size prefix over the small list
    for (uint32_t k = tid; k < nsmall; k += NT) L.psz[k] = L.hist[L.lsmall[k]];
    __syncthreads();
    const uint32_t small_total = block_scan(L.psz, (int)nsmall, L.tmp, true, AddOp(), 0u);
    if (tid == 0) L.psz[nsmall] = small_total;
    // large children: keep the largest, queue the others
    const uint32_t nlarge = uni(L.nlarge);
    const uint32_t keep = uni((uint32_t)(L.best & 0xFFFF));
    if (tid == 0 && nlarge > 1) {
        add_agent(&P.ctl->pending, (unsigned long long)(nlarge - 1));
        L.qpos = add_agent(&P.ctl->tail, (unsigned long long)(nlarge - 1));
    }
    __syncthreads();
    if (nlarge > 1) {
        for (uint32_t k = tid; k < nlarge; k += NT) {
            if (k == keep) continue;
            const uint32_t b = L.llarge[k];
            Task c{begin + L.bst[b], L.hist[b], child_depth(L.sp, h, b), cpar, t.setbase};
            stage(P, L.qpos + (k < keep ? k : k - 1), c, &L.qfail);
        }
    }
    // identical buckets
    const uint32_t nident = uni(L.nident);
    for (uint32_t k = 0; k < nident; ++k) {
        const uint32_t b = L.lident[k];
        finish_ident(P, out, begin + L.bst[b], L.hist[b], t.setbase);
    }
    __syncthreads();
    // the child this workgroup goes on with (read before the chunks reuse
    // the bucket arrays)
    Task next{0, 0, 0, 0, 0};
    if (nlarge >= 1) {
        const uint32_t b = uni(L.llarge[keep]);
        next = Task{begin + uni(L.bst[b]), uni(L.hist[b]), child_depth(L.sp, h, b), cpar, t.setbase};
    }
    // small buckets: base-case chunks of at most C strings, never splitting a
    // group.  Every small bucket gets a group descriptor (at most one per
    // group over the whole sort); chunks of at least cap / 2 strings become
    // tasks of their own so that idle workgroups sort them, except the last
    // one when this workgroup has no large child to go on with; the rest are
    // sorted here after the step.
    uint32_t nchunk = 0;
    if (nsmall) {
        const uint32_t cap = (P.tbase * 2 <= (uint32_t)C) ? (uint32_t)C - P.tbase : 0u;
        for (uint32_t k = tid; k < nsmall; k += NT) {
            const uint32_t ck = cap ? L.psz[k] / cap : k;
            const uint32_t cp = k ? (cap ? L.psz[k - 1] / cap : k - 1) : 0xFFFFFFFFu;
            if (ck != cp) L.cfirst[ck] = (uint16_t)k;
            if (k == nsmall - 1) L.nchunk = ck + 1;
        }
        __syncthreads();
        nchunk = uni(L.nchunk);
        if (tid == 0) {
            L.cfirst[nchunk] = (uint16_t)nsmall;
            L.st[ST_BASE] += nsmall;
            const unsigned long long db = add_agent(&P.ctl->desc_top, (unsigned long long)nsmall);
            uint32_t npub = 0;
            if (db + nsmall > P.desc_cap) {
                atomicOr(&P.ctl->error, ERR_DESC_CAP);
                L.nchunk = 0;
            } else if (cap) {
                for (uint32_t c = 0; c < nchunk; ++c) {
                    const uint32_t k0 = L.cfirst[c], k1 = L.cfirst[c + 1];
                    const bool last = c + 1 == nchunk;
                    if ((!last || nlarge >= 1) && L.psz[k1] - L.psz[k0] >= cap / 2) {
                        L.lident[c] = (uint16_t)npub++;
                        L.cfirst[c] = (uint16_t)(k0 | 0x8000u);
                    }
                }
                if (npub) {
                    add_agent(&P.ctl->pending, (unsigned long long)npub);
                    L.qpos2 = add_agent(&P.ctl->tail, (unsigned long long)npub);
                    L.st[ST_PUBCHUNKS] += npub;
                }
            }
            L.dbase = db;
            L.npub = npub;
        }
        __syncthreads();
        nchunk = uni(L.nchunk);
        if (nchunk) {
            const unsigned long long db = uni64(L.dbase);
            for (uint32_t k = tid; k < nsmall; k += NT) {
                const uint32_t b = L.lsmall[k];
                st_desc(&P.desc[db + k], begin + L.bst[b], L.hist[b], child_depth(L.sp, h, b));
            }
            if (uni(L.npub)) {
                for (uint32_t c = tid; c < nchunk; c += NT) {
                    const uint32_t f0 = L.cfirst[c];
                    if (!(f0 & 0x8000)) continue;
                    const uint32_t k0 = f0 & 0x7FFF, k1 = L.cfirst[c + 1] & 0x7FFF;
                    stage(P, L.qpos2 + L.lident[c],
                          Task{(uint32_t)(db + k0), k1 - k0, L.psz[k1] - L.psz[k0], M_CHUNK | cpar, t.setbase},
                          &L.qfail);
                }
            }
        }
    } else if (tid == 0) {
        L.nchunk = 0;
    }
    // one release for the step's records, descriptors and slot fields, then
    // the sequence numbers that hand the tasks over
    const uint32_t npub = uni(L.npub);
    if (nlarge > 1 || npub) {
        release_wg();
        if (!uni(L.qfail)) {
            for (uint32_t k = tid; k + 1 < nlarge; k += NT) commit(P, L.qpos + k);
            for (uint32_t k = tid; k < npub; k += NT) commit(P, L.qpos2 + k);
        }
    } else {
        __builtin_amdgcn_s_waitcnt(0);
    }
    __syncthreads();
    mark(L, PH_CHILDREN);
    if (nlarge >= 1) {
        t = next;
        return true;
    }
    return false;
}

template <int K, int C, typename KC>
__device__ __forceinline__ void run_task(const Params &P, Task t, StepLDS<K, C> &L, const KC &kc) {
    if (t.size == 0) return;
    if (t.meta & M_IDENT) {
        const Rec *src = (t.meta & M_PARITY) ? P.R1 : P.R0;
        finish_ident(P, src, t.begin, t.size, t.setbase);
        __syncthreads();
        mark(L, PH_CHILDREN);
        return;
    }
    const int tid = tid_here();
    bool seg = false;              // t is a segment still to classify
    uint32_t ud0 = 0, ung = 0;     // group descriptors to unpack next
    uint32_t ng = 0;               // groups ready in the bucket arrays
    uint32_t nchunk = 0, c = 0;    // chunks of the last step, the next to look at
    unsigned long long db = 0;
    bool coh = true;               // the data to read next was written by another workgroup
    const Rec *src = (t.meta & M_PARITY) ? P.R1 : P.R0;
    if (t.meta & M_CHUNK) {
        ud0 = t.begin;
        ung = t.size;
    } else if (t.size <= P.tbase) {
        if (t.meta & M_IDENT_SRC) {
            // a whole set small enough for the base case: stage its records first
            for (uint32_t i = tid; i < t.size; i += NT) P.R0[t.begin + i] = make_rec(P.S, t.begin + i);
            __threadfence();
            src = P.R0;
            coh = false;
        }
        if (tid == 0) {
            L.bst[0] = t.begin;
            L.hist[0] = t.size;
            L.psz[0] = t.size;
            L.gdep[0] = t.depth;
            L.st[ST_BASE] += 1;
        }
        __syncthreads();
        ng = 1;
    } else {
        seg = true;
    }
    for (;;) {
        if (ung) {
            // a descriptor outside the string range or a chunk larger than
            // the LDS holds is a device error, never an access
            if (tid == 0) L.qfail = 0;
            __syncthreads();
            for (uint32_t g = tid; g < min(ung, (uint32_t)NBPAD); g += NT) {
                GroupDesc d;
                if (coh) {
                    const uint64_t *q = reinterpret_cast<const uint64_t *>(&P.desc[ud0 + g]);
                    const uint64_t a = ld_coh64(q), b = ld_coh64(q + 1);
                    d = GroupDesc{(uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32)};
                } else {
                    d = P.desc[ud0 + g];
                }
                if (d.start > P.S.n || d.size > P.S.n - d.start || d.size == 0 || d.size > P.tbase) L.qfail = 1;
                L.bst[g] = d.start;
                L.hist[g] = d.size;
                L.psz[g] = d.size;
                L.gdep[g] = d.depth;
            }
            __syncthreads();
            ng = uni((ung > (uint32_t)NBPAD || L.qfail) ? 0u : ung);
            if (ng == 0 && tid == 0) atomicOr(&P.ctl->error, ERR_TASK);
            ung = 0;
        }
        if (ng) {
            const uint32_t M = uni(block_scan(L.psz, (int)ng, L.tmp, true, AddOp(), 0u));
            if (M > (uint32_t)C) {
                if (tid == 0) atomicOr(&P.ctl->error, ERR_CHUNK);
            } else {
                DescGroups g{L.bst, L.hist, L.gdep, L.psz};
                base_chunk<C>(P, L.u.base, L.tmp, src, t.setbase, ng, M, g, [&](int i) { mark(L, i); }, L.st, kc, coh);
            }
            mark(L, PH_BASE);
            ng = 0;
        }
        // the last step's chunks that stayed here
        while (c < nchunk && (uni(L.cfirst[c]) & 0x8000)) ++c;
        if (c < nchunk) {
            const uint32_t k0 = uni(L.cfirst[c]), k1 = uni(L.cfirst[c + 1]) & 0x7FFF;
            ud0 = (uint32_t)(db + k0);
            ung = k1 - k0;
            ++c;
            continue;
        }
        if (!seg) break;
        const bool to1 = out_is_r1(t.meta);
        seg = seg_step<K, C>(P, t, L, kc, coh);
        coh = false;   // the next child and the local chunks are this workgroup's own output
        src = to1 ? P.R1 : P.R0;
        nchunk = uni(L.nchunk);
        db = uni64(L.dbase);
        c = 0;
    }
}

// The key codec of a launch: bytes, or the input's packed alphabet codes.
template <bool Z> struct KeyOf;
template <> struct KeyOf<false> {
    static __device__ __forceinline__ ByteKey make(const Params &) { return ByteKey{}; }
};
template <> struct KeyOf<true> {
    static __device__ __forceinline__ PackedKey make(const Params &P) {
        return PackedKey{P.alpha->code, P.alpha->b, P.alpha->q};
    }
};

#ifndef SSD_WORKER_OCC
#define SSD_WORKER_OCC 4
#endif

template <int K, int C, bool Z>
__global__ __launch_bounds__(NT, SSD_WORKER_OCC) void k_worker(Params P) {
    __shared__ StepLDS<K, C> L;
    __shared__ unsigned long long claim;
    __shared__ int outcome;
    if (P.ctl->error) return;
    const int w = threadIdx.x >> 6;
    if (threadIdx.x < NPH) L.ph[threadIdx.x] = 0;
    if (threadIdx.x < NST) L.st[threadIdx.x] = 0;
    if (threadIdx.x == 0) L.ph_last = wall_clock64();
    for (;;) {
        // a barrier between the previous task's thread-0 epilogue and this
        // claim keeps the two thread-0 regions from being merged across the
        // loop's back edge (which would let the other lanes loop without it)
        __syncthreads();
        if (threadIdx.x == 0)
            claim = __hip_atomic_fetch_add(&P.ctl->head, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const unsigned long long pos = uni64(claim);
        Slot *s = &P.ring[pos & P.ring_mask];
        // one wave polls, the others wait at the barrier
        if (uni((uint32_t)w) == 0) {
            const int oc = poll_slot(P, s, pos);
            if (lane_id() == 0) outcome = oc;
        }
        __syncthreads();
        const int o = (int)uni((uint32_t)outcome);
        mark(L, o > 0 ? PH_WAIT : PH_DRAIN);
        if (o <= 0) break;
        const Task t{uni(ld_coh32(&s->begin)), uni(ld_coh32(&s->size)), uni(ld_coh32(&s->depth)),
                     uni(ld_coh32(&s->meta)), uni(ld_coh32(&s->setbase))};
        __syncthreads();   // every wave has read the slot: hand it back to the ring
        if (threadIdx.x == 0) st_rlx(&s->seq, pos + P.ring_mask + 1);
        const unsigned long long t_task = wall_clock64();
        if (t.begin > P.S.n || t.size > P.S.n - t.begin) {
            if (threadIdx.x == 0) atomicOr(&P.ctl->error, ERR_TASK);
        } else {
            run_task<K, C>(P, t, L, KeyOf<Z>::make(P));
        }
        if (threadIdx.x == 0)
            L.st[ST_MAX_TASK] = max(L.st[ST_MAX_TASK], ((wall_clock64() - t_task) << 24) | min(t.size, 0xFFFFFFu));
        // the task's outputs need no release: nothing in this launch reads
        // them, and the launch's end makes them visible
        __syncthreads();
        mark(L, PH_OTHER);
        if (threadIdx.x == 0) add_agent(&P.ctl->pending, ~0ull);
    }
    __syncthreads();
    if (threadIdx.x < NPH)
        __hip_atomic_fetch_add(&P.ctl->ph[threadIdx.x], L.ph[threadIdx.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (threadIdx.x < NST && L.st[threadIdx.x]) {
        if (threadIdx.x >= ST_MAX_DEPTH)
            __hip_atomic_fetch_max(&P.ctl->st[threadIdx.x], L.st[threadIdx.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
            __hip_atomic_fetch_add(&P.ctl->st[threadIdx.x], L.st[threadIdx.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ---------------------------------------------------------------------------
// Initialisation: queue ring sequence numbers and the control block.
__global__ void k_init(Params P, unsigned long long cap) {
    const unsigned long long i0 = blockIdx.x * (unsigned long long)NT + threadIdx.x;
    const unsigned long long stride = (unsigned long long)gridDim.x * NT;
    for (unsigned long long i = i0; i < cap; i += stride) P.ring[i].seq = i;
    if (i0 == 0) {
        Ctl *c = P.ctl;
        c->head = 0;
        c->tail = 0;
        c->pending = 0;
        c->error = 0;
        c->desc_top = 0;
        for (int l = 0; l < LMAX; ++l) c->lvl[l][0] = c->lvl[l][1] = 0;
        for (int k = 0; k < NST; ++k) c->st[k] = 0;
        for (int k = 0; k < NPH; ++k) c->ph[k] = 0;
    }
    if (P.alpha && i0 < 8) P.alpha->present[i0] = 0;
}

// Alphabet compression, first pass: the byte values that occur in the
// character buffer (aligned words inside it, the partial words at its two
// ends byte by byte; the value 0 ends strings and is never a character).  Each
// thread keeps a 256-bit set in registers, then ORs it into the workgroup's
// and the device's.
__global__ __launch_bounds__(NT) void k_alpha_scan(Params P) {
    __shared__ uint32_t bm[8];
    if (threadIdx.x < 8) bm[threadIdx.x] = 0;
    __syncthreads();
    const uintptr_t a = (uintptr_t)P.S.chars, e = a + P.S.nchars;
    const uint32_t lead = (uint32_t)(a & 7);   // bytes of the first aligned word before the buffer
    const uint64_t nw = P.S.nchars ? (e + 7 - (a - lead)) >> 3 : 0;
    uint64_t m0 = 0, m1 = 0, m2 = 0, m3 = 0;
    for (uint64_t i = blockIdx.x * (uint64_t)NT + threadIdx.x; i < nw; i += (uint64_t)gridDim.x * NT) {
        // word i starts lead bytes before chars + 8i (pointer arithmetic from
        // chars: the loads stay global-memory loads)
        const int64_t o = (int64_t)(8 * i) - (int64_t)lead;   // its offset from chars
        const bool whole = o >= 0 && (uint64_t)o + 8 <= P.S.nchars;
        // the two edge words are read byte by byte: no load leaves the buffer
        uint64_t w = 0;
        if (whole) {
            w = *reinterpret_cast<const uint64_t *>(P.S.chars + o);
        } else {
            for (int b = 0; b < 8; ++b)
                if (o + b >= 0 && (uint64_t)(o + b) < P.S.nchars) w |= (uint64_t)P.S.chars[o + b] << (8 * b);
        }
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint32_t c = (uint32_t)(w >> (8 * b)) & 0xFF;
            const bool in = whole || (o + b >= 0 && (uint64_t)(o + b) < P.S.nchars);
            const uint64_t bit = in ? 1ull << (c & 63) : 0ull;
            m0 |= (c >> 6) == 0 ? bit : 0ull;
            m1 |= (c >> 6) == 1 ? bit : 0ull;
            m2 |= (c >> 6) == 2 ? bit : 0ull;
            m3 |= (c >> 6) == 3 ? bit : 0ull;
        }
    }
    const uint64_t mm[4] = {m0, m1, m2, m3};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if ((uint32_t)mm[k]) atomicOr(&bm[2 * k], (uint32_t)mm[k]);
        if ((uint32_t)(mm[k] >> 32)) atomicOr(&bm[2 * k + 1], (uint32_t)(mm[k] >> 32));
    }
    __syncthreads();
    if (threadIdx.x < 8 && bm[threadIdx.x]) atomicOr(&P.alpha->present[threadIdx.x], bm[threadIdx.x]);
}

// Second pass (one workgroup): the order-preserving codes, bits per
// character and characters per key.
__global__ __launch_bounds__(NT) void k_alpha_codes(Params P) {
    __shared__ uint32_t pres[8];
    Alphabet *A = P.alpha;
    if (threadIdx.x < 8) pres[threadIdx.x] = A->present[threadIdx.x] & (threadIdx.x == 0 ? ~1u : ~0u);
    __syncthreads();
    const uint32_t c = threadIdx.x;   // NT == 256 byte values
    uint32_t below = 0;
    for (uint32_t k = 0; k < (c >> 5); ++k) below += __popc(pres[k]);
    below += __popc(pres[c >> 5] & ((1u << (c & 31)) - 1u));
    const bool here = (pres[c >> 5] >> (c & 31)) & 1u;
    A->code[c] = here ? (uint8_t)(below + 1) : (uint8_t)0;
    if (c == 0) {
        uint32_t sigma = 0;
        for (int k = 0; k < 8; ++k) sigma += __popc(pres[k]);
        const uint32_t b = sigma ? 32 - __clz(sigma) : 1u;   // values 0..sigma
        A->sigma = sigma;
        A->b = b;
        A->q = min(64u / b, 32u);
    }
}

// Optional input validation: bounds and zero bytes.
__global__ void k_validate(Params P) {
    const uint32_t i0 = blockIdx.x * NT + threadIdx.x, stride = gridDim.x * NT;
    if (P.S.flags & TO_END) {
        for (uint64_t p = i0; p < P.S.nchars; p += stride)
            if (P.S.chars[p] == 0) atomicOr(&P.ctl->error, ERR_ZERO);
        for (uint32_t i = i0; i < P.S.n; i += stride)
            if (P.S.off[i] > P.S.nchars || P.S.nchars - P.S.off[i] >= 0x80000000ull) atomicOr(&P.ctl->error, ERR_BOUNDS);
        return;
    }
    for (uint32_t i = i0; i < P.S.n; i += stride) {
        const uint64_t st = P.S.off[i];
        uint64_t ln;
        if (P.S.len) ln = P.S.len[i];
        else ln = P.S.off[i + 1] >= st ? P.S.off[i + 1] - st : ~0ull;
        if (st > P.S.nchars || ln > P.S.nchars - st || ln >= 0x80000000ull) {
            atomicOr(&P.ctl->error, ERR_BOUNDS);
            continue;
        }
        for (uint64_t p = 0; p < ln; ++p)
            if (P.S.chars[st + p] == 0) { atomicOr(&P.ctl->error, ERR_ZERO); break; }
    }
}

// ---------------------------------------------------------------------------
// Root step across the whole GPU (the fully parallel step of pS5).
// ---------------------------------------------------------------------------
// Whole-GPU levels.  Every segment of a level is classified and redistributed
// by the whole GPU: one workgroup samples each segment (k_lvl_sample), tiles
// of every segment are classified in parallel with per-tile histograms
// (k_lvl_classify), the histograms are scanned per segment and bucket
// (k_lvl_colscan), the tiles redistribute their records (k_lvl_scatter), and
// one workgroup per segment turns its buckets into the next level's segments,
// worker tasks and base-case chunk tasks (k_lvl_schedule).  A grid is sized
// for the level's capacity; workgroups beyond the level's count exit.

// Records of a segment: from the input (identity) or from a record buffer.
__device__ __forceinline__ Rec seg_rec(const Params &P, uint32_t meta, uint32_t i) {
    if (meta & M_IDENT_SRC) return make_rec(P.S, i);
    return ((meta & M_PARITY) ? P.R1 : P.R0)[i];
}

// Append a segment to level l (its tiles get consecutive numbers).
// Returns the segment's tile count once its record is written (0 on
// overflow); with fill = false the caller maps the tiles (*idx, *t0).
__device__ uint32_t lvl_append(const Params &P, uint32_t l, const LvlSeg &g0, bool fill = true, uint32_t *oidx = nullptr,
                               uint32_t *ot0 = nullptr) {
    LvlSeg g = g0;
    g.ntile = (g.size + P.tile - 1) / P.tile;
    const unsigned long long idx = add_agent(&P.ctl->lvl[l][0], 1ull);
    const unsigned long long t0 = add_agent(&P.ctl->lvl[l][1], (unsigned long long)g.ntile);
    if (idx >= P.lmaxseg || t0 + g.ntile > P.lmaxtiles) {
        atomicOr(&P.ctl->error, ERR_LEVEL);
        return 0;
    }
    g.tile0 = (uint32_t)t0;
    P.lseg[l][idx] = g;
    if (fill)
        for (uint32_t j = 0; j < g.ntile; ++j) P.tile2seg[l][t0 + j] = (uint32_t)idx;
    if (oidx) *oidx = (uint32_t)idx;
    if (ot0) *ot0 = (uint32_t)t0;
    return g.ntile;
}

// Put a worker task at a queue position reserved before the workers start
// (the launch boundary orders it before any read).
__device__ __forceinline__ void seed_task(const Params &P, unsigned long long pos, const Task &t) {
    Slot *s = &P.ring[pos & P.ring_mask];
    s->begin = t.begin;
    s->size = t.size;
    s->depth = t.depth;
    s->meta = t.meta;
    s->setbase = t.setbase;
    s->seq = pos + 1;
}

__device__ __forceinline__ uint32_t lvl_count(const Params &P, uint32_t l, int which) {
    return (uint32_t)min(P.ctl->lvl[l][which], which ? (unsigned long long)P.lmaxtiles : (unsigned long long)P.lmaxseg);
}

// Level 0: the whole input (mode 1) or every batched set (mode 2); a segment
// of at most ROOT_MIN strings (unless force) goes straight to the workers.
__global__ void k_seed(Params P, uint32_t mode, uint32_t depth, uint32_t force) {
    __shared__ uint32_t whole[3];   // mode 1: the input's level-0 segment, its first tile, its tile count
    if (threadIdx.x == 0) whole[2] = 0;
    __syncthreads();
    const uint32_t nset = P.ctl->error ? 0u : (mode == 1 ? 1u : P.m);
    for (uint32_t i = blockIdx.x * NT + threadIdx.x; i < nset; i += gridDim.x * NT) {
        const uint32_t b = mode == 1 ? 0u : P.set_begin[i], e = mode == 1 ? P.S.n : P.set_begin[i + 1];
        if (e <= b) continue;
        if (P.lcp) P.lcp[b] = 0;
        const uint32_t setbase = mode == 2 ? b : 0u;
        if (force || e - b > ROOT_MIN) {
            // the whole input (one launch of one workgroup) maps its tiles with every thread below
            if (mode == 1)
                whole[2] = lvl_append(P, 0, LvlSeg{b, e - b, depth, M_IDENT_SRC, 0, 0, setbase, 0}, false, &whole[0],
                                      &whole[1]);
            else
                lvl_append(P, 0, LvlSeg{b, e - b, depth, M_IDENT_SRC, 0, 0, setbase, 0});
        } else {
            add_agent(&P.ctl->pending, 1ull);
            seed_task(P, add_agent(&P.ctl->tail, 1ull), Task{b, e - b, depth, M_IDENT_SRC, setbase});
        }
    }
    __syncthreads();
    const uint32_t nt = whole[2];
    for (uint32_t j = threadIdx.x; j < nt; j += NT) P.tile2seg[0][whole[1] + j] = whole[0];
}

struct LvlSampleLDS {
    Split sp;
    uint64_t samp[SAMPLE_MAX + 1];
    uint64_t srt[SAMPLE_MAX + 1];
    uint32_t fl[SAMPLE_MAX + 1];
    uint32_t tmp[NW];
};

template <bool Z>
__global__ __launch_bounds__(NT) void k_lvl_sample(Params P, uint32_t l) {
    __shared__ LvlSampleLDS L;
    if (P.ctl->error || blockIdx.x >= lvl_count(P, l, 0)) return;
    const LvlSeg g = P.lseg[l][blockIdx.x];
    const auto kc = KeyOf<Z>::make(P);
    auto kload = [&](uint32_t e, uint32_t hh) -> uint64_t {
        const Rec r = seg_rec(P, g.meta, g.begin + e);
        return kc.key(P.S, r.st, r.ln, hh);
    };
    select_splitters(L.sp, g.size, g.depth, hash32(g.begin * 0x85EBCA6Bu ^ g.depth * 0xC2B2AE35u ^ g.size), P.vmax,
                     P.equal, L.samp, L.srt, L.fl, L.tmp, kload, kc);
    const uint32_t *src = (const uint32_t *)&L.sp;
    uint32_t *dst = (uint32_t *)&P.lsplit[l][blockIdx.x];
    for (uint32_t i = threadIdx.x; i < sizeof(Split) / 4; i += NT) dst[i] = src[i];
}

__device__ void load_split(Split &sp, const Split *g) {
    const uint32_t *src = (const uint32_t *)g;
    uint32_t *dst = (uint32_t *)&sp;
    for (uint32_t i = threadIdx.x; i < sizeof(Split) / 4; i += NT) dst[i] = src[i];
    __syncthreads();
}

template <int K, bool Z>
__global__ __launch_bounds__(NT) void k_lvl_classify(Params P, uint32_t l) {
    __shared__ Split sp;
    __shared__ uint32_t hist[NBPAD];
    if (P.ctl->error || blockIdx.x >= lvl_count(P, l, 1)) return;
    const uint32_t seg = P.tile2seg[l][blockIdx.x];
    if (seg >= lvl_count(P, l, 0)) {
        if (threadIdx.x == 0) atomicOr(&P.ctl->error, ERR_LEVEL);
        return;
    }
    const LvlSeg g = P.lseg[l][seg];
    if (g.begin > P.S.n || g.size > P.S.n - g.begin) {
        if (threadIdx.x == 0) atomicOr(&P.ctl->error, ERR_LEVEL);
        return;
    }
    const auto kc = KeyOf<Z>::make(P);
    load_split(sp, &P.lsplit[l][seg]);
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    for (int b = tid; b < NBPAD; b += NT) hist[b] = 0;
    __syncthreads();
    const uint32_t nb = uni(sp.nb);
    const int nbits = (int)uni(sp.nbits);
    const uint32_t lt = blockIdx.x - g.tile0;
    // one tile = ROOT_CHUNKS chunks of NT*K strings, classified chunk by chunk
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
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const uint32_t e = c0 + (uint32_t)(w * 64 * K + j * 64 + lane);
            k[j] = e < g.size ? kc.key(P.S, r[j].st, r[j].ln, g.depth) : 0;
        }
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const uint32_t e = c0 + (uint32_t)(w * 64 * K + j * 64 + lane);
            const bool valid = e < g.size;
            const uint32_t m = valid ? classify_any(k[j], sp) : nb;
            const uint64_t mask = match_any(m, nbits);
            if (valid && lane == 63 - (int)__clzll(mask)) atomicAdd(&hist[m], (uint32_t)__popcll(mask));
            if (valid) P.bkt[g.begin + e] = (uint16_t)m;
        }
    }
    __syncthreads();
    for (uint32_t b = tid; b < nb; b += NT) P.hist[(size_t)blockIdx.x * NBPAD + b] = hist[b];
}

// Exclusive scan over a segment's tiles, per bucket, of the tile histograms
// (stored tile-major: one contiguous row of counters per tile), giving every
// (tile, bucket) pair its offset inside the bucket, and the bucket totals.  A
// workgroup owns B buckets of one segment; thread t handles bucket B g + t%B
// over the tile range t/B, so B neighbouring threads read B adjacent counters
// of a row.  B = 16 when a level has many segments (16 counters fill a
// 64-byte line); B = 2 for the one segment of a plain sort's first level, so
// that 256 workgroups share its tiles instead of 32 (4096 tiles at 2^24
// strings: 32 per thread instead of 256).
constexpr int CS_B = 16;
// nbw > 0: every segment has nbw columns (the digits of a wide level's
// distribution passes), else its splitters' bucket count.
template <int B>
__global__ __launch_bounds__(NT) void k_lvl_colscan(Params P, uint32_t l, uint32_t nbw) {
    constexpr int R = NT / B, G = NBPAD / B;
    __shared__ uint32_t part[R][B];
    const uint32_t seg = blockIdx.x / G, grp = blockIdx.x % G;
    if (P.ctl->error || seg >= lvl_count(P, l, 0)) return;
    const LvlSeg g = P.lseg[l][seg];
    const uint32_t nb = nbw ? nbw : uni(P.lsplit[l][seg].nb);
    if (grp * B >= nb) return;
    const uint32_t b = grp * B + (threadIdx.x % B);
    const uint32_t r = threadIdx.x / B;
    const uint32_t T = g.ntile;
    const uint32_t per = (T + R - 1) / R;
    const uint32_t lo = g.tile0 + min(T, r * per), hi = g.tile0 + min(T, r * per + per);
    uint32_t s = 0;
    if (b < nb) {
#pragma unroll 8
        for (uint32_t i = lo; i < hi; ++i) s += P.hist[(size_t)i * NBPAD + b];
    }
    part[r][threadIdx.x % B] = s;
    __syncthreads();
    if (threadIdx.x < B) {
        uint32_t run = 0;
        for (int k = 0; k < R; ++k) {
            const uint32_t x = part[k][threadIdx.x];
            part[k][threadIdx.x] = run;
            run += x;
        }
        const uint32_t bb = grp * B + threadIdx.x;
        if (bb < nb) P.ltot[l][(size_t)seg * NBPAD + bb] = run;
    }
    __syncthreads();
    if (b < nb) {
        uint32_t run = part[r][threadIdx.x % B];
        for (uint32_t i = lo; i < hi; ++i) {
            uint32_t *c = &P.hist[(size_t)i * NBPAD + b];
            const uint32_t x = *c;
            *c = run;
            run += x;
        }
    }
}

// Column scan of level l: one workgroup per B buckets of every segment the
// level can hold, or, for the single first-level segment of a plain sort,
// 256 workgroups of 2 buckets.
inline void launch_colscan(const Params &P, uint32_t maxseg, uint32_t l, uint32_t nbw, hipStream_t s) {
    if (l == 0 && !P.set_begin)
        hipLaunchKernelGGL(k_lvl_colscan<2>, dim3(NBPAD / 2), dim3(NT), 0, s, P, l, nbw);
    else
        hipLaunchKernelGGL(k_lvl_colscan<CS_B>, dim3(maxseg * (NBPAD / CS_B)), dim3(NT), 0, s, P, l, nbw);
}

template <int K>
struct LvlScatterLDS {
    Split sp;
    uint32_t run[NBPAD];
    uint32_t tmp[NW];
    ScatterLDS<K> sc;
};

template <int K>
__global__ __launch_bounds__(NT) void k_lvl_scatter(Params P, uint32_t l) {
    __shared__ LvlScatterLDS<K> L;
    if (P.ctl->error || blockIdx.x >= lvl_count(P, l, 1)) return;
    const uint32_t seg = P.tile2seg[l][blockIdx.x];
    if (seg >= lvl_count(P, l, 0)) {
        if (threadIdx.x == 0) atomicOr(&P.ctl->error, ERR_LEVEL);
        return;
    }
    const LvlSeg g = P.lseg[l][seg];
    if (g.begin > P.S.n || g.size > P.S.n - g.begin) {
        if (threadIdx.x == 0) atomicOr(&P.ctl->error, ERR_LEVEL);
        return;
    }
    load_split(L.sp, &P.lsplit[l][seg]);
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const uint32_t nb = uni(L.sp.nb);
    const uint32_t *tot = &P.ltot[l][(size_t)seg * NBPAD];
    for (uint32_t b = tid; b < NBPAD; b += NT) L.run[b] = b < nb ? tot[b] : 0u;
    __syncthreads();
    block_scan(L.run, (int)nb, L.tmp, true, AddOp(), 0u);
    for (uint32_t b = tid; b < nb; b += NT) L.run[b] += g.begin + P.hist[(size_t)blockIdx.x * NBPAD + b];
    __syncthreads();
    Rec *out = out_is_r1(g.meta) ? P.R1 : P.R0;
    const uint32_t lt = blockIdx.x - g.tile0;
    for (uint32_t ch = 0; ch < ROOT_CHUNKS; ++ch) {
        const uint32_t c0 = (lt * ROOT_CHUNKS + ch) * (uint32_t)(NT * K);
        if (c0 >= g.size) break;
        Rec r[K];
        uint32_t m[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const uint32_t e = c0 + (uint32_t)(w * 64 * K + j * 64 + lane);
            if (e < g.size) {
                r[j] = seg_rec(P, g.meta, g.begin + e);
                m[j] = P.bkt[g.begin + e];
            } else {
                m[j] = nb;
            }
        }
        scatter_chunk<K>(L.sc, L.tmp, nb, (int)uni(L.sp.nbits), m, r, nullptr, min((uint32_t)(NT * K), g.size - c0),
                         L.run, out, nullptr, P.S.n, &P.ctl->error);
    }
}

template <int NBC>
struct SchedLDS {
    uint32_t bst[NBC];        // bucket starts (segment-relative)
    uint32_t cnt[NBC];
    uint8_t kind[NBC];        // 0 empty or next-level segment, 1 worker task, 2 small (base case), 3 identical
    uint32_t rk[NBC + 1];     // worker task rank; later the small list's size prefix
    uint16_t lsmall[NBC];
    uint16_t cfirst[NBC + 1];
    uint32_t nchunk;
    unsigned long long pos, db;
    uint32_t tmp[NW];
};

// Children of buckets b0 .. b0 + nb - 1 of a level's segment, once their
// sizes and starts are in L.cnt / L.bst (indexed from b0): the next level's
// segments, worker tasks for the other large buckets, identical strings
// finished here, and the small buckets as base-case chunk tasks (group
// descriptors, chunks of at most C - threshold strings, never splitting a
// group).  SP (Split or WSplit, in LDS or device memory) gives the
// end-of-string flags and splitter LCPs.
template <int NBC, typename SP>
__device__ void schedule_buckets(const Params &P, uint32_t l, const LvlSeg &g, uint32_t b0, uint32_t nb, const SP &sp,
                                 SchedLDS<NBC> &L) {
    const int tid = threadIdx.x;
    const uint32_t h = g.depth;
    const uint32_t cpar = out_is_r1(g.meta) ? M_PARITY : 0u;
    const Rec *out = out_is_r1(g.meta) ? P.R1 : P.R0;
    for (uint32_t b = tid; b < nb; b += NT) {
        const uint32_t c = L.cnt[b];
        uint32_t kind = 0;
        if (c) {
            const uint32_t gb = b0 + b;
            const bool ident = (gb & 1) && sp.zr[gb >> 1];
            if (ident) kind = 3;
            else if (!(c > LVL_MIN && l + 1 < LMAX)) kind = c > P.tbase ? 1u : 2u;
        }
        L.kind[b] = (uint8_t)kind;
        L.rk[b] = kind == 1 ? 1u : 0u;
    }
    __syncthreads();
    const uint32_t ntask = uni(block_scan(L.rk, (int)nb, L.tmp, true, AddOp(), 0u));
    // seams and next-level segments
    for (uint32_t b = tid; b < nb; b += NT) {
        const uint32_t c = L.cnt[b], st = L.bst[b];
        if (!c) continue;
        if (P.lcp && st > 0) P.lcp[g.begin + st] = SEAM | h;
        if (L.kind[b] == 0)
            lvl_append(P, l + 1, LvlSeg{g.begin + st, c, child_depth(sp, h, b0 + b), cpar, 0, 0, g.setbase, 0});
    }
    // identical strings (an equality bucket whose splitter ends the string):
    // already in input order, lcp = length
    for (uint32_t b = (b0 & 1) ? 0u : 1u; b < nb; b += 2) {
        if (uni(L.kind[b]) != 3) continue;
        const uint32_t c = L.cnt[b], st = g.begin + L.bst[b];
        for (uint32_t i = tid; i < c; i += NT) {
            const Rec r = out[st + i];
            P.perm[st + i] = r.id - g.setbase;
            if (P.lcp && i > 0) P.lcp[st + i] = r.ln;
        }
    }
    // worker tasks
    if (tid == 0 && ntask) {
        add_agent(&P.ctl->pending, (unsigned long long)ntask);
        L.pos = add_agent(&P.ctl->tail, (unsigned long long)ntask);
    }
    __syncthreads();
    if (ntask) {
        const unsigned long long pos = uni64(L.pos);
        for (uint32_t b = tid; b < nb; b += NT)
            if (L.kind[b] == 1)
                seed_task(P, pos + L.rk[b],
                          Task{g.begin + L.bst[b], L.cnt[b], child_depth(sp, h, b0 + b), cpar, g.setbase});
    }
    __syncthreads();
    // small list and chunks
    uint32_t *psz = L.rk;
    for (uint32_t b = tid; b < nb; b += NT) psz[b] = L.kind[b] == 2 ? 1u : 0u;
    __syncthreads();
    const uint32_t nsmall = uni(block_scan(psz, (int)nb, L.tmp, true, AddOp(), 0u));
    for (uint32_t b = tid; b < nb; b += NT)
        if (L.kind[b] == 2) L.lsmall[psz[b]] = (uint16_t)b;
    __syncthreads();
    for (uint32_t k = tid; k < nsmall; k += NT) psz[k] = L.cnt[L.lsmall[k]];
    __syncthreads();
    const uint32_t small_total = block_scan(psz, (int)nsmall, L.tmp, true, AddOp(), 0u);
    if (tid == 0) {
        psz[nsmall] = small_total;
        L.nchunk = 0;
    }
    __syncthreads();
    const uint32_t cap = (P.tbase * 2 <= P.chunk) ? P.chunk - P.tbase : 0u;
    for (uint32_t k = tid; k < nsmall; k += NT) {
        const uint32_t ck = cap ? psz[k] / cap : k;
        const uint32_t cp = k ? (cap ? psz[k - 1] / cap : k - 1) : 0xFFFFFFFFu;
        if (ck != cp) L.cfirst[ck] = (uint16_t)k;
        if (k == nsmall - 1) L.nchunk = ck + 1;
    }
    __syncthreads();
    const uint32_t nchunk = uni(L.nchunk);
    if (tid == 0) {
        L.cfirst[nchunk] = (uint16_t)nsmall;
        if (nchunk) {
            add_agent(&P.ctl->pending, (unsigned long long)nchunk);
            L.pos = add_agent(&P.ctl->tail, (unsigned long long)nchunk);
        }
        L.db = nsmall ? add_agent(&P.ctl->desc_top, (unsigned long long)nsmall) : 0ull;
        if (L.db + nsmall > P.desc_cap) atomicOr(&P.ctl->error, ERR_DESC_CAP);
    }
    __syncthreads();
    const unsigned long long pos = uni64(L.pos), db = uni64(L.db);
    if (db + nsmall > P.desc_cap) return;
    for (uint32_t k = tid; k < nsmall; k += NT) {
        const uint32_t b = L.lsmall[k];
        P.desc[db + k] = GroupDesc{g.begin + L.bst[b], L.cnt[b], child_depth(sp, h, b0 + b), 0u};
    }
    for (uint32_t c = tid; c < nchunk; c += NT) {
        const uint32_t k0 = L.cfirst[c], k1 = L.cfirst[c + 1];
        seed_task(P, pos + c, Task{(uint32_t)(db + k0), k1 - k0, psz[k1] - psz[k0], M_CHUNK | cpar, g.setbase});
    }
}

struct LvlSchedLDS {
    Split sp;
    SchedLDS<NBPAD> s;
};

// A level's segment: bucket sizes from the column scan's totals, starts by a
// prefix sum over them.
__global__ __launch_bounds__(NT) void k_lvl_schedule(Params P, uint32_t l) {
    __shared__ LvlSchedLDS L;
    if (P.ctl->error || blockIdx.x >= lvl_count(P, l, 0)) return;
    const int tid = threadIdx.x;
    const LvlSeg g = P.lseg[l][blockIdx.x];
    load_split(L.sp, &P.lsplit[l][blockIdx.x]);
    const uint32_t nb = uni(L.sp.nb);
    const uint32_t *tot = &P.ltot[l][(size_t)blockIdx.x * NBPAD];
    for (uint32_t b = tid; b < NBPAD; b += NT) {
        const uint32_t c = b < nb ? tot[b] : 0u;
        L.s.cnt[b] = c;
        L.s.bst[b] = c;
    }
    __syncthreads();
    block_scan(L.s.bst, (int)nb, L.s.tmp, true, AddOp(), 0u);
    schedule_buckets<NBPAD>(P, l, g, 0u, nb, L.sp, L.s);
}

// ---------------------------------------------------------------------------
// Boundary LCPs: a position still holding SEAM|h was the first string of a
// bucket created by a step at depth h; its predecessor lies in an earlier
// bucket of that step, so their keys at depth h differ and the LCP is h plus
// the equal leading bytes of the two keys.
//
// After a device error the workers stop early and leave permutation entries
// unwritten (the outputs are undefined then), so the pass does not run: an
// unwritten entry is not a string index.  An index outside a set is a device
// error too, never an access.
// Each workgroup takes SEAM_RANGE consecutive positions, SU per thread, each
// stage's loads issued for all of them before the next stage needs the
// results (the lcp word, the two permutation entries, the two records, the
// two keys), so the dependent round trips overlap across positions.  In a
// batched sort the permutation is set-local: the boundaries of the sets that
// overlap the range are staged in LDS once (one search in device memory per
// workgroup), and each seam finds its set there.
constexpr int SU = 4;
constexpr uint32_t SEAM_RANGE = NT * SU;
template <bool Z>
__global__ __launch_bounds__(NT) void k_seam(Params P) {
    __shared__ uint32_t sb[SEAM_RANGE + 2];
    __shared__ uint32_t sfirst;
    if (P.ctl->error) return;
    const uint32_t n = P.S.n;
    const uint32_t r0 = blockIdx.x * SEAM_RANGE;
    if (r0 >= n) return;
    const auto kc = KeyOf<Z>::make(P);
    if (P.set_begin) {
        if (threadIdx.x == 0) {
            uint32_t lo = 0, hi = P.m;   // last set starting at or before r0
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (P.set_begin[mid] <= r0) lo = mid; else hi = mid;
            }
            sfirst = lo;
        }
        __syncthreads();
        // the boundaries from that set on; past the last set, above every position
        for (uint32_t i = threadIdx.x; i < SEAM_RANGE + 2; i += NT) {
            const uint32_t j = sfirst + i;
            sb[i] = j < P.m ? P.set_begin[j] : 0xFFFFFFFFu;
        }
        __syncthreads();
    }
    uint32_t v[SU], ia[SU], ib[SU];
    bool on[SU];
#pragma unroll
    for (int u = 0; u < SU; ++u) {
        const uint32_t p = r0 + threadIdx.x + u * NT;
        v[u] = (p >= 1 && p < n) ? P.lcp[p] : 0u;
        on[u] = (v[u] & SEAM) != 0;
    }
#pragma unroll
    for (int u = 0; u < SU; ++u) {
        ia[u] = 0;
        ib[u] = 0;
        if (!on[u]) continue;
        const uint32_t p = r0 + threadIdx.x + u * NT;
        uint32_t base = 0;
        if (P.set_begin) {
            uint32_t lo = 0, hi = SEAM_RANGE + 2;   // last boundary at or before p (sb[0] <= r0 <= p)
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (sb[mid] <= p) lo = mid; else hi = mid;
            }
            base = sb[lo];
        }
        ia[u] = P.perm[p - 1] + base;
        ib[u] = P.perm[p] + base;
        if (ia[u] >= n || ib[u] >= n) {
            atomicOr(&P.ctl->error, ERR_SEAM);
            on[u] = false;
        }
    }
    Rec ra[SU], rb[SU];
#pragma unroll
    for (int u = 0; u < SU; ++u) {
        if (!on[u]) continue;
        ra[u] = make_rec(P.S, ia[u]);
        rb[u] = make_rec(P.S, ib[u]);
    }
#pragma unroll
    for (int u = 0; u < SU; ++u) {
        if (!on[u]) continue;
        const uint32_t h = v[u] & ~SEAM;
        const uint64_t z = kc.key(P.S, ra[u].st, ra[u].ln, h) ^ kc.key(P.S, rb[u].st, rb[u].ln, h);
        P.lcp[r0 + threadIdx.x + u * NT] = h + (z ? kc.eqc(z) : kc.q());
    }
}

// Debug dump of one root step.
__global__ void k_debug_dump(Params P, uint32_t depth, uint64_t *keys, uint64_t *split, uint64_t *tree,
                             uint32_t *info, uint16_t *bucket, uint32_t *hist, uint32_t *perm) {
    const Split *sp = &P.lsplit[0][0];
    const uint32_t n = P.S.n;
    for (uint32_t i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT) {
        const Rec r = make_rec(P.S, i);
        keys[i] = key_at(P.S.chars, P.S.nchars, r.st, r.ln, depth);
        bucket[i] = P.bkt[i];
        perm[i] = P.R1[i].id;
    }
    if (blockIdx.x == 0) {
        for (uint32_t j = threadIdx.x; j < 256; j += NT) {
            split[j] = j < sp->v ? splitter(*sp, j) : 0;
            tree[j] = (j < sp->v) ? sp->tree[j + 1] : 0;
        }
        for (uint32_t b = threadIdx.x; b < NBPAD; b += NT) hist[b] = b < sp->nb ? P.ltot[0][b] : 0;
        if (threadIdx.x == 0) {
            info[0] = sp->v;
            info[1] = sp->d;
            info[2] = sp->ndistinct;
            info[3] = 0;
        }
    }
}

// Debug: one segment step of the persistent worker (sample, any common-prefix
// extension, classification, count, prefix sum, redistribution, children) on
// the whole input as one segment at `depth`, by one workgroup, then its
// splitters, splitter LCPs, end flags, classification depth and every
// bucket's start, size and child depth.  The children it queues are never
// run; its small buckets are not sorted.
template <int K, int C, bool Z>
__global__ __launch_bounds__(NT) void k_debug_segstep(Params P, uint32_t depth, uint64_t *split, uint32_t *info,
                                                      uint32_t *hl, uint32_t *zr, uint32_t *bst, uint32_t *bsz,
                                                      uint32_t *bdep) {
    __shared__ StepLDS<K, C> L;
    if (threadIdx.x < NPH) L.ph[threadIdx.x] = 0;
    if (threadIdx.x < NST) L.st[threadIdx.x] = 0;
    if (threadIdx.x == 0) L.ph_last = wall_clock64();
    __syncthreads();
    Task t{0, P.S.n, depth, M_IDENT_SRC, 0};
    seg_step<K, C>(P, t, L, KeyOf<Z>::make(P), false);
    __syncthreads();
    const uint32_t v = L.sp.v, nb = L.sp.nb, h = L.hstep;
    for (uint32_t j = threadIdx.x; j < (uint32_t)(VMAX + 1); j += NT) {
        split[j] = j < v ? splitter(L.sp, j) : 0;
        hl[j] = j <= v ? L.sp.hl[j] : 0;
        zr[j] = j < v ? L.sp.zr[j] : 0;
    }
    for (uint32_t b = threadIdx.x; b < (uint32_t)NBPAD; b += NT) {
        bst[b] = b < nb ? L.bst[b] : 0;
        bsz[b] = b < nb ? L.hist[b] : 0;
        bdep[b] = b < nb ? child_depth(L.sp, h, b) : 0;
    }
    if (threadIdx.x == 0) {
        info[0] = v;
        info[1] = L.sp.d;
        info[2] = L.sp.ndistinct;
        info[3] = h;
    }
}

// Debug: the permutation after a segment step (its records are in R1).
__global__ void k_debug_perm(Params P, uint32_t *perm) {
    for (uint32_t i = blockIdx.x * NT + threadIdx.x; i < P.S.n; i += gridDim.x * NT) perm[i] = P.R1[i].id;
}

// Packing of a server batch: job k's strings are rows set_begin[k] ..
// set_begin[k+1] of the flat space; its characters start at char_base and its
// raw offsets (CSR n+1, or n starts for suffixes of its text) at raw_base.
struct PackJob {
    unsigned long long char_base, raw_base, off0, nchars;
    uint32_t n, flags;
};

__global__ void k_pack(const PackJob *jobs, const uint32_t *set_begin, uint32_t m, const unsigned long long *raw,
                       unsigned long long *starts, uint32_t *lengths, uint32_t n) {
    for (uint32_t i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT) {
        uint32_t lo = 0, hi = m;                 // last job with set_begin <= i
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (set_begin[mid] <= i) lo = mid; else hi = mid;
        }
        const PackJob J = jobs[lo];
        const uint32_t j = i - set_begin[lo];
        const unsigned long long o = raw[J.raw_base + j];
        starts[i] = J.char_base + (o - J.off0);
        lengths[i] = (J.flags & TO_END) ? (uint32_t)(J.nchars - o) : (uint32_t)(raw[J.raw_base + j + 1] - o);
    }
}

// explicit instantiations used by the host code
template __global__ void k_worker<4, 512, false>(Params);
template __global__ void k_worker<4, 1024, false>(Params);
template __global__ void k_worker<8, 512, false>(Params);
template __global__ void k_worker<8, 1024, false>(Params);
template __global__ void k_worker<4, 512, true>(Params);
template __global__ void k_worker<4, 1024, true>(Params);
template __global__ void k_worker<8, 512, true>(Params);
template __global__ void k_worker<8, 1024, true>(Params);
template __global__ void k_debug_segstep<4, 512, false>(Params, uint32_t, uint64_t *, uint32_t *, uint32_t *,
                                                        uint32_t *, uint32_t *, uint32_t *, uint32_t *);
template __global__ void k_debug_segstep<4, 1024, false>(Params, uint32_t, uint64_t *, uint32_t *, uint32_t *,
                                                         uint32_t *, uint32_t *, uint32_t *, uint32_t *);
template __global__ void k_debug_segstep<8, 512, false>(Params, uint32_t, uint64_t *, uint32_t *, uint32_t *,
                                                        uint32_t *, uint32_t *, uint32_t *, uint32_t *);
template __global__ void k_debug_segstep<8, 1024, false>(Params, uint32_t, uint64_t *, uint32_t *, uint32_t *,
                                                         uint32_t *, uint32_t *, uint32_t *, uint32_t *);
template __global__ void k_lvl_sample<false>(Params, uint32_t);
template __global__ void k_lvl_sample<true>(Params, uint32_t);
template __global__ void k_lvl_classify<4, false>(Params, uint32_t);
template __global__ void k_lvl_classify<8, false>(Params, uint32_t);
template __global__ void k_lvl_classify<4, true>(Params, uint32_t);
template __global__ void k_lvl_classify<8, true>(Params, uint32_t);
template __global__ void k_seam<false>(Params);
template __global__ void k_seam<true>(Params);
template __global__ void k_lvl_scatter<4>(Params, uint32_t);
template __global__ void k_lvl_scatter<8>(Params, uint32_t);

}  // namespace ssd
