// Host side of libssort.so: the C ABI declared in include/ssort.h.
// One translation unit with the kernels so that every template instance the
// host launches is compiled here.
#include <hip/hip_runtime.h>
#include <stdlib.h>
#include <string.h>
#include <algorithm>
#include <mutex>

#include "ssort.h"
#include "ssort_kernels.hip"
#include "ssort_wide.hip"
#include "ssort_merge.hip"
#include "ssort_serve.hip"

using namespace ssd;

struct ssort_ctx {
    int device;
    ssort_tuning tun;
    int cus;
    int worker_blocks;
    unsigned long long wall_khz;
    uint32_t wait_ms;
    void *last_ws;
    void *scratch;     // this device's copy of `scratch` (ssort_sort_noalloc), or null
    int prof;
    hipEvent_t ev[4];
};

// Workspace of ssort_sort_noalloc, for callers that cannot allocate: a
// file-scope device array, one copy per GPU the library is loaded on, held
// until the process ends.  Host code never passes `scratch` itself to a
// kernel (on the host the name is a stand-in, not a device address): each
// context looks up its device's address once, in ssort_create, and passes
// that.
static __device__ __align__(256) unsigned char scratch[SSORT_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_ptr[MAX_DEVICES];   // device address of `scratch` per device, once looked up

// The device address of this device's `scratch` (the device is current).
void *scratch_of(int device) {
    if (device < 0 || device >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> g(scratch_mu);
    if (!scratch_ptr[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        scratch_ptr[device] = p;
    }
    return scratch_ptr[device];
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

uint64_t next_pow2(uint64_t x) {
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

uint32_t grid_for(uint64_t work) {
    uint64_t g = (work + NT - 1) / NT;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    return (uint32_t)g;
}

struct Layout {
    size_t ctl, r0, r1, bkt, ring, lseg[LMAX], t2s[LMAX], lsplit[LMAX], ltot[LMAX], hist, desc, alpha, total;
    size_t wsplit, wst, wen, btmp;   // wide level 0 only (0 otherwise)
    uint64_t cap;
    uint32_t maxseg, maxtiles, tile;
};

// Splitters of the wide level 0 (0: every level narrow); the worker's steps
// use at most VMAX.
uint32_t wide_v(const ssort_tuning &t) { return t.v > (uint32_t)VMAX ? t.v : 0u; }
uint32_t narrow_v(const ssort_tuning &t) { return t.v > (uint32_t)VMAX ? (uint32_t)VMAX : t.v; }

// Bits of the wide level's second distribution digit: bucket numbers are
// below 2(v+1) = 2^(WLO + hbits).
uint32_t wide_hbits(uint32_t wv) {
    uint32_t b = 0;
    while ((1u << b) < 2 * (wv + 1)) ++b;
    return b - WLO;
}

Layout layout(const ssort_ctx *c, uint32_t n, uint32_t m) {
    Layout L;
    const uint32_t K = c->tun.keys_per_thread;
    L.tile = (uint32_t)NT * K * ROOT_CHUNKS;
    // a level holds segments of more than LVL_MIN strings (level 0: the input
    // or sets of more than ROOT_MIN), and their tiles
    L.maxseg = n / std::min(LVL_MIN, ROOT_MIN) + 1;
    L.maxtiles = n / L.tile + L.maxseg;
    // queued tasks: segments of more than base_threshold strings (at most
    // two per such disjoint set of strings), the batched sets, base-case
    // chunks (of at least (chunk - threshold) / 2 >= 128 strings when formed
    // in a worker step; at most one per bucket when formed by a level); twice
    // that bound leaves every slot's previous occupant consumed long before
    // the slot is reused
    const uint32_t wv = wide_v(c->tun);
    const uint64_t nb0 = wv ? 2 * (uint64_t)wv + 1 : (uint64_t)NBMAX;   // buckets of a level-0 segment
    // (level-0 segments: at most one per set; their chunks of small buckets
    // never span more than one scheduling workgroup's buckets)
    const uint64_t seg0 = std::min<uint64_t>(m, L.maxseg);
    const uint64_t live = 2 * (uint64_t)n / (c->tun.base_threshold + 1) + (uint64_t)n / 128 + m +
                          (nb0 + 16) * seg0 + (uint64_t)NBMAX * (L.maxseg + 1) + (uint64_t)c->worker_blocks;
    L.cap = next_pow2(2 * live + 1024);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes, 256);
        return at;
    };
    L.ctl = take(sizeof(Ctl));
    L.r0 = take(sizeof(Rec) * (size_t)n);
    L.r1 = take(sizeof(Rec) * (size_t)n);
    L.bkt = take(2 * (size_t)n);
    L.ring = take(sizeof(Slot) * (size_t)L.cap);
    for (int l = 0; l < LMAX; ++l) {
        L.lseg[l] = take(sizeof(LvlSeg) * (size_t)L.maxseg);
        L.t2s[l] = take(4 * (size_t)L.maxtiles);
        L.lsplit[l] = take(sizeof(Split) * (size_t)L.maxseg);
        L.ltot[l] = take(4 * (size_t)NBPAD * L.maxseg);
    }
    L.hist = take(4 * (size_t)NBPAD * L.maxtiles);
    L.desc = take(sizeof(GroupDesc) * (size_t)n);   // at most one descriptor per base-case group
    L.alpha = take(sizeof(Alphabet));
    L.wsplit = L.wst = L.wen = L.btmp = 0;
    if (wv) {
        L.wsplit = take(sizeof(WSplit) * (size_t)L.maxseg);
        L.wst = take(4 * (size_t)WNBPAD * L.maxseg);
        L.wen = take(4 * (size_t)WNBPAD * L.maxseg);
        L.btmp = take(2 * (size_t)n);
    }
    L.total = off;
    return L;
}

bool valid_tuning(const ssort_tuning &t) {
    const uint32_t v = t.v;
    if (v < 1 || ((v + 1) & v) != 0) return false;
    if (v > VMAX && v != 1023 && v != 2047 && v != (uint32_t)WVMAX) return false;
    if (t.keys_per_thread != 4 && t.keys_per_thread != 8) return false;
    if (t.base_threshold < 16 || t.base_threshold > (uint32_t)CH) return false;
    if (t.flags & ~(SSORT_VALIDATE | SSORT_EQUAL | SSORT_ALPHABET)) return false;
    return true;
}

int chunk_for(uint32_t tbase) { return tbase <= 256 ? 512 : 1024; }

template <int K, int C, bool Z>
hipError_t worker_occupancy(int *nb) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, (const void *)k_worker<K, C, Z>, NT, 0);
}

template <bool Z>
hipError_t occupancy_z(const ssort_tuning &t, int *nb) {
    const int C = chunk_for(t.base_threshold);
    if (t.keys_per_thread == 4) return C == 512 ? worker_occupancy<4, 512, Z>(nb) : worker_occupancy<4, 1024, Z>(nb);
    return C == 512 ? worker_occupancy<8, 512, Z>(nb) : worker_occupancy<8, 1024, Z>(nb);
}

hipError_t occupancy(const ssort_tuning &t, int *nb) {
    return (t.flags & SSORT_ALPHABET) ? occupancy_z<true>(t, nb) : occupancy_z<false>(t, nb);
}

bool packed(const ssort_ctx *c) { return (c->tun.flags & SSORT_ALPHABET) != 0; }

// Persistent workers: as many as fit on the GPU, but no more than the work
// can use (about one per 512 strings, at least one per root task).
uint32_t worker_grid(const ssort_ctx *c, uint64_t n, uint64_t roots) {
    uint64_t want = std::max<uint64_t>((n + 511) / 512, roots);
    want = std::max<uint64_t>(want, 1);
    return (uint32_t)std::min<uint64_t>(want, (uint64_t)c->worker_blocks);
}

template <bool Z>
void launch_worker_z(const ssort_ctx *c, const Params &P, uint32_t grid, hipStream_t s) {
    const int C = chunk_for(c->tun.base_threshold);
    const dim3 g(grid), b(NT);
    if (c->tun.keys_per_thread == 4) {
        if (C == 512) hipLaunchKernelGGL((k_worker<4, 512, Z>), g, b, 0, s, P);
        else hipLaunchKernelGGL((k_worker<4, 1024, Z>), g, b, 0, s, P);
    } else {
        if (C == 512) hipLaunchKernelGGL((k_worker<8, 512, Z>), g, b, 0, s, P);
        else hipLaunchKernelGGL((k_worker<8, 1024, Z>), g, b, 0, s, P);
    }
}

void launch_worker(const ssort_ctx *c, const Params &P, uint32_t grid, hipStream_t s) {
    if (packed(c)) launch_worker_z<true>(c, P, grid, s);
    else launch_worker_z<false>(c, P, grid, s);
}

// Alphabet compression: the input's byte values and their codes, before
// anything reads a key.
void launch_alphabet(const ssort_ctx *c, const Params &P, hipStream_t s) {
    if (!packed(c)) return;
    hipLaunchKernelGGL(k_alpha_scan, dim3(grid_for(P.S.nchars / 8 + 1)), dim3(NT), 0, s, P);
    hipLaunchKernelGGL(k_alpha_codes, dim3(1), dim3(NT), 0, s, P);
}

void launch_seam(const ssort_ctx *c, const Params &P, hipStream_t s) {
    const dim3 g((uint32_t)(((uint64_t)P.S.n + SEAM_RANGE - 1) / SEAM_RANGE));
    if (packed(c)) hipLaunchKernelGGL((k_seam<true>), g, dim3(NT), 0, s, P);
    else hipLaunchKernelGGL((k_seam<false>), g, dim3(NT), 0, s, P);
}

// The whole-GPU levels (grids sized for each level's capacity; workgroups
// beyond the level's actual count exit at once).  With schedule = false only
// level 0 runs, without turning its buckets into tasks (the debug step).
// Wide level 0 (v > 255): sample and tree with its jump table, classify,
// two stable distribution passes by the digits of the bucket number, bucket
// bounds, children.
void launch_wide_level(const ssort_ctx *c, const Params &P, const Layout &L, bool schedule, hipStream_t s) {
    const int K = c->tun.keys_per_thread;
    const bool z = packed(c) && P.alpha;
    const uint32_t hb = wide_hbits(P.wv);
    const size_t lds = 8 * ((size_t)P.wv + 1) + 2 * ((size_t)1 << JA) + 4 * ((size_t)1 << WLO);
    const dim3 tiles(L.maxtiles), b(NT);
    if (z) hipLaunchKernelGGL((k_wsample<true>), dim3(L.maxseg), b, 0, s, P);
    else hipLaunchKernelGGL((k_wsample<false>), dim3(L.maxseg), b, 0, s, P);
    if (K == 4 && z) hipLaunchKernelGGL((k_wclassify<4, true>), tiles, b, lds, s, P);
    else if (K == 4) hipLaunchKernelGGL((k_wclassify<4, false>), tiles, b, lds, s, P);
    else if (z) hipLaunchKernelGGL((k_wclassify<8, true>), tiles, b, lds, s, P);
    else hipLaunchKernelGGL((k_wclassify<8, false>), tiles, b, lds, s, P);
    launch_colscan(P, L.maxseg, 0u, 1u << WLO, s);
    if (K == 4) hipLaunchKernelGGL((k_wscatter<4, 1>), tiles, b, 0, s, P, hb);
    else hipLaunchKernelGGL((k_wscatter<8, 1>), tiles, b, 0, s, P, hb);
    hipLaunchKernelGGL(k_whist2, tiles, b, 0, s, P, hb);
    launch_colscan(P, L.maxseg, 0u, 1u << hb, s);
    if (K == 4) hipLaunchKernelGGL((k_wscatter<4, 2>), tiles, b, 0, s, P, hb);
    else hipLaunchKernelGGL((k_wscatter<8, 2>), tiles, b, 0, s, P, hb);
    hipLaunchKernelGGL(k_wbounds, tiles, b, 0, s, P);
    if (schedule) hipLaunchKernelGGL(k_wschedule, dim3(L.maxseg * WSCHED_G), b, 0, s, P);
}

void launch_levels(const ssort_ctx *c, const Params &P, const Layout &L, bool schedule, hipStream_t s) {
    const int K = c->tun.keys_per_thread;
    const bool z = packed(c) && P.alpha;
    for (uint32_t l = 0; l < (schedule ? (uint32_t)LMAX : 1u); ++l) {
        if (l == 0 && P.wv) {
            launch_wide_level(c, P, L, schedule, s);
            continue;
        }
        if (z) hipLaunchKernelGGL((k_lvl_sample<true>), dim3(L.maxseg), dim3(NT), 0, s, P, l);
        else hipLaunchKernelGGL((k_lvl_sample<false>), dim3(L.maxseg), dim3(NT), 0, s, P, l);
        if (K == 4 && z) hipLaunchKernelGGL((k_lvl_classify<4, true>), dim3(L.maxtiles), dim3(NT), 0, s, P, l);
        else if (K == 4) hipLaunchKernelGGL((k_lvl_classify<4, false>), dim3(L.maxtiles), dim3(NT), 0, s, P, l);
        else if (z) hipLaunchKernelGGL((k_lvl_classify<8, true>), dim3(L.maxtiles), dim3(NT), 0, s, P, l);
        else hipLaunchKernelGGL((k_lvl_classify<8, false>), dim3(L.maxtiles), dim3(NT), 0, s, P, l);
        launch_colscan(P, L.maxseg, l, 0u, s);
        if (K == 4) hipLaunchKernelGGL((k_lvl_scatter<4>), dim3(L.maxtiles), dim3(NT), 0, s, P, l);
        else hipLaunchKernelGGL((k_lvl_scatter<8>), dim3(L.maxtiles), dim3(NT), 0, s, P, l);
        if (schedule) hipLaunchKernelGGL(k_lvl_schedule, dim3(L.maxseg), dim3(NT), 0, s, P, l);
    }
}

ssort_status check_strings(const ssort_strings *in) {
    if (!in) return SSORT_EINVAL;
    if (in->n == 0) return SSORT_OK;
    if (in->n > 0xFFFFFFFEu || !in->offsets) return SSORT_EINVAL;
    if (!in->chars && in->nchars) return SSORT_EINVAL;
    if ((in->flags & SSORT_TO_END) && in->nchars >= 0x80000000ull) return SSORT_EINVAL;
    if (in->flags & ~SSORT_TO_END) return SSORT_EINVAL;
    return SSORT_OK;
}

Params make_params(const ssort_ctx *c, const ssort_strings *in, uint32_t *perm, uint32_t *lcp, void *ws,
                   const Layout &L, uint32_t m, const uint32_t *set_begin) {
    Params P;
    memset(&P, 0, sizeof(P));
    P.S.chars = in->chars;
    P.S.nchars = in->nchars;
    P.S.off = in->offsets;
    P.S.len = in->lengths;
    P.S.n = in->n;
    P.S.flags = in->flags;
    char *w = (char *)ws;
    P.R0 = (Rec *)(w + L.r0);
    P.R1 = (Rec *)(w + L.r1);
    P.bkt = (uint16_t *)(w + L.bkt);
    P.perm = perm;
    P.lcp = lcp;
    P.ring = (Slot *)(w + L.ring);
    P.ring_mask = L.cap - 1;
    P.ctl = (Ctl *)(w + L.ctl);
    for (int l = 0; l < LMAX; ++l) {
        P.lseg[l] = (LvlSeg *)(w + L.lseg[l]);
        P.tile2seg[l] = (uint32_t *)(w + L.t2s[l]);
        P.lsplit[l] = (Split *)(w + L.lsplit[l]);
        P.ltot[l] = (uint32_t *)(w + L.ltot[l]);
    }
    P.hist = (uint32_t *)(w + L.hist);
    P.desc = (GroupDesc *)(w + L.desc);
    P.desc_cap = in->n;
    P.set_begin = set_begin;
    P.m = m;
    P.lmaxseg = L.maxseg;
    P.lmaxtiles = L.maxtiles;
    P.tile = L.tile;
    P.chunk = (uint32_t)chunk_for(c->tun.base_threshold);
    P.tbase = c->tun.base_threshold;
    P.vmax = narrow_v(c->tun);
    P.wv = wide_v(c->tun);
    if (P.wv) {
        P.wsplit = (WSplit *)(w + L.wsplit);
        P.wst = (uint32_t *)(w + L.wst);
        P.wen = (uint32_t *)(w + L.wen);
        P.btmp = (uint16_t *)(w + L.btmp);
    }
    P.equal = (c->tun.flags & SSORT_EQUAL) ? 1u : 0u;
    P.limit_ticks = (unsigned long long)c->wait_ms * c->wall_khz;
    P.limit_iters = (unsigned long long)c->wait_ms * 2000ull;   // polls take well over 0.5 us each
    P.alpha = (c->tun.flags & SSORT_ALPHABET) ? (Alphabet *)(w + L.alpha) : nullptr;
    return P;
}

}  // namespace

extern "C" {

const char *ssort_strerror(ssort_status s) {
    switch (s) {
    case SSORT_OK: return "ok";
    case SSORT_EINVAL: return "invalid argument";
    case SSORT_ENOMEM: return "out of memory";
    case SSORT_EWORKSPACE: return "workspace too small";
    case SSORT_EBOUNDS: return "string outside the character buffer";
    case SSORT_EZEROBYTE: return "string contains a zero byte";
    case SSORT_EDEVICE: return "HIP runtime error";
    case SSORT_EBUSY: return "job larger than the memory budget";
    case SSORT_ETIMEOUT: return "device work-queue wait timed out";
    case SSORT_ENOTFOUND: return "unknown ticket";
    }
    return "unknown status";
}

ssort_status ssort_create(int device, const ssort_tuning *t, ssort_ctx **out) {
    if (!out) return SSORT_EINVAL;
    *out = nullptr;
    ssort_tuning tun = t ? *t : ssort_tuning{255, 4, 128, 0};
    if (!valid_tuning(tun)) return SSORT_EINVAL;
    if (device < 0 && hipGetDevice(&device) != hipSuccess) return SSORT_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return SSORT_EDEVICE;
    ssort_ctx *c = (ssort_ctx *)calloc(1, sizeof(ssort_ctx));
    if (!c) return SSORT_ENOMEM;
    c->device = device;
    c->tun = tun;
    c->wait_ms = 20000;
    if (hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) {
        free(c);
        return SSORT_EDEVICE;
    }
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) != hipSuccess || khz <= 0) khz = 100000;
    c->wall_khz = (unsigned long long)khz;
    int nb = 0;
    if (occupancy(tun, &nb) != hipSuccess || nb < 1) nb = 1;
    c->worker_blocks = c->cus * nb;
    c->scratch = scratch_of(device);
    *out = c;
    return SSORT_OK;
}

void ssort_destroy(ssort_ctx *ctx) {
    if (!ctx) return;
    if (ctx->prof)
        for (int i = 0; i < 4; ++i) (void)hipEventDestroy(ctx->ev[i]);
    free(ctx);
}

ssort_status ssort_profile(ssort_ctx *ctx, int enable) {
    if (!ctx) return SSORT_EINVAL;
    if (enable && !ctx->prof) {
        for (int i = 0; i < 4; ++i)
            if (hipEventCreate(&ctx->ev[i]) != hipSuccess) return SSORT_EDEVICE;
        ctx->prof = 1;
    } else if (!enable && ctx->prof) {
        for (int i = 0; i < 4; ++i) (void)hipEventDestroy(ctx->ev[i]);
        ctx->prof = 0;
    }
    return SSORT_OK;
}

ssort_status ssort_phase_ms(ssort_ctx *ctx, float *ms) {
    if (!ctx || !ms || !ctx->prof) return SSORT_EINVAL;
    if (hipEventSynchronize(ctx->ev[3]) != hipSuccess) return SSORT_EDEVICE;
    if (hipEventElapsedTime(&ms[0], ctx->ev[0], ctx->ev[1]) != hipSuccess) return SSORT_EDEVICE;
    if (hipEventElapsedTime(&ms[1], ctx->ev[1], ctx->ev[2]) != hipSuccess) return SSORT_EDEVICE;
    if (hipEventElapsedTime(&ms[2], ctx->ev[2], ctx->ev[3]) != hipSuccess) return SSORT_EDEVICE;
    if (hipEventElapsedTime(&ms[3], ctx->ev[0], ctx->ev[3]) != hipSuccess) return SSORT_EDEVICE;
    return SSORT_OK;
}

ssort_status ssort_get_tuning(const ssort_ctx *ctx, ssort_tuning *t) {
    if (!ctx || !t) return SSORT_EINVAL;
    *t = ctx->tun;
    return SSORT_OK;
}

ssort_status ssort_device_info(const ssort_ctx *ctx, uint64_t *out) {
    if (!ctx || !out) return SSORT_EINVAL;
    out[0] = (uint64_t)ctx->cus;
    out[1] = (uint64_t)ctx->worker_blocks;
    out[2] = ctx->wall_khz;
    out[3] = (uint64_t)ctx->device;
    return SSORT_OK;
}

ssort_status ssort_set_wait_limit(ssort_ctx *ctx, uint32_t ms) {
    if (!ctx || ms == 0) return SSORT_EINVAL;
    ctx->wait_ms = ms;
    return SSORT_OK;
}

ssort_status ssort_workspace_bytes(const ssort_ctx *ctx, uint32_t n, uint32_t m, size_t *bytes) {
    if (!ctx || !bytes || m == 0) return SSORT_EINVAL;
    *bytes = layout(ctx, n, m).total;
    return SSORT_OK;
}

ssort_status ssort_sort(ssort_ctx *ctx, const ssort_strings *in, uint32_t *out_perm, uint32_t *out_lcp, void *ws,
                        size_t ws_bytes, void *stream) {
    if (!ctx) return SSORT_EINVAL;
    ssort_status st = check_strings(in);
    if (st != SSORT_OK) return st;
    if (in->n == 0) return SSORT_OK;
    if (!out_perm || !ws) return SSORT_EINVAL;
    const Layout L = layout(ctx, in->n, 1);
    if (ws_bytes < L.total) return SSORT_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (hipSetDevice(ctx->device) != hipSuccess) return SSORT_EDEVICE;
    Params P = make_params(ctx, in, out_perm, out_lcp, ws, L, 1, nullptr);
    if (ctx->prof) (void)hipEventRecord(ctx->ev[0], s);
    hipLaunchKernelGGL(k_init, dim3(grid_for(L.cap)), dim3(NT), 0, s, P, (unsigned long long)L.cap);
    if (ctx->tun.flags & SSORT_VALIDATE) hipLaunchKernelGGL(k_validate, dim3(grid_for(in->n)), dim3(NT), 0, s, P);
    launch_alphabet(ctx, P, s);
    hipLaunchKernelGGL(k_seed, dim3(1), dim3(NT), 0, s, P, 1u, 0u, 0u);
    if (in->n > ROOT_MIN) launch_levels(ctx, P, L, true, s);
    if (ctx->prof) (void)hipEventRecord(ctx->ev[1], s);
    launch_worker(ctx, P, worker_grid(ctx, in->n, in->n > ROOT_MIN ? NBMAX : 1), s);
    if (ctx->prof) (void)hipEventRecord(ctx->ev[2], s);
    if (out_lcp) launch_seam(ctx, P, s);
    if (ctx->prof) (void)hipEventRecord(ctx->ev[3], s);
    ctx->last_ws = ws;
    return hipGetLastError() == hipSuccess ? SSORT_OK : SSORT_EDEVICE;
}

ssort_status ssort_sort_noalloc(ssort_ctx *ctx, const ssort_strings *in, uint32_t *out_perm, uint32_t *out_lcp,
                                void *stream) {
    if (!ctx) return SSORT_EINVAL;
    ssort_status st = check_strings(in);
    if (st != SSORT_OK) return st;
    if (in->n == 0) return SSORT_OK;
    if (!out_perm) return SSORT_EINVAL;
    if (layout(ctx, in->n, 1).total > (size_t)SSORT_NOALLOC_SCRATCH_BYTES) return SSORT_EWORKSPACE;
    if (!ctx->scratch) return SSORT_EDEVICE;
    // the same launches as ssort_sort, on the device's scratch array (k_init
    // clears its control block and queue; every other part is written before
    // it is read)
    return ssort_sort(ctx, in, out_perm, out_lcp, ctx->scratch, (size_t)SSORT_NOALLOC_SCRATCH_BYTES, stream);
}

ssort_status ssort_sort_batched(ssort_ctx *ctx, const ssort_strings *flat, const uint32_t *set_begin, uint32_t m,
                                uint32_t *out_perm, uint32_t *out_lcp, void *ws, size_t ws_bytes, void *stream) {
    if (!ctx || m == 0 || !set_begin) return SSORT_EINVAL;
    ssort_status st = check_strings(flat);
    if (st != SSORT_OK) return st;
    if (flat->n == 0) return SSORT_OK;
    if (!out_perm || !ws) return SSORT_EINVAL;
    const Layout L = layout(ctx, flat->n, m);
    if (ws_bytes < L.total) return SSORT_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (hipSetDevice(ctx->device) != hipSuccess) return SSORT_EDEVICE;
    Params P = make_params(ctx, flat, out_perm, out_lcp, ws, L, m, set_begin);
    if (ctx->prof) (void)hipEventRecord(ctx->ev[0], s);
    hipLaunchKernelGGL(k_init, dim3(grid_for(L.cap)), dim3(NT), 0, s, P, (unsigned long long)L.cap);
    if (ctx->tun.flags & SSORT_VALIDATE) hipLaunchKernelGGL(k_validate, dim3(grid_for(flat->n)), dim3(NT), 0, s, P);
    launch_alphabet(ctx, P, s);
    hipLaunchKernelGGL(k_seed, dim3(grid_for(m)), dim3(NT), 0, s, P, 2u, 0u, 0u);
    if (flat->n > ROOT_MIN) launch_levels(ctx, P, L, true, s);
    if (ctx->prof) (void)hipEventRecord(ctx->ev[1], s);
    launch_worker(ctx, P, worker_grid(ctx, flat->n, m), s);
    if (ctx->prof) (void)hipEventRecord(ctx->ev[2], s);
    if (out_lcp) launch_seam(ctx, P, s);
    if (ctx->prof) (void)hipEventRecord(ctx->ev[3], s);
    ctx->last_ws = ws;
    return hipGetLastError() == hipSuccess ? SSORT_OK : SSORT_EDEVICE;
}

// ---- K-way LCP-merge ----
namespace {
constexpr uint32_t MERGE_G = 128;   // sample spacing: n / MERGE_G jobs of about MERGE_G strings each
constexpr uint32_t MERGE_LCAP = 64;   // longer jobs are split

struct MergeLayout {
    size_t ctl, ent, cuts, cuth, cutc, ja, jb, xd, total;
    uint32_t nsamp, xcap;
};

MergeLayout merge_layout(uint32_t n, const uint32_t *run_begin, uint32_t K) {
    MergeLayout L;
    L.nsamp = 0;
    for (uint32_t k = 0; k < K; ++k) L.nsamp += (run_begin[k + 1] - run_begin[k] + MERGE_G - 1) / MERGE_G;
    size_t off = 0;
    L.ctl = off;
    off = align_up(off + sizeof(Ctl), 256);
    L.ent = off;
    off = align_up(off + sizeof(ssm::MEnt) * (size_t)n, 256);
    L.xcap = n / MERGE_LCAP + 1;
    const size_t rows = (size_t)(L.nsamp + 1 + L.xcap) * K;
    L.cuts = off;
    off = align_up(off + 4 * rows, 256);
    L.cuth = off;
    off = align_up(off + 4 * rows, 256);
    L.cutc = off;
    off = align_up(off + 8 * rows, 256);
    L.ja = off;
    off = align_up(off + 4 * (size_t)(L.nsamp + L.xcap), 256);
    L.jb = off;
    off = align_up(off + 4 * (size_t)(L.nsamp + L.xcap), 256);
    L.xd = off;
    off = align_up(off + 12 * (size_t)L.xcap, 256);
    L.total = off;
    return L;
}

bool valid_runs(const uint32_t *run_begin, uint32_t K) {
    if (!run_begin || K < 1 || K > (uint32_t)ssm::MKMAX || run_begin[0] != 0) return false;
    for (uint32_t k = 0; k < K; ++k)
        if (run_begin[k + 1] < run_begin[k]) return false;
    return true;
}
}  // namespace

ssort_status ssort_merge_workspace_bytes(const ssort_ctx *ctx, const uint32_t *run_begin, uint32_t K, size_t *bytes) {
    if (!ctx || !bytes || !valid_runs(run_begin, K)) return SSORT_EINVAL;
    *bytes = merge_layout(run_begin[K], run_begin, K).total;
    return SSORT_OK;
}

ssort_status ssort_merge(ssort_ctx *ctx, const ssort_strings *in, const uint32_t *run_begin, uint32_t K,
                         const uint32_t *perm_in, const uint32_t *lcp_in, uint32_t *out_perm, uint32_t *out_lcp,
                         void *ws, size_t ws_bytes, void *stream) {
    if (!ctx) return SSORT_EINVAL;
    ssort_status st = check_strings(in);
    if (st != SSORT_OK) return st;
    if (!valid_runs(run_begin, K)) return SSORT_EINVAL;
    const uint32_t n = run_begin[K];
    if (n == 0) return SSORT_OK;
    if (!perm_in || !lcp_in || !out_perm || !ws) return SSORT_EINVAL;
    const MergeLayout L = merge_layout(n, run_begin, K);
    if (ws_bytes < L.total) return SSORT_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (hipSetDevice(ctx->device) != hipSuccess) return SSORT_EDEVICE;
    ssm::MergeParams M;
    memset(&M, 0, sizeof(M));
    M.S.chars = in->chars;
    M.S.nchars = in->nchars;
    M.S.off = in->offsets;
    M.S.len = in->lengths;
    M.S.n = in->n;
    M.S.flags = in->flags;
    for (uint32_t k = 0; k <= K; ++k) M.rb[k] = run_begin[k];
    M.pin = perm_in;
    M.hin = lcp_in;
    M.pout = out_perm;
    M.hout = out_lcp;
    char *w = (char *)ws;
    M.err = &((Ctl *)(w + L.ctl))->error;
    M.next_job = &((Ctl *)(w + L.ctl))->head;
    M.nsplit = &((Ctl *)(w + L.ctl))->tail;
    M.ent = (ssm::MEnt *)(w + L.ent);
    M.cuts = (uint32_t *)(w + L.cuts);
    M.cuth = (uint32_t *)(w + L.cuth);
    M.cutc = (uint64_t *)(w + L.cutc);
    M.ja = (uint32_t *)(w + L.ja);
    M.jb = (uint32_t *)(w + L.jb);
    M.xd = (uint32_t *)(w + L.xd);
    M.K = K;
    M.n = n;
    M.g = MERGE_G;
    M.nsamp = L.nsamp;
    M.lcap = MERGE_LCAP;
    M.xcap = L.xcap;
    hipLaunchKernelGGL(ssm::k_mreset, dim3(grid_for((uint64_t)(L.nsamp + 1) * K)), dim3(NT), 0, s, M);
    hipLaunchKernelGGL(ssm::k_mcache, dim3(grid_for(n)), dim3(NT), 0, s, M);
    {
        // KP lanes per sample (KP: the smallest power of two >= K, at most 32)
        uint32_t kps = 1;
        while (kps < K) kps <<= 1;
        hipLaunchKernelGGL(ssm::k_msample, dim3((uint32_t)(((size_t)L.nsamp * kps + 63) / 64)), dim3(64), 0, s, M);
        hipLaunchKernelGGL(ssm::k_msplit, dim3((uint32_t)(((size_t)L.nsamp * kps + ssm::SPLIT_NT - 1) / ssm::SPLIT_NT)),
                           dim3(ssm::SPLIT_NT), 0, s, M);
        hipLaunchKernelGGL(ssm::k_msplit_rows, dim3((uint32_t)(((size_t)L.xcap * kps + 63) / 64)), dim3(64), 0, s, M);
    }
    {
        // the loser tree's LDS arrays sized for the smallest power of two >= K
        uint32_t kp = 2;
        while (kp < K) kp <<= 1;
        // one lane per job up to what the chip holds at once (lanes claim
        // further jobs as they finish theirs): the merge is bound by each
        // lane's chain of dependent loads, so every resident lane counts
        const void *fn = kp <= 2    ? (const void *)ssm::k_mmerge<2>
                         : kp == 4  ? (const void *)ssm::k_mmerge<4>
                         : kp == 8  ? (const void *)ssm::k_mmerge<8>
                         : kp == 16 ? (const void *)ssm::k_mmerge<16>
                                    : (const void *)ssm::k_mmerge<ssm::MKMAX>;
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, ssm::MNT, 0) != hipSuccess || per_cu < 1) per_cu = 1;
        const uint64_t want = ((uint64_t)L.nsamp + L.xcap + ssm::MNT - 1) / ssm::MNT;
        const dim3 g((uint32_t)std::min<uint64_t>(want, (uint64_t)per_cu * (uint64_t)ctx->cus)), b(ssm::MNT);
        if (kp <= 2) hipLaunchKernelGGL(ssm::k_mmerge<2>, g, b, 0, s, M);
        else if (kp == 4) hipLaunchKernelGGL(ssm::k_mmerge<4>, g, b, 0, s, M);
        else if (kp == 8) hipLaunchKernelGGL(ssm::k_mmerge<8>, g, b, 0, s, M);
        else if (kp == 16) hipLaunchKernelGGL(ssm::k_mmerge<16>, g, b, 0, s, M);
        else hipLaunchKernelGGL(ssm::k_mmerge<ssm::MKMAX>, g, b, 0, s, M);
    }
    if (out_lcp) hipLaunchKernelGGL(ssm::k_mseam, dim3((L.nsamp + L.xcap + 63) / 64), dim3(64), 0, s, M);
    ctx->last_ws = ws;
    return hipGetLastError() == hipSuccess ? SSORT_OK : SSORT_EDEVICE;
}

ssort_status ssort_query_error(ssort_ctx *ctx, void *stream) {
    if (!ctx) return SSORT_EINVAL;
    if (!ctx->last_ws) return SSORT_OK;
    Ctl c;
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(&c, ctx->last_ws, sizeof(Ctl), hipMemcpyDeviceToHost, s) != hipSuccess) return SSORT_EDEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return SSORT_EDEVICE;
    if (c.error & ERR_BOUNDS) return SSORT_EBOUNDS;
    if (c.error & ERR_ZERO) return SSORT_EZEROBYTE;
    if (c.error & ERR_TIMEOUT) return SSORT_ETIMEOUT;
    if (c.error) return SSORT_EDEVICE;
    return SSORT_OK;
}

ssort_status ssort_stats(ssort_ctx *ctx, ssort_stats_t *out, void *stream) {
    if (!ctx || !out) return SSORT_EINVAL;
    memset(out, 0, sizeof(*out));
    if (!ctx->last_ws) return SSORT_OK;
    Ctl c;
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(&c, ctx->last_ws, sizeof(Ctl), hipMemcpyDeviceToHost, s) != hipSuccess) return SSORT_EDEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return SSORT_EDEVICE;
    out->segments = c.st[ST_SEGMENTS];
    out->strings = c.st[ST_STRINGS];
    out->base_groups = c.st[ST_BASE];
    out->max_depth = c.st[ST_MAX_DEPTH];
    for (int k = 0; k < NPH; ++k) out->phase_ticks[k] = c.ph[k];
    out->base_chunks = c.st[ST_CHUNKS];
    out->base_rounds = c.st[ST_ROUNDS];
    out->max_task = c.st[ST_MAX_TASK];
    out->max_chunk = c.st[ST_MAX_CHUNK];
    out->published_chunks = c.st[ST_PUBCHUNKS];
    out->error_bits = c.error;
    return SSORT_OK;
}

ssort_status ssort_debug_step(ssort_ctx *ctx, const ssort_strings *in, uint32_t depth, uint64_t *keys, uint64_t *split,
                              uint64_t *tree, uint16_t *jump, uint32_t *info, uint16_t *bucket, uint32_t *hist,
                              uint32_t *perm, void *ws, size_t ws_bytes, void *stream) {
    if (!ctx) return SSORT_EINVAL;
    ssort_status st = check_strings(in);
    if (st != SSORT_OK) return st;
    if (in->n == 0 || !keys || !split || !tree || !info || !bucket || !hist || !perm || !ws) return SSORT_EINVAL;
    const Layout L = layout(ctx, in->n, 1);
    if (ws_bytes < L.total) return SSORT_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (hipSetDevice(ctx->device) != hipSuccess) return SSORT_EDEVICE;
    Params P = make_params(ctx, in, perm, nullptr, ws, L, 1, nullptr);
    P.alpha = nullptr;   // the dump reports 8-byte keys
    hipLaunchKernelGGL(k_init, dim3(grid_for(L.cap)), dim3(NT), 0, s, P, (unsigned long long)L.cap);
    hipLaunchKernelGGL(k_seed, dim3(1), dim3(NT), 0, s, P, 1u, depth, 1u);
    launch_levels(ctx, P, L, false, s);
    if (P.wv)
        hipLaunchKernelGGL(k_wdebug_dump, dim3(grid_for(in->n)), dim3(NT), 0, s, P, depth, keys, split, tree, jump, info,
                           bucket, hist, perm);
    else
        hipLaunchKernelGGL(k_debug_dump, dim3(grid_for(in->n)), dim3(NT), 0, s, P, depth, keys, split, tree, info,
                           bucket, hist, perm);
    ctx->last_ws = ws;
    return hipGetLastError() == hipSuccess ? SSORT_OK : SSORT_EDEVICE;
}

ssort_status ssort_debug_segment_step(ssort_ctx *ctx, const ssort_strings *in, uint32_t depth, uint64_t *split,
                                      uint32_t *info, uint32_t *splitter_lcp, uint32_t *ends, uint32_t *bucket_start,
                                      uint32_t *bucket_size, uint32_t *child_depth, uint32_t *perm, void *ws,
                                      size_t ws_bytes, void *stream) {
    if (!ctx) return SSORT_EINVAL;
    ssort_status st = check_strings(in);
    if (st != SSORT_OK) return st;
    if (in->n == 0 || !split || !info || !splitter_lcp || !ends || !bucket_start || !bucket_size || !child_depth ||
        !perm || !ws)
        return SSORT_EINVAL;
    const Layout L = layout(ctx, in->n, 1);
    if (ws_bytes < L.total) return SSORT_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (hipSetDevice(ctx->device) != hipSuccess) return SSORT_EDEVICE;
    Params P = make_params(ctx, in, perm, nullptr, ws, L, 1, nullptr);
    P.alpha = nullptr;   // byte keys
    hipLaunchKernelGGL(k_init, dim3(grid_for(L.cap)), dim3(NT), 0, s, P, (unsigned long long)L.cap);
    const int C = chunk_for(ctx->tun.base_threshold);
    const dim3 g(1), b(NT);
    if (ctx->tun.keys_per_thread == 4 && C == 512)
        hipLaunchKernelGGL((k_debug_segstep<4, 512, false>), g, b, 0, s, P, depth, split, info, splitter_lcp, ends,
                           bucket_start, bucket_size, child_depth);
    else if (ctx->tun.keys_per_thread == 4)
        hipLaunchKernelGGL((k_debug_segstep<4, 1024, false>), g, b, 0, s, P, depth, split, info, splitter_lcp, ends,
                           bucket_start, bucket_size, child_depth);
    else if (C == 512)
        hipLaunchKernelGGL((k_debug_segstep<8, 512, false>), g, b, 0, s, P, depth, split, info, splitter_lcp, ends,
                           bucket_start, bucket_size, child_depth);
    else
        hipLaunchKernelGGL((k_debug_segstep<8, 1024, false>), g, b, 0, s, P, depth, split, info, splitter_lcp, ends,
                           bucket_start, bucket_size, child_depth);
    hipLaunchKernelGGL(k_debug_perm, dim3(grid_for(in->n)), dim3(NT), 0, s, P, perm);
    ctx->last_ws = ws;
    return hipGetLastError() == hipSuccess ? SSORT_OK : SSORT_EDEVICE;
}

struct ssort_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

ssort_status ssort_graph_create(ssort_ctx *ctx, const ssort_strings *in, const uint32_t *set_begin, uint32_t m,
                                uint32_t *out_perm, uint32_t *out_lcp, void *ws, size_t ws_bytes, void *stream,
                                ssort_graph **out) {
    if (!ctx || !out || !stream) return SSORT_EINVAL;
    *out = nullptr;
    hipStream_t s = (hipStream_t)stream;
    const int prof = ctx->prof;
    ctx->prof = 0;   // no event records inside the graph
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        ctx->prof = prof;
        return SSORT_EDEVICE;
    }
    ssort_status rc = set_begin ? ssort_sort_batched(ctx, in, set_begin, m, out_perm, out_lcp, ws, ws_bytes, stream)
                                : ssort_sort(ctx, in, out_perm, out_lcp, ws, ws_bytes, stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &g);
    ctx->prof = prof;
    if (rc != SSORT_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess || !g) return SSORT_EDEVICE;
    ssort_graph *G = (ssort_graph *)calloc(1, sizeof(ssort_graph));
    if (!G) {
        (void)hipGraphDestroy(g);
        return SSORT_ENOMEM;
    }
    G->graph = g;
    if (hipGraphInstantiate(&G->exec, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        free(G);
        return SSORT_EDEVICE;
    }
    *out = G;
    return SSORT_OK;
}

ssort_status ssort_graph_launch(ssort_graph *g, void *stream) {
    if (!g) return SSORT_EINVAL;
    return hipGraphLaunch(g->exec, (hipStream_t)stream) == hipSuccess ? SSORT_OK : SSORT_EDEVICE;
}

void ssort_graph_destroy(ssort_graph *g) {
    if (!g) return;
    (void)hipGraphExecDestroy(g->exec);
    (void)hipGraphDestroy(g->graph);
    free(g);
}

}  // extern "C"
