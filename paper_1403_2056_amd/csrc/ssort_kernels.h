// Kernels of the string sample sorter and the state they share.
#pragma once
#include "ssort_dev.h"

namespace ssd {

constexpr int NPH = 16;
constexpr int NST = 9;

// Whole-GPU steps: segments of more than LVL_MIN strings (the input itself,
// or a batched set, when larger than ROOT_MIN) are classified and
// redistributed by every workgroup of the GPU at once, LMAX levels deep,
// before the persistent workers take over.
constexpr int LMAX = 2;
constexpr uint32_t ROOT_MIN = 1u << 16;
constexpr uint32_t LVL_MIN = 1u << 16;

// One segment of a whole-GPU level: its strings, depth and record source,
// and its tiles (ROOT_CHUNKS chunks of NT*K strings each) in the level's tile
// numbering.
struct __align__(32) LvlSeg {
    uint32_t begin, size, depth, meta;
    uint32_t tile0, ntile, setbase, pad;
};

// Control block at the start of the workspace.  The queue counters each
// sit on a cache line of their own: every idle workgroup polls `pending`,
// and traffic to one line is served by one L2 channel, whose congestion
// slows every other access mapped to that channel.  Statistics are summed
// per workgroup in LDS and added here once, when the workgroup exits.
struct Ctl {
    alignas(128) unsigned long long head;      // next queue position to claim
    alignas(128) unsigned long long tail;      // next queue position to fill
    alignas(128) unsigned long long pending;   // tasks enqueued or running, not finished
    alignas(128) unsigned long long error;     // bit mask of device errors
    alignas(128) unsigned long long desc_top;  // group descriptors handed out
    alignas(128) unsigned long long lvl[LMAX][2];   // whole-GPU levels: segments, tiles
    alignas(128) unsigned long long st[NST];   // statistics (ST_*)
    unsigned long long ph[NPH];                // worker time per phase, wall-clock ticks summed over workgroups
};

// statistics: sums, except the ST_MAX_* entries (maxima)
enum {
    ST_SEGMENTS = 0, ST_STRINGS = 1, ST_BASE = 2, ST_CHUNKS = 3, ST_ROUNDS = 4, ST_PUBCHUNKS = 5,
    ST_MAX_DEPTH = 6,   // largest classification depth
    ST_MAX_TASK = 7,    // longest task: ticks << 24 | size (capped)
    ST_MAX_CHUNK = 8,   // longest base chunk: ticks << 24 | rounds << 12 | strings
};

// worker phases timed on the device
enum { PH_WAIT = 0, PH_SAMPLE = 1, PH_CLASSIFY = 2, PH_SCATTER = 3, PH_CHILDREN = 4, PH_BASE = 5,
       PH_EXTEND = 6, PH_OTHER = 7, PH_BEXT = 8, PH_BKEY = 9, PH_BRANK = 10,
       PH_DRAIN = 11, PH_BSPLIT = 12 };

// Device error bits (the mask reads back through the statistics): input
// errors, the wait limit, and one bit per internal consistency check, each of
// which ends the sort instead of letting an access leave its buffer.
enum : unsigned long long {
    ERR_TIMEOUT = 1,     // a work-queue wait exceeded its limit
    ERR_BOUNDS = 2,      // a string lies outside the character buffer (validation)
    ERR_ZERO = 4,        // a string holds the byte 0 (validation)
    ERR_QUEUE = 8,       // a ring slot to fill still held an unconsumed task
    ERR_DESC_CAP = 16,   // the group-descriptor array is full
    ERR_TASK = 32,       // a task or group descriptor outside the string range
    ERR_CHUNK = 64,      // a base-case chunk larger than the workgroup holds
    ERR_SCATTER = 128,   // a redistribution target outside the segment's range
    ERR_LEVEL = 256,     // a whole-GPU level's segment or tile table overflowed
    ERR_MERGE = 512,     // a merge job's rank beyond the sample count, or a run index outside the set
    ERR_SEAM = 1024      // an output permutation entry outside its set at a bucket seam
};

// Task meta bits
enum : uint32_t {
    M_PARITY = 1u,       // records of the segment are in R[1] (else R[0])
    M_IDENT_SRC = 2u,    // records come straight from the input (identity order)
    M_IDENT = 4u,        // all strings identical (equality bucket of a terminated splitter)
    M_CHUNK = 8u,        // a base-case chunk: begin = first group descriptor, size = groups, depth = strings
};

// A base-case group: global start, size and common depth of its strings.
struct __align__(16) GroupDesc {
    uint32_t start, size, depth, pad;
};

// Wide whole-GPU level (the larger trees of the paper's implementation
// details, v up to 4095, with the multipass distribution and jump table of its
// refinements): the splitters of one segment, built by one workgroup and read
// by every tile.  Same fields as Split, larger arrays, plus the jump table:
// jump[p] is the tree node where the descent of every key whose top JA bits
// are p still has to continue (or the leaf it reaches).
constexpr int WVMAX = 4095;               // largest wide splitter count (d = 12)
constexpr int WDMAX = 12;
constexpr int WNBPAD = 8192;              // 2 * WVMAX + 1 buckets, padded
constexpr int JA = 12;                    // key bits indexing the jump table
constexpr int WLO = 7;                    // bits of the first distribution digit
struct WSplit {
    uint64_t tree[WVMAX + 1];   // level order, tree[1..v]
    uint16_t jump[1 << JA];
    uint8_t hl[WVMAX + 1];
    uint8_t zr[WVMAX + 1];
    uint32_t v, d, nb, nbits, ndistinct, ulast, equal, q;
};

// One queue slot (bounded MPMC ring with per-slot sequence numbers).
struct __align__(32) Slot {
    unsigned long long seq;
    uint32_t begin, size, depth, meta;
    uint32_t setbase, pad0;
};

struct Params {
    Strs S;
    Rec *R0, *R1;
    uint16_t *bkt;
    uint32_t *perm;
    uint32_t *lcp;           // may be null
    Slot *ring;
    unsigned long long ring_mask;
    Ctl *ctl;
    LvlSeg *lseg[LMAX];      // whole-GPU levels: segments
    uint32_t *tile2seg[LMAX];   // tile -> segment
    Split *lsplit[LMAX];     // splitters per segment
    uint32_t *ltot[LMAX];    // bucket totals per segment [seg][NBPAD]
    uint32_t *hist;          // tile histograms of the current level, tile-major [tile][NBPAD]
    GroupDesc *desc;         // base-case group descriptors (at most one per group)
    uint64_t desc_cap;
    const uint32_t *set_begin;   // batched: m+1 set boundaries, else null
    uint32_t m;              // number of sets (1 for a plain sort)
    uint32_t lmaxseg, lmaxtiles;   // capacity of each level's segment and tile arrays
    uint32_t tile;           // strings per tile (ROOT_CHUNKS * NT * K)
    uint32_t chunk;          // base-case chunk capacity C
    uint32_t tbase;
    uint32_t vmax;
    uint32_t equal;          // S5-Equal classification
    unsigned long long limit_ticks;
    unsigned long long limit_iters;
    Alphabet *alpha;         // alphabet compression: codes of the input's byte values, else null
    // wide level 0 (wv > 0 splitters): splitters, bucket bounds per segment
    // (segment-relative first and one-past-last position of each bucket),
    // and the bucket numbers between the two distribution passes
    uint32_t wv;
    WSplit *wsplit;
    uint32_t *wst, *wen;
    uint16_t *btmp;
};

}  // namespace ssd
