// Kernels of the string sample sorter and the state they share.
#pragma once
#include "ssort_dev.h"

namespace ssd {

// Control block at the start of the workspace.
struct Ctl {
    unsigned long long head;      // next queue position to claim
    unsigned long long tail;      // next queue position to fill
    unsigned long long pending;   // tasks enqueued or running, not finished
    unsigned long long error;     // bit mask of device errors
    unsigned long long st_segments, st_strings, st_base, st_maxdepth;
    unsigned long long ph[8];     // worker time per phase, wall-clock ticks summed over workgroups
};

// worker phases timed on the device
enum { PH_WAIT = 0, PH_SAMPLE = 1, PH_CLASSIFY = 2, PH_SCATTER = 3, PH_CHILDREN = 4, PH_BASE = 5,
       PH_EXTEND = 6, PH_OTHER = 7 };

enum : unsigned long long { ERR_TIMEOUT = 1, ERR_BOUNDS = 2, ERR_ZERO = 4, ERR_QUEUE = 8, ERR_INTERNAL = 16 };

// Task meta bits
enum : uint32_t {
    M_PARITY = 1u,       // records of the segment are in R[1] (else R[0])
    M_IDENT_SRC = 2u,    // records come straight from the input (identity order)
    M_IDENT = 4u,        // all strings identical (equality bucket of a terminated splitter)
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
    Split *gsplit;           // root step splitters (global copy)
    uint32_t *hist;          // root step tile histograms, bucket-major [nb][ntiles]
    uint32_t *totals;        // root step bucket totals [NBPAD]
    const uint32_t *set_begin;   // batched: m+1 set boundaries, else null
    uint32_t m;              // number of sets (1 for a plain sort)
    uint32_t ntiles;
    uint32_t tbase;
    uint32_t vmax;
    uint32_t equal;          // S5-Equal classification
    unsigned long long limit_ticks;
    unsigned long long limit_iters;
    uint32_t dbg;            // debug step: stop after the root redistribution
    uint32_t pad;
};

}  // namespace ssd
