/*
 * ssort.h: C ABI of libssort.so, a string sorter for one AMD Instinct MI355X
 * (gfx950) built on parallel super scalar string sample sort.
 *
 * Problem (Preliminaries): n strings of total length N over an alphabet that
 * excludes the zero byte; sort them lexicographically (unsigned bytes, a
 * proper prefix before its extensions) and return the sorted order together
 * with the LCP array H, H[0] = 0 and H[i] = lcp(s_perm[i-1], s_perm[i]).
 * Identical strings appear in ascending input index, so the result is unique.
 *
 * Conventions for every call below:
 *  - "device pointer" means memory of the context's GPU (hipMalloc or a torch
 *    CUDA tensor); "host pointer" means ordinary process memory.
 *  - The caller owns every buffer.  No call allocates device memory except
 *    ssort_graph_create / ssort_server_create (and ssort_profile, which
 *    creates HIP events); ssort_create may load the library's code on the
 *    device, which holds the ssort_sort_noalloc array.
 *  - Sorting calls are asynchronous: they only enqueue work on `stream` (a
 *    hipStream_t, or NULL for the default stream) and return.  Outputs are valid
 *    once the stream has been synchronised.  They do not synchronise and do not
 *    allocate, so they can be captured into a HIP graph.
 *  - Host-checkable errors (null pointers, sizes, a workspace that is too
 *    small, an invalid tuning) are returned synchronously and nothing is
 *    enqueued.  Errors found on the device (a work-queue wait that exceeded its
 *    time limit, a zero byte or an out-of-range string under SSORT_VALIDATE) are
 *    reported by ssort_query_error after the stream has been synchronised; the
 *    outputs are undefined then.
 *  - A context may be used by one host thread at a time.  Sorts enqueued on
 *    different streams with the same context must use different workspaces.
 */
#ifndef SSORT_H
#define SSORT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SSORT_OK = 0,
    SSORT_EINVAL = 1,      /* bad argument */
    SSORT_ENOMEM = 2,      /* allocation failed (create calls only) */
    SSORT_EWORKSPACE = 3,  /* workspace smaller than ssort_workspace_bytes */
    SSORT_EBOUNDS = 4,     /* device: a string lies outside the character buffer */
    SSORT_EZEROBYTE = 5,   /* device: a string contains the byte 0 */
    SSORT_EDEVICE = 6,     /* HIP runtime error */
    SSORT_EBUSY = 7,       /* serving: job larger than the whole memory budget */
    SSORT_ETIMEOUT = 8,    /* device: a work-queue wait exceeded its time limit */
    SSORT_ENOTFOUND = 9    /* serving: unknown ticket */
} ssort_status;

/* flags of ssort_strings */
#define SSORT_TO_END 1u    /* string i runs from offsets[i] to the end of chars (suffixes) */

/* Input string set (a host struct holding device pointers).
 *  chars    device, nchars bytes, any alignment.  Characters are fetched as
 *           whole aligned 8-byte words: the kernels read only aligned words
 *           that hold at least one byte of [chars, chars + nchars), so a read
 *           may touch up to 7 bytes before chars or after chars + nchars
 *           inside those words (the same pages as the buffer's first and
 *           last bytes, always mapped when the buffer is); those bytes are
 *           never used and may hold anything.
 *  offsets  device uint64: n+1 CSR offsets (string i = chars[offsets[i], offsets[i+1]))
 *           when lengths is NULL and SSORT_TO_END is not set; else n start offsets.
 *  lengths  device uint32[n] or NULL.
 *  n        number of strings, n <= 2^32 - 2.
 * Every string must be shorter than 2^31 bytes and must not contain the byte 0
 * (the terminator is outside the alphabet, Preliminaries). */
typedef struct {
    const uint8_t *chars;
    uint64_t nchars;
    const uint64_t *offsets;
    const uint32_t *lengths;
    uint32_t n;
    uint32_t flags;
} ssort_strings;

/* Tuning of one context.
 *  v               splitters per classification step, 2^d - 1 with d in 1..8
 *                  (63, 127 or 255 in practice; the tree and its 2v+1 bucket
 *                  counters live in LDS).  Algorithm 1; tree size choice in the
 *                  implementation details of S5.  Also 1023, 2047 or 4095:
 *                  then the first whole-GPU level classifies against that
 *                  many splitters, with a jump table over the keys' top 12
 *                  bits for the top of the descent and a distribution in two
 *                  stable passes by the digits of the bucket number (the
 *                  multipass distribution and jump tables of the paper's
 *                  refinements), and every later step uses 255.
 *  keys_per_thread keys each thread classifies at a time: 4 or 8.
 *  base_threshold  segments of at most this many strings go to the LCP-aware
 *                  base case (16..1024).
 *  flags           SSORT_VALIDATE: check strings for bounds and zero bytes
 *                  first (one extra pass over the characters);
 *                  SSORT_EQUAL: classify with an equality test at every tree
 *                  node and an early exit ("S5-Equal", fourth equality-check
 *                  variant of the implementation details of S5) instead of a
 *                  full descent and one equality test ("S5-Unroll").
 *                  SSORT_ALPHABET: alphabet compression (outlook of the
 *                  paper): a first pass finds the sigma' byte values that
 *                  occur in the character buffer; keys then hold
 *                  q = min(64 / b, 32) characters of b = ceil(log2(sigma'+1))
 *                  bits (order-preserving codes, 0 = end of string) instead
 *                  of 8 bytes, e.g. 21 DNA characters.  The permutation and
 *                  LCP array are identical to those without the flag. */
typedef struct {
    uint32_t v;
    uint32_t keys_per_thread;
    uint32_t base_threshold;
    uint32_t flags;
} ssort_tuning;

#define SSORT_VALIDATE 1u
#define SSORT_EQUAL 2u
#define SSORT_ALPHABET 4u

typedef struct ssort_ctx ssort_ctx;

/* Counters of the last sort (filled on the device, read after a sync).
 *  segments     classification steps run (one per segment of > base_threshold strings)
 *  strings      sum over those steps of their sizes (the active strings per level)
 *  base_groups  groups handled by the base case
 *  max_depth    largest depth (bytes) at which a step or base-case round ran
 *  base_chunks  base-case chunks (one workgroup each, several groups)
 *  base_rounds  base-case rounds summed over chunks */
typedef struct {
    uint64_t segments;
    uint64_t strings;
    uint64_t base_groups;
    uint64_t max_depth;
    /* persistent-worker time per phase, summed over workgroups, in wall-clock
     * ticks (ssort_device_info out[2] kHz): 0 waiting for a task, 1 sample and
     * tree, 2 classify and count, 3 redistribution, 4 child scheduling and
     * identical buckets, 5 base case (loading and writing the chunk),
     * 6 common-prefix extension of a segment, 7 other, 8 base-case prefix
     * extension, 9 base-case key gathers, 10 base-case ranking, 11 the last
     * wait (for the queue to drain), 12 base-case class splitting, 13-15
     * unused */
    uint64_t phase_ticks[16];
    uint64_t base_chunks;
    uint64_t base_rounds;
    /* slowest work-queue task: wall-clock ticks << 24 | its string count
     * (capped at 2^24 - 1); slowest base-case chunk: ticks << 24 | rounds
     * << 12 | strings */
    uint64_t max_task;
    uint64_t max_chunk;
    uint64_t published_chunks;   /* base-case chunks handed to other workgroups */
    /* device error mask of the last sort or merge (0: none).  1 wait limit,
     * 2 string outside the buffer, 4 zero byte (these three map to
     * SSORT_ETIMEOUT, SSORT_EBOUNDS, SSORT_EZEROBYTE); the internal
     * consistency checks, each reported as SSORT_EDEVICE: 8 work-queue slot
     * still occupied, 16 group-descriptor array full, 32 task or descriptor
     * outside the string range, 64 base-case chunk too large, 128
     * redistribution target outside its segment, 256 whole-GPU level tables
     * full, 512 merge: an index outside the set, a sample rank out of range,
     * or a cut row unwritten or out of order, 1024 an output permutation
     * entry outside its set at a bucket seam */
    uint64_t error_bits;
} ssort_stats_t;

/* Create a context on HIP device `device` (the current device if < 0).
 * t may be NULL for the default tuning.  Looks up the device address of the
 * ssort_sort_noalloc array (once per device).  Returns SSORT_EINVAL for an
 * invalid tuning. */
ssort_status ssort_create(int device, const ssort_tuning *t, ssort_ctx **out);
void ssort_destroy(ssort_ctx *ctx);
ssort_status ssort_get_tuning(const ssort_ctx *ctx, ssort_tuning *t);

/* Bytes of device workspace ssort_sort needs for n strings (m sets for the
 * batched call; m = 1 for a plain sort). */
ssort_status ssort_workspace_bytes(const ssort_ctx *ctx, uint32_t n, uint32_t m, size_t *bytes);

/* Sort one string set (Algorithm 1 applied recursively, parallel S5).
 *  out_perm  device uint32[n]: input index of the i-th smallest string.
 *  out_lcp   device uint32[n] or NULL: the LCP array, out_lcp[0] = 0.
 *  ws        device workspace of at least ssort_workspace_bytes(ctx, n, 1) bytes.
 * n = 0 enqueues nothing. */
ssort_status ssort_sort(ssort_ctx *ctx, const ssort_strings *in, uint32_t *out_perm,
                        uint32_t *out_lcp, void *ws, size_t ws_bytes, void *stream);

/* ---- sorting without allocation ----
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): ssort_sort
 * without a workspace argument.  The workspace is a device array inside the
 * library of SSORT_NOALLOC_SCRATCH_BYTES bytes, one per GPU, created when the
 * library is loaded on that GPU and held until the process ends; the call
 * itself allocates nothing (no hipMalloc, hipFree or allocating library
 * routine).  The caller still passes the inputs and outputs, as for
 * ssort_sort.  Returns SSORT_EWORKSPACE, enqueuing nothing, when
 * ssort_workspace_bytes(ctx, n, 1) exceeds the array (about 1.2 million
 * strings with the default tuning; 2^20 strings fit with every
 * base_threshold of at least 32), and SSORT_EDEVICE if the array's device
 * address could not be looked up when the context was created.
 * Every call on one GPU uses that GPU's one array, whatever the context:
 * calls whose work overlaps on the device (different streams, or different
 * host threads) race and give undefined results; serialise them (one
 * stream, or a synchronisation between calls).  The array keeps the last
 * call's contents; each call clears what it needs cleared.
 * ssort_query_error and ssort_stats report on it as on a workspace. */
#define SSORT_NOALLOC_SCRATCH_BYTES (64u << 20)
ssort_status ssort_sort_noalloc(ssort_ctx *ctx, const ssort_strings *in, uint32_t *out_perm,
                                uint32_t *out_lcp, void *stream);

/* Sort m independent sets in one launch sequence.  The strings of all sets
 * form one string space `flat`; set s is strings [set_begin[s], set_begin[s+1]).
 *  set_begin  device uint32[m+1], non-decreasing, set_begin[m] = flat->n.
 *  out_perm   device uint32[flat->n]: per set, set-local indices (0-based) in
 *             sorted order, stored at the set's positions.
 *  out_lcp    device uint32[flat->n] or NULL: per-set LCP arrays, 0 at each
 *             set's first position.
 *  ws         at least ssort_workspace_bytes(ctx, flat->n, m) bytes. */
ssort_status ssort_sort_batched(ssort_ctx *ctx, const ssort_strings *flat, const uint32_t *set_begin,
                                uint32_t m, uint32_t *out_perm, uint32_t *out_lcp, void *ws,
                                size_t ws_bytes, void *stream);

/* Device-side errors of the last sort or merge enqueued with this context;
 * call after synchronising its stream (the call copies the error word on
 * `stream` and waits for it).  The word is not reset here: the next sort or
 * merge clears it when it starts. */
ssort_status ssort_query_error(ssort_ctx *ctx, void *stream);

/* Counters of the last sort with this context (after synchronising). */
ssort_status ssort_stats(ssort_ctx *ctx, ssort_stats_t *out, void *stream);

/* Time limit of each work-queue wait, in milliseconds (default 20000).  A wait
 * beyond it ends the sort with SSORT_ETIMEOUT instead of hanging. */
ssort_status ssort_set_wait_limit(ssort_ctx *ctx, uint32_t ms);

/* Device facts the context runs with: out[0] compute units, out[1] resident
 * persistent workgroups (units x occupancy), out[2] wall-clock rate in kHz
 * used for wait limits, out[3] HIP device index.  Host pointer, 4 entries. */
ssort_status ssort_device_info(const ssort_ctx *ctx, uint64_t *out);

/* Phase timing.  With enable = 1 every later sort on this context records
 * HIP events on its stream around its phases (creating them here, the only
 * allocation); ssort_phase_ms then returns, after the stream has been
 * synchronised, the milliseconds of the last sort's phases:
 * ms[0] initialisation and whole-GPU root step, ms[1] persistent workers
 * (segment steps and base cases), ms[2] boundary LCPs, ms[3] whole sort.
 * Host pointer, 4 entries.  Not for use under graph capture. */
ssort_status ssort_profile(ssort_ctx *ctx, int enable);
ssort_status ssort_phase_ms(ssort_ctx *ctx, float *ms);

const char *ssort_strerror(ssort_status s);

/* ---- K-way LCP-merge (Section 5: Algorithm 2, binary LCP-compare; Algorithm
 * 4, K-way LCP-merge with an LCP-aware tournament tree; the caching variant of
 * its implementation details) ----
 * Merges K sorted runs of strings of `in` into one sorted sequence with its
 * LCP array.
 *  run_begin HOST uint32[K+1], run_begin[0] = 0, non-decreasing; run k is
 *            positions run_begin[k] .. run_begin[k+1]-1 of perm_in / lcp_in;
 *            n = run_begin[K] strings in all; 1 <= K <= 32
 *  perm_in   device uint32[n]: indices into `in`, each index in at most one
 *            run (distinct over all runs); each run sorted by (string, index),
 *            i.e. equal strings in index order (as ssort_sort returns them).
 *            Runs that break this are detected on the device (an index outside
 *            the set, two samples of the same rank, cuts out of order) and
 *            reported as SSORT_EDEVICE by ssort_query_error; they never make
 *            the merge access memory outside its buffers.
 *  lcp_in    device uint32[n]: lcp_in[p] = LCP of the strings at positions
 *            p-1 and p of the same run; the entry at a run's start is ignored.
 *            LCPs (in and out) must stay below 2^24 - 8 bytes; a longer one
 *            is reported as SSORT_EDEVICE
 *  out_perm  device uint32[n]: all indices sorted, equal strings by index
 *  out_lcp   device uint32[n] (may be NULL): out_lcp[0] = 0, out_lcp[i] = LCP
 *            of the strings at positions i-1 and i
 * When the runs together hold every index of `in` once, the result equals
 * ssort_sort of `in`.  Workspace from ssort_merge_workspace_bytes (about 40
 * bytes per string).  Asynchronous on `stream`; ssort_query_error reports device
 * errors.  SSORT_EINVAL for bad runs or K. */
ssort_status ssort_merge_workspace_bytes(const ssort_ctx *ctx, const uint32_t *run_begin, uint32_t K, size_t *bytes);
ssort_status ssort_merge(ssort_ctx *ctx, const ssort_strings *in, const uint32_t *run_begin, uint32_t K,
                         const uint32_t *perm_in, const uint32_t *lcp_in, uint32_t *out_perm, uint32_t *out_lcp,
                         void *ws, size_t ws_bytes, void *stream);

/* ---- one classification step with its intermediates (parity checks) ----
 * Runs one step of Algorithm 1 over all n strings of `in` at common depth
 * `depth` (the caller guarantees the strings share that prefix), on the input
 * order, with the library's own sample and splitters: the whole-GPU level-0
 * step, wide (v > 255: jump table and two distribution passes) when the
 * context's tuning asks for it.  Outputs (device):
 *  keys      uint64[n]    8-byte big-endian keys at `depth` (zero past the end)
 *  split     uint64[4096] sorted splitters x_0..x_{v'-1} actually used
 *  tree      uint64[4096] level-order tree, tree[j-1] = node j
 *  jump      uint16[4096] or NULL: the wide step's jump table (jump[p] = the
 *                         node where the descent of keys with top 12 bits p
 *                         continues, > v' for a leaf); untouched when narrow
 *  info      uint32[4]    {v', d', number of distinct sample keys, jump-table
 *                         bits (0 for a narrow step)}
 *  bucket    uint16[n]    bucket of each string (input order), 0..2v'
 *  hist      uint32[8192] strings per bucket
 *  perm      uint32[n]    input indices after the stable redistribution
 * Entries past v' (2v'+1 for hist) are zero up to 256 (512) for a narrow
 * step and up to 4096 (8192) for a wide one.  ws as for ssort_sort with n
 * strings. */
ssort_status ssort_debug_step(ssort_ctx *ctx, const ssort_strings *in, uint32_t depth,
                              uint64_t *keys, uint64_t *split, uint64_t *tree, uint16_t *jump,
                              uint32_t *info, uint16_t *bucket, uint32_t *hist, uint32_t *perm, void *ws,
                              size_t ws_bytes, void *stream);

/* ---- one segment step of the persistent worker with its intermediates ----
 * Runs the step a worker applies to a segment (Algorithm 1 on one segment by
 * one workgroup: sample and splitters, the exact common-prefix extension when
 * every sampled key is equal, classification, count, prefix sum, stable
 * redistribution, scheduling of the children) on all n strings of `in` as one
 * segment at common depth `depth`; the children are not run.  Outputs (device):
 *  split         uint64[256]  sorted splitters x_0..x_{v'-1}
 *  info          uint32[4]    {v', d', distinct sample keys, depth h of the
 *                             classification (>= depth after an extension)}
 *  splitter_lcp  uint32[256]  h'[l] = lcp of x_{l-1} and x_l in bytes (at most
 *                             8), h'[0] = h'[v'] = 0
 *  ends          uint32[256]  1 where x_l ends its string (last byte zero)
 *  bucket_start, bucket_size, child_depth  uint32[512]: per bucket 0..2v',
 *                             its first position in the redistributed order,
 *                             its size, and the common prefix length its
 *                             strings are recursed with (Algorithm 1's output)
 *  perm          uint32[n]    input indices after the stable redistribution
 * Byte keys whatever the tuning's flags.  ws as for ssort_sort with n strings. */
ssort_status ssort_debug_segment_step(ssort_ctx *ctx, const ssort_strings *in, uint32_t depth, uint64_t *split,
                                      uint32_t *info, uint32_t *splitter_lcp, uint32_t *ends, uint32_t *bucket_start,
                                      uint32_t *bucket_size, uint32_t *child_depth, uint32_t *perm, void *ws,
                                      size_t ws_bytes, void *stream);

/* ---- graph-captured launch (the batched form) ----
 * Capture one sort (set_begin == NULL: ssort_sort of `in`; else
 * ssort_sort_batched of m sets) with fixed buffers into a HIP graph on
 * `stream` (which must not be the legacy default stream) and instantiate it;
 * ssort_graph_launch replays the whole sort as one graph launch.  The graph
 * holds no memset nodes: the queue and counters are reset by a kernel in
 * every replay.  Buffers must stay valid while the graph exists. */
typedef struct ssort_graph ssort_graph;
ssort_status ssort_graph_create(ssort_ctx *ctx, const ssort_strings *in, const uint32_t *set_begin, uint32_t m,
                                uint32_t *out_perm, uint32_t *out_lcp, void *ws, size_t ws_bytes, void *stream,
                                ssort_graph **out);
ssort_status ssort_graph_launch(ssort_graph *g, void *stream);
void ssort_graph_destroy(ssort_graph *g);

/* ---- serving: a request loop with continuous batching on one GPU ----
 * The server owns a resident HBM arena of `hbm_budget` bytes (allocated at
 * creation) and `slots` launch slots (streams with pinned staging buffers; 4
 * matches the hardware queues of one process).  A scheduler thread admits
 * waiting jobs in FIFO order while their packed device buffers (characters,
 * descriptors, outputs, sort workspace) fit into the arena and the per-launch
 * limits, sorts each admitted group with one batched launch sequence
 * (ssort_sort_batched) on a free slot, and copies the results back; jobs that
 * arrive while others run join the next free slot, so work overlaps on the
 * device.  Each job's result is identical to sorting it alone. */
typedef struct ssort_server ssort_server;

/* One job: HOST pointers, owned by the caller until ssort_server_wait returns.
 *  chars/nchars/offsets/n/flags  as in ssort_strings (CSR n+1 offsets, or n
 *                                starts with SSORT_TO_END), in host memory
 *  out_perm  host uint32[n], written on completion
 *  out_lcp   host uint32[n] or NULL */
typedef struct {
    const uint8_t *chars;
    uint64_t nchars;
    const uint64_t *offsets;
    uint32_t n;
    uint32_t flags;
    uint32_t *out_perm;
    uint32_t *out_lcp;
} ssort_job;

typedef struct {
    uint64_t ticket;
    int status;          /* ssort_status of the job */
    double latency_ms;   /* submission to completion */
    double queue_ms;     /* submission to launch */
    uint64_t device_error;   /* the launch's device error mask (ssort_stats_t.error_bits) */
} ssort_result;

/* Optional limits (0 = default): pinned staging bytes per slot and direction
 * (256 MiB), jobs per launch (4096), strings per launch (2^26). */
typedef struct {
    size_t stage_bytes;
    uint32_t max_jobs_per_launch;
    uint64_t max_strings_per_launch;
} ssort_server_config;

typedef struct {
    uint64_t submitted, completed, launches, jobs_launched, max_jobs_per_launch;
    uint64_t arena_used, waiting;
} ssort_server_stats_t;

/* Allocates the arena (hipMalloc), pinned staging (hipHostMalloc), streams and
 * contexts; t and cfg may be NULL.  SSORT_ENOMEM if any allocation fails. */
ssort_status ssort_server_create(int device, size_t hbm_budget, uint32_t slots, const ssort_tuning *t,
                                 const ssort_server_config *cfg, ssort_server **out);
/* Queue a job.  SSORT_EBUSY if it could never fit (larger than the arena or a
 * staging buffer); otherwise it waits for memory, FIFO. */
ssort_status ssort_server_submit(ssort_server *srv, const ssort_job *job, uint64_t *ticket);
/* Wait for a job (timeout_ms < 0: forever); returns its status and forgets
 * the ticket.  SSORT_ETIMEOUT if still running, SSORT_ENOTFOUND if unknown or
 * cancelled. */
ssort_status ssort_server_wait(ssort_server *srv, uint64_t ticket, int timeout_ms, ssort_result *res);
/* Remove a job that is still waiting for admission. */
ssort_status ssort_server_cancel(ssort_server *srv, uint64_t ticket);
ssort_status ssort_server_stats(ssort_server *srv, ssort_server_stats_t *out);
void ssort_server_destroy(ssort_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* SSORT_H */
