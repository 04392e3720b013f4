/*
 * mergeshuffle.h -- C ABI of the MI355X (gfx950) MergeShuffle library.
 *
 * MergeShuffle (Bacher, Bodini, Hollender, Lumbroso, arXiv 1508.03167) draws a
 * uniformly random permutation of an array: the array is cut into q = 2^c
 * blocks [n*i/q, n*(i+1)/q), c the least level count with (n >> c) <= cutoff
 * (Algorithm MergeShuffle; shuffle() listing in Appendix A.2); each block is
 * shuffled with Fisher-Yates (Algorithm 1); then for levels L = 1..c each
 * pair of adjacent shuffled blocks is merged by Merge (Algorithm 2, Section
 * 1.1; merge() listing in Appendix A.1): coin flips interleave the two halves
 * until a flip falls on an exhausted half, and the remaining slots are placed
 * by Fisher-Yates insertion.  Lemma 1 shows the result is uniform.
 *
 * Result contract.  Every entry point computes out[t] = in[pi(t)], where pi is
 * the permutation MergeShuffle(n, cutoff, seed) produces under this library's
 * bit source:
 *   - coin flip t of merge m at level L: bit (t & 31) of word (t >> 5) & 3 of
 *     Philox-4x32-10(counter = (t >> 7, m, L, 1 << 28), key = (lo32(seed),
 *     hi32(seed)));
 *   - the d-th bounded draw of unit u (leaf block u at level 0, merge u at
 *     level L >= 1) is a Fast Dice Roller draw [Lumbroso13] whose bits are read
 *     most-significant first from word d & 3 of Philox(d >> 2, u, L, 2 << 28),
 *     then from Philox(d, u, L, (3 << 28) | j), j = 0, 1, ..., words 0..3;
 *   - the coin-flip loop places elements as a stable interleave: output slot
 *     a+b takes A[a] on a 0 flip and B[b] on a 1 flip.
 * pi depends only on (n, cutoff, seed): not on element values, element size,
 * stream, launch shape or batching.
 *
 * Random bits.  The optional device counter d_bits of the _ex entry points is
 * incremented by the number of fair bits the call consumed: P+1 flips per
 * merge (P = slots filled by the coin-flip loop, including the flip that ends
 * it) plus every bit read by the bounded draws -- the cost Lemma 2 and the
 * paper's bit-count table measure.
 *
 * Memory and ownership.  Data pointers are device pointers owned by the
 * caller, aligned to the element size; elements are 4, 8 or 16 bytes; arrays
 * hold n < 2^32 - 2^16 elements.  The library owns per-(device, stream)
 * scratch: one array of n * elem_bytes bytes (the HBM merge levels run
 * out of place between the caller's array and this scratch) and the merge
 * plan (about n/64 bytes plus the tail tables).  Scratch is allocated on first
 * use and grown (after synchronizing that stream) when a larger call needs it;
 * ms_release() frees it.
 *
 * Asynchrony and errors.  Calls validate their arguments, make the scratch,
 * enqueue kernels on `stream` (a hipStream_t; NULL = the default stream) and
 * return.  Argument, allocation and launch errors are returned at once as a
 * negative status; ms_last_error() gives the calling thread's last message.
 * Kernel faults surface at the caller's next synchronization.  The merge plan
 * keeps the insertion-loop tables of every level in capacity-bounded pools
 * sized far above the expected need (the chance that a call exceeds them is
 * below 2^-60); if one ever overflows the call's output is wrong and a flag
 * is set that ms_device_status() reports for the call's stream.  Calls on
 * different streams may run concurrently, also from different host threads
 * (each stream has its own scratch, status word and side streams); calls on
 * one stream run in order.
 */
#ifndef MERGESHUFFLE_H
#define MERGESHUFFLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MS_OK = 0,
  MS_ERR_INVALID = -1,     /* null pointer with n > 0, misaligned pointer, bad cutoff */
  MS_ERR_UNSUPPORTED = -2, /* element size not 4/8/16, n too large, leaf too large */
  MS_ERR_NOMEM = -3,       /* scratch allocation failed */
  MS_ERR_HIP = -4,         /* a HIP runtime call failed (no device, launch error) */
  MS_ERR_CAPACITY = -5     /* ms_device_status: a plan pool overflowed */
};

/* Knobs of the _ex entry points; a NULL config means all defaults.
 * leaf_B changes the permutation (it is the paper's cutoff); the others never do. */
typedef struct ms_config {
  uint32_t leaf_B;          /* cutoff: leaves hold at most leaf_B+1 elements; 0 = 4096; at most 4096 */
  uint32_t levels_per_pass; /* HBM merge levels fused into one pass over the array (each
                               workgroup runs a tile of the top level and, below it, the
                               windows of the lower levels that feed it); 0 = default (3;
                               4 when there are at least 13 HBM levels, for 4-byte elements
                               only if 3 does not divide them); clamped to 1..4; the passes
                               split the levels as evenly as possible */
  uint32_t lds_levels_max;  /* cap on merge levels run in LDS by the leaf kernel; 0 = as many as fit */
  uint32_t flags;           /* MS_CFG_HBM_ONLY: run every merge level as an HBM pass;
                               MS_CFG_ONE_LEVEL_PASSES: one streaming pass plus one patch
                               kernel per HBM level instead of fused passes (levels_per_pass
                               is then ignored);
                               MS_CFG_PLACEMENT_R1: place the elements of each merge's
                               coin-flip loop as the printed Merge listing's in-place swaps do
                               (Appendix A.1 merge() listing; the default places them by the stable
                               interleave).  The same bits, break steps and draws are used and
                               the same B elements land on the same slots; only the order of
                               the A elements differs.  Every level then runs as a one-level
                               HBM pass (implies the two flags above) and the A slots are
                               gathered, so this mode is much slower; it exists to reproduce the
                               listing exactly. */
} ms_config;

#define MS_CFG_HBM_ONLY 1u
#define MS_CFG_ONE_LEVEL_PASSES 2u
#define MS_CFG_PLACEMENT_R1 4u
/* MS_CFG_LEAF_BIG: run the leaves in 128 KiB super-blocks of 1024 threads
 * (the default is 64 KiB and 512 threads): a workgroup shape, the permutation
 * does not depend on it. */
#define MS_CFG_LEAF_BIG 8u
/* MS_CFG_TUNED: take leaf_B, levels_per_pass and MS_CFG_LEAF_BIG from the
 * tuning table entry of the call's (elem_bytes, floor(log2 n)), if there is
 * one (see ms_tune_set); the other fields as given.  The tuned cutoff changes
 * the permutation like any cutoff: ms_leaf_B_for reports it. */
#define MS_CFG_TUNED 16u
/* MS_CFG_PLACEMENT_BALANCED: BalancedShuffle (Section 2): every merge
 * interleaves its two shuffled halves by a uniformly random word of
 * C(n1+n2, n1) -- the side labels that Algorithm 2 leaves when it merges the
 * labels 0^n1 1^n2 (its coin flips up to the break step, the remaining side
 * after it, then its insertion loop applied to the labels), drawn with the
 * same bits, break steps and draws as the default merge -- and slot k takes
 * the next element of the side its label names.  Every merge level runs as a
 * one-level HBM pass (implies MS_CFG_HBM_ONLY and MS_CFG_ONE_LEVEL_PASSES);
 * the plan materializes each level's final labels (one bit per element).
 * Not combinable with MS_CFG_PLACEMENT_R1. */
#define MS_CFG_PLACEMENT_BALANCED 32u

/* Shuffle n elements of elem_bytes bytes at dev_ptr in place (Algorithm
 * MergeShuffle with cutoff 4096), seed as above, on stream. */
int ms_shuffle(void* dev_ptr, uint64_t n, uint32_t elem_bytes, uint64_t seed, void* stream);

/* Write the random permutation of 0..n-1 to the device array out (uint32),
 * i.e. ms_shuffle of the identity, generating the identity in the leaf kernel
 * instead of reading it.  Default stream. */
int ms_permutation(uint32_t* out, uint64_t n, uint64_t seed);

/* Shuffle `count` independent uint32 device arrays ptrs[a] of sizes[a]
 * elements (host arrays of pointers and sizes), array a with seed + a: each
 * array ends exactly as ms_shuffle(ptrs[a], sizes[a], 4, seed + a) leaves it.
 * Arrays must not overlap.  Every argument is checked before anything is
 * launched (errors as for ms_shuffle, naming the array).  Arrays of up to
 * 2^21 elements run in waves on `stream`: per wave, one launch per plan stage,
 * one leaf launch per element size and one launch per fused pass class, all
 * arrays of the wave together (at most 8192 arrays and 4 GiB of scratch per
 * wave: each array's plan tables and array copy; the descriptors pass through
 * two pinned host buffers kept per stream, and the host waits before reusing
 * one until the copy out of it has run).  Larger arrays take the full path on
 * four library streams that wait for `stream` and that `stream` waits for
 * before its next work, so the call is ordered on `stream` like any other;
 * their scratch as for ms_shuffle, on those streams. */
int ms_shuffle_batched(void* const* ptrs, const uint64_t* sizes, uint32_t count, uint64_t seed, void* stream);

/* As above with explicit knobs and an optional device counter (+= bits). */
int ms_shuffle_ex(void* dev_ptr, uint64_t n, uint32_t elem_bytes, uint64_t seed, void* stream,
                  const ms_config* cfg, unsigned long long* d_bits);
int ms_permutation_ex(uint32_t* out, uint64_t n, uint64_t seed, void* stream, const ms_config* cfg,
                      unsigned long long* d_bits);
/* elem_bytes: host array of per-array element sizes, or NULL for all-uint32;
 * d_bits_per_array: device array of count counters, or NULL. */
int ms_shuffle_batched_ex(void* const* ptrs, const uint64_t* sizes, const uint32_t* elem_bytes, uint32_t count,
                          uint64_t seed, void* stream, const ms_config* cfg, unsigned long long* d_bits_per_array);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc): the same
 * result as ms_shuffle_ex with the same arguments, but the library allocates
 * nothing.  Its scratch -- a status word, the array copy and the merge plan --
 * lives in one fixed device array of 64 MiB (MS_NOALLOC_SCRATCH_BYTES) per
 * device, which each device holds until the process ends; a call whose
 * scratch (256 + ms_scratch_bytes, rounded up) exceeds it returns
 * MS_ERR_UNSUPPORTED before launching anything (4-byte arrays up to about
 * 2^23 elements fit).  Every kernel runs on `stream` in order (no side stream,
 * no events).  All calls on one device share the array, which keeps the last
 * call's contents: calls that overlap in time on one device (on different
 * streams or from different host threads) race and give wrong results; calls
 * on one stream are ordered and safe.  Status flags as for ms_shuffle, read by
 * ms_device_status. */
#define MS_NOALLOC_SCRATCH_BYTES (64ull << 20)
int ms_shuffle_noalloc(void* dev_ptr, uint64_t n, uint32_t elem_bytes, uint64_t seed, void* stream,
                       const ms_config* cfg, unsigned long long* d_bits);

/* As ms_shuffle_batched_ex, with an explicit seed per array: array a ends
 * exactly as ms_shuffle_ex(ptrs[a], sizes[a], elem_bytes[a], seeds[a], ...)
 * leaves it (seeds: host array of count seeds).  For callers that batch
 * unrelated requests, such as a serving loop. */
int ms_shuffle_batched_seeds(void* const* ptrs, const uint64_t* sizes, const uint32_t* elem_bytes,
                             const uint64_t* seeds, uint32_t count, void* stream, const ms_config* cfg,
                             unsigned long long* d_bits_per_array);

/* A batched call captured once in a HIP graph and replayed: for callers
 * that shuffle the same set of device arrays again and again (an epoch loop
 * over fixed buffers).  ms_batch_graph_create plans every array (array a with
 * sizes[a] elements of elem_bytes[a] bytes (NULL: 4), seed seeds[a] and the
 * knobs cfgs[a] (NULL: defaults), as ms_shuffle_ex would), allocates the
 * graph's own scratch (every wave's plan tables and array copies, the
 * full-path arrays' plan tables and copies, a status word; about
 * ms_batch_graph_bytes), writes the launch descriptors to the device once and
 * captures the launch sequence of ms_shuffle_batched_seeds into a graph:
 * kernel launches only, no host work and no memset nodes.  Nothing runs at
 * creation.  Each ms_batch_graph_launch then shuffles every array in place on
 * `stream` exactly as ms_shuffle_ex(ptrs[a], sizes[a], elem_bytes[a],
 * seeds[a], stream, &cfgs[a], ...) would (the k-th launch leaves the k-fold
 * permutation), adding the bits to d_bits_per_array (device, count counters,
 * or NULL).  The arrays must stay allocated while the graph lives.  Launches
 * of one graph must not overlap in time (they share its scratch): launch it on
 * one stream, or order the streams.  ms_batch_graph_status synchronizes
 * `stream`, then reads and clears the graph's status word (as
 * ms_device_status).  ms_batch_graph_destroy synchronizes the device and
 * frees everything the graph holds. */
typedef struct ms_batch_graph ms_batch_graph;
int ms_batch_graph_create(void* const* ptrs, const uint64_t* sizes, const uint32_t* elem_bytes,
                          const uint64_t* seeds, uint32_t count, const ms_config* cfgs,
                          unsigned long long* d_bits_per_array, ms_batch_graph** out);
int ms_batch_graph_launch(ms_batch_graph* g, void* stream);
int ms_batch_graph_status(ms_batch_graph* g, void* stream, uint32_t* flags);
uint64_t ms_batch_graph_bytes(const ms_batch_graph* g);
int ms_batch_graph_destroy(ms_batch_graph* g);

/* Plan of one call, computed on the host (no GPU needed). */
typedef struct ms_plan_info {
  uint32_t levels;        /* c */
  uint32_t lds_levels;    /* merge levels done inside the leaf kernel */
  uint32_t hbm_levels;    /* merge levels done as HBM passes */
  uint32_t leaf_B;        /* cutoff used */
  uint64_t leaves;        /* q = 2^c */
  uint64_t scratch_bytes; /* library scratch for this call (array copy + plan) */
  uint64_t pass_tiles;    /* workgroups of one HBM merge pass */
  uint32_t hbm_passes;    /* passes over HBM that run the hbm_levels */
  uint32_t max_levels_per_pass; /* merge levels of the largest such pass */
} ms_plan_info;

int ms_plan(uint64_t n, uint32_t elem_bytes, const ms_config* cfg, ms_plan_info* out);

/* Library scratch a call of this size needs, in bytes (0 if unsupported). */
uint64_t ms_scratch_bytes(uint64_t n, uint32_t elem_bytes);

/* Tuning table (process-wide, all devices): one entry per element size and
 * size bucket [2^log2_n, 2^(log2_n+1)), as an autotuner measured them.
 * ms_tune_set replaces the whole table (count 0 clears it); it returns
 * MS_ERR_INVALID, and keeps the old table, if an entry has an element size
 * other than 4/8/16, log2_n above 32, a cutoff outside 1..4096, more than 4
 * levels per pass or a flag other than MS_CFG_LEAF_BIG.  Calls with
 * MS_CFG_TUNED read it when they are planned. */
typedef struct ms_tune_entry {
  uint32_t elem_bytes;
  uint32_t log2_n;
  uint32_t leaf_B;          /* cutoff */
  uint32_t levels_per_pass; /* 0 = default */
  uint32_t flags;           /* 0 or MS_CFG_LEAF_BIG */
} ms_tune_entry;
int ms_tune_set(const ms_tune_entry* entries, uint32_t count);

/* The cutoff a call of this size with MS_CFG_TUNED uses: the tuning table's
 * entry for its bucket, else the default 4096 (for replaying a call on
 * another implementation, such as a CPU reference). */
uint32_t ms_leaf_B_for(uint64_t n, uint32_t elem_bytes);

/* Synchronize `stream`, then read and clear the status flags of the calls
 * made on `stream` (each stream has its own word; a batched call's large
 * arrays flag the caller's stream's word) and of the allocation-free entry
 * point on the current device (bit 0: target pool overflow, bit 1: tail pool
 * overflow, bit 2: a placement chain of MS_CFG_PLACEMENT_R1 did not descend;
 * bit 3: the leaf kernel found two same-slot list pushes out of step order,
 * i.e. the device did not apply one wave's same-address LDS exchanges in lane
 * order; bits 2 and 3 are internal errors that mean a wrong result).
 * Returns MS_OK if clear, MS_ERR_CAPACITY if a flag was set. */
int ms_device_status(void* stream, uint32_t* flags);

/* Free every scratch buffer, status word and library stream of the current
 * device (synchronizes it; no call may run concurrently). */
int ms_release(void);

/* The calling thread's last error message ("" if none). */
const char* ms_last_error(void);

/* Kernel timing: while enabled, each kernel class launched by the library is
 * bracketed by HIP events on the call's stream.  Classes: 0 plan, 1 leaf,
 * 2 merge pass, 3 patch.  ms_profile_read synchronizes the recorded events,
 * writes total milliseconds and launch counts per class, and clears them. */
int ms_profile_enable(int on);
int ms_profile_read(double ms_per_class[4], uint64_t launches_per_class[4]);

#ifdef __cplusplus
}
#endif

#endif /* MERGESHUFFLE_H */
