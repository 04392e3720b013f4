// ms_plan.hpp -- launch plan shared by the host runtime and the kernels.
//
// MergeShuffle (Algorithm MergeShuffle; shuffle() listing, Appendix A.2)
// splits n elements into q = 2^c blocks [n*i/q, n*(i+1)/q), c the least level
// count with (n >> c) <= cutoff, shuffles each block with Fisher-Yates and
// then merges adjacent blocks for levels L = 1..c.  On the GPU:
//   * the leaf kernel shuffles each leaf in LDS and runs the first `lds_levels`
//     merge levels inside the same workgroup (a super-block of 2^lds_levels
//     leaves fits in LDS);
//   * every remaining level is one streaming pass over HBM, prepared by a
//     data-independent plan: coin-flip counts per 128-flip granule (one
//     Philox block) and per 32768-flip chunk, the break step P of every merge,
//     and the insertion-loop ("tail") resolution into a list of patches.
#pragma once

#include <stdint.h>

namespace ms {

constexpr int kMaxLevels = 32;
constexpr int kBitsParts = 256;        // partial bit counters of the insertion-loop count kernel
constexpr int kGroupMax = 4;           // merge levels fused into one HBM pass, at most
constexpr uint32_t kGranLog = 7;       // 128 flips per granule (one Philox block)
constexpr uint32_t kChunkGranLog = 8;  // 256 granules per chunk
constexpr uint32_t kChunkLog = kGranLog + kChunkGranLog;  // 32768 flips per chunk

// One merge level that runs as an HBM pass.
struct HbmLevel {
  uint32_t L;             // level, 1..c
  uint32_t nmerge;        // q >> L
  uint32_t nmax;          // largest merge size at this level
  uint32_t cpm;           // flip chunks per merge
  uint32_t bpm;           // tail buckets per merge
  uint32_t wpm;           // tail workgroups per merge
  uint32_t tpm;           // merge-pass tiles per merge
  uint32_t group_bottom;  // 1 if this level reads the pass input (first level of its fused pass)
  uint32_t blog;          // target-entry buckets of 2^blog slots (about 2.5 sqrt(N): ~1.6 entries each)
  uint32_t grp;           // fused pass this level belongs to
  uint32_t gli;           // its index within the pass, 0 = the level reading the pass input
  uint32_t mpw;           // merges per tail workgroup: 4 (one to a wave) for small merges, else 1
  uint64_t chunk_base;    // first chunk of this level (ctot, zc); granules at chunk_base << 8
  uint64_t merge_base;    // first merge of this level in the per-merge arrays
  uint64_t bucket_base;   // first bucket of this level
  uint64_t wg_base;       // first workgroup of this level in the tail kernels
};

// One fused pass: levels lev[lf .. lf+lam).  Its top level's merges are cut
// into tiles of T output slots; a tile's "boundary record" holds, for each
// node of the tile's window tree (breadth first, 2^lam - 1 nodes), the
// window's start slot and the rank (zeros before it) at that slot.
constexpr int kBndStride = 2 * ((1 << kGroupMax) - 1);  // u32 per boundary record
struct GroupInfo {
  uint32_t lf, lam;
  uint32_t tpm, T;        // tiles per top merge, slots per tile
  uint64_t bnd_first;     // first boundary record (each top merge has tpm + 1)
};

struct PlanArgs {
  uint64_t n;
  uint32_t c;             // levels
  uint32_t lds_levels;    // levels run inside the leaf kernel
  uint32_t nlev;          // HBM levels: L = lds_levels+1 .. c
  uint32_t placement;     // 0: stable interleave; 1: in-place swaps of the printed Merge listing;
                          // 2: BalancedShuffle (interleave by the final side labels)
  uint32_t key0, key1;    // seed
  uint64_t total_chunks;
  uint64_t total_merges;
  uint64_t total_buckets;
  uint64_t total_tail_wgs;
  uint64_t pool_cap;      // capacity of the target-entry pool (all levels)
  uint64_t tail_cap;      // capacity of the dense per-step tail arrays (all levels)
  // device arrays
  uint16_t* zloc;         // per granule: zeros before it within its chunk
  uint32_t* ctot;         // per chunk: zeros in the chunk
  uint32_t* zc;           // per chunk: zeros before it within its merge
  uint32_t* zg;           // per chunk (+1): zeros before it over all chunks (modulo 2^32)
  uint32_t* P;            // per merge: break step (coin-flip prefix length)
  uint8_t* side;          // per merge: 0 = A ran out first, 1 = B ran out first
  uint32_t* kcnt;         // per merge: insertion steps N - P
  uint32_t* toff;         // per merge (+1): exclusive prefix of kcnt
  uint32_t* lab;          // placement 2: per chunk, 1024 words of final side labels (bit t of a merge)
  uint32_t* tail_src;     // per insertion step i: input offset of slot i's final value, or ~0
  uint32_t* bcnt;         // per bucket: target entries (step i, slot j_i < i)
  uint32_t* bfill;        // per bucket: fill cursor
  uint32_t* boff;         // per bucket (+1): exclusive prefix of bcnt
  uint32_t* part;         // scan partials
  uint32_t* pool_x;       // target entry: merge-relative slot j
  uint32_t* pool_step;    // target entry: the step i that writes C0[i] into slot j
  uint32_t* pool_src;     // target entry: input offset of slot j's final value, or ~0
  uint32_t* tail_xsrc;    // as tail_src, traced down to the input of the fused pass
  uint32_t* pool_xsrc;    // as pool_src, traced down to the input of the fused pass
  uint32_t* bnd;          // boundary records of every fused pass
  uint64_t total_bnd;
  uint32_t* desc;         // tile descriptors of every fused pass
  uint64_t total_desc;    // their words
  unsigned long long* bits;
  unsigned long long* bits_part;  // kBitsParts partial sums of the insertion-loop draws' bits
  uint32_t* status;
  uint32_t ngroup;
  uint32_t pad1;
  HbmLevel lev[kMaxLevels];
  GroupInfo grp[kMaxLevels];
};


// Kernels take PlanArgs by value: it must fit the 4 KiB kernel-argument block.
static_assert(sizeof(PlanArgs) <= 4096, "PlanArgs exceeds the kernel-argument limit");

// Arguments of the data kernels (shared by the host runtime and the kernels).
struct LeafArgs {
  const void* in;
  void* out;
  uint64_t n;
  uint32_t c;
  uint32_t lds_levels;
  uint32_t key0, key1;
  unsigned long long* bits;
  uint32_t* status;  // device status flags (bit 3: list order check)
};

struct PassArgs {
  const void* in;
  void* out;
  uint64_t n;
  uint32_t c, L, tpm, cpm;
  uint64_t chunk_base;  // global chunk of merge 0 of this level
  uint64_t merge_base;  // global merge index of merge 0 of this level
  const uint16_t* zloc;
  const uint32_t* zc;
  const uint32_t* P;
  const uint8_t* side;
  uint32_t key0, key1;
  uint32_t vec_ok;  // base pointer 16-byte aligned
  const uint32_t* lab;  // BalancedShuffle: the level's final side labels (else null: coin flips)
};

struct GroupArgs {
  const void* X;
  void* Z;
  uint64_t n;
  uint32_t c;
  uint32_t tpm;     // tiles per top merge
  uint32_t key0, key1;
  uint32_t vec_ok;  // input and output 16-byte aligned
  uint32_t ntiles;  // tiles of this pass (top merges x tpm)
  const uint32_t* P;
  const uint8_t* side;
  const uint32_t* toff;       // per merge: first insertion step in the dense arrays
  const uint32_t* bnd;        // boundary records of this pass (first one of top merge 0)
  const uint32_t* tail_xsrc;  // per insertion step: pass-input offset of the slot's final value, or ~0
  const uint32_t* boff;       // per bucket (+1): first target entry
  const uint32_t* pool_x;     // target entry: slot
  const uint32_t* pool_xsrc;  // target entry: pass-input offset of the slot's final value, or ~0
  uint64_t tail_cap, pool_cap;
  uint32_t* desc;             // tile descriptors of this pass (built by the plan, read by the pass)
  uint32_t desc_words;        // 32-bit words per tile descriptor
  uint32_t pad2;
  // per level of the pass, bottom first
  uint32_t L[kGroupMax];
  uint32_t blog[kGroupMax];
  uint32_t bpm[kGroupMax];
  uint64_t merge_base[kGroupMax];
  uint64_t bucket_base[kGroupMax];
};

}  // namespace ms
