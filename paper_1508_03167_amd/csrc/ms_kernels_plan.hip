// ms_kernels_plan.hip -- the data-independent plan of the HBM merge levels.
//
// For every merge (L, m) handled by an HBM pass this computes, before any
// element moves:
//   * zeros among the coin flips per 128-flip granule (prefix within its
//     32768-flip chunk) and per chunk (prefix within the merge), so the rank
//     of any slot t -- how many A elements the coin-flip loop placed before
//     t -- is a table lookup plus one Philox block;
//   * the break step P: the loop of Algorithm 2 stops on the first flip whose
//     side is already empty, i.e. at the (n1+1)-th zero or the (n2+1)-th one,
//     whichever comes first; it has consumed P+1 flips (Lemma 1's proof);
//   * the insertion loop (second loop of Algorithm 2): for i = P..N-1 it swaps
//     slot i with a slot drawn uniformly in [0, i].  Its net effect is a small
//     set of slots whose final value comes from another slot of the pre-
//     insertion array C0.  Slots P..N-1 (one per step) are kept densely per
//     merge; every step whose target j differs from i adds a "target entry"
//     (j, i), bucketed by j.  Every slot is then resolved on its own:
//       - slot x < P or x targeted by a later step: the last step i that
//         targets x left C0[i] there;
//       - slot p >= P otherwise holds what slot j_p held just before step p:
//         the last earlier step targeting j_p left C0 of that step, or, if
//         j_p >= P is itself a step before p, what j_p's own step fetched
//         (followed recursively), or else C0[j_p];
//     and is finally mapped to the input offset C0 reads it from.
#include <algorithm>

#include "ms_device.hpp"
#include "ms_plan.hpp"

namespace ms {

// The HBM level whose range of a per-level index (chunk, merge or tail
// workgroup) holds idx: the last level whose first index is <= idx (binary
// search: most indices belong to the lowest levels).
#define MS_LEVEL_OF(name, field)                                         \
  __device__ __forceinline__ int name(const PlanArgs& pa, uint64_t idx) { \
    int lo = 0, hi = (int)pa.nlev - 1;                                    \
    while (lo < hi) {                                                     \
      const int mid = (lo + hi + 1) >> 1;                                 \
      if (pa.lev[mid].field <= idx) lo = mid;                             \
      else hi = mid - 1;                                                  \
    }                                                                     \
    return lo;                                                            \
  }
MS_LEVEL_OF(level_of_chunk, chunk_base)
MS_LEVEL_OF(level_of_merge, merge_base)
MS_LEVEL_OF(level_of_wg, wg_base)
#undef MS_LEVEL_OF

struct MergeGeom {
  uint64_t s;   // first element
  uint32_t n1, n2, N;
};

__device__ __forceinline__ MergeGeom merge_geom(const PlanArgs& pa, uint32_t L, uint32_t m) {
  const uint64_t i0 = (uint64_t)m << L;
  const uint64_t s = bound(pa.n, i0, pa.c);
  const uint64_t mid = bound(pa.n, i0 + (1ull << (L - 1)), pa.c);
  const uint64_t e = bound(pa.n, i0 + (1ull << L), pa.c);
  MergeGeom g;
  g.s = s;
  g.n1 = (uint32_t)(mid - s);
  g.n2 = (uint32_t)(e - mid);
  g.N = (uint32_t)(e - s);
  return g;
}

// ---------------------------------------------------------------------------
// 1. zeros per granule and per chunk
// ---------------------------------------------------------------------------
__device__ __forceinline__ void plan_count_body(const PlanArgs& pa, uint64_t chunk, uint32_t* tmp) {
  const int l = level_of_chunk(pa, chunk);
  const HbmLevel& lv = pa.lev[l];
  // chunks of one level number fewer than 2^32: a 32-bit division
  const uint32_t rel = (uint32_t)(chunk - lv.chunk_base);
  const uint32_t m = rel / lv.cpm;
  const uint32_t ch = rel - m * lv.cpm;
  const Key key{pa.key0, pa.key1};
  const uint32_t g = (ch << kChunkGranLog) + threadIdx.x;
  const W4 f = flip_block(g, m, lv.L, key);
  const uint32_t z = 128u - (uint32_t)(__popc(f.w[0]) + __popc(f.w[1]) + __popc(f.w[2]) + __popc(f.w[3]));
  uint32_t total;
  const uint32_t ex = block_excl_scan<256>(z, tmp, &total);
  pa.zloc[(chunk << kChunkGranLog) + threadIdx.x] = (uint16_t)ex;
  if (threadIdx.x == 0) pa.ctot[chunk] = total;
}
// The same, one wave per chunk (4 granules per lane, a wave scan, no
// barrier), kCountChunksPerWave chunks per wave one after the other: a
// workgroup per chunk spent more on starting workgroups than on the flips.
constexpr uint32_t kCountChunksPerWave = 4;
__global__ void __launch_bounds__(256) plan_count_kernel(PlanArgs pa) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t c0 = ((uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * kCountChunksPerWave;
  const uint64_t c1 = min(c0 + kCountChunksPerWave, pa.total_chunks);
  const Key key{pa.key0, pa.key1};
  for (uint64_t chunk = c0; chunk < c1; ++chunk) {
    const int l = level_of_chunk(pa, chunk);
    const HbmLevel& lv = pa.lev[l];
    const uint32_t rel = (uint32_t)(chunk - lv.chunk_base);
    const uint32_t m = rel / lv.cpm;
    const uint32_t ch = rel - m * lv.cpm;
    const uint32_t g0 = (ch << kChunkGranLog) + 4u * lane;
    uint32_t z[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const W4 f = flip_block(g0 + (uint32_t)e, m, lv.L, key);
      z[e] = 128u - (uint32_t)(__popc(f.w[0]) + __popc(f.w[1]) + __popc(f.w[2]) + __popc(f.w[3]));
    }
    const uint32_t sum = z[0] + z[1] + z[2] + z[3];
    const uint32_t incl = wave_incl_scan(sum);
    const uint32_t ex = incl - sum;
    // four 16-bit prefixes, as two 32-bit words
    uint32_t* zl = reinterpret_cast<uint32_t*>(pa.zloc + (chunk << kChunkGranLog) + 4u * lane);
    zl[0] = (ex & 0xFFFFu) | ((ex + z[0]) << 16);
    zl[1] = ((ex + z[0] + z[1]) & 0xFFFFu) | ((ex + z[0] + z[1] + z[2]) << 16);
    if (lane == 63) pa.ctot[chunk] = incl;
  }
}

// Position (0..127) of the r-th zero (want_one = 0) or one (want_one = 1) of a block.
__device__ int select_in_block(const W4& f, uint32_t r, int want_one) {
  for (int w = 0; w < 4; ++w) {
    const uint32_t word = want_one ? f.w[w] : ~f.w[w];
    const uint32_t c = (uint32_t)__popc(word);
    if (r < c) return 32 * w + select_one(word, (int)r);
    r -= c;
  }
  return 128;  // not reached for a valid r
}

// Slot of the (target+1)-th zero (want_one = 0) or one in chunk ch of merge m.
__device__ __forceinline__ uint32_t locate_in_chunk(const PlanArgs& pa, uint64_t chunk_global, uint32_t ch, uint32_t m,
                                    uint32_t L, uint32_t r, int want_one) {
  const uint16_t* zl = pa.zloc + (chunk_global << kChunkGranLog);
  // largest granule g with (zeros or ones before g) <= r
  int lo = 0, hi = 255;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const uint32_t before = want_one ? ((uint32_t)mid << kGranLog) - zl[mid] : zl[mid];
    if (before <= r) lo = mid; else hi = mid - 1;
  }
  const uint32_t before = want_one ? ((uint32_t)lo << kGranLog) - zl[lo] : zl[lo];
  const uint32_t gi = (ch << kChunkGranLog) + (uint32_t)lo;
  const W4 f = flip_block(gi, m, L, Key{pa.key0, pa.key1});
  const int pos = select_in_block(f, r - before, want_one);
  return (gi << kGranLog) + (uint32_t)pos;
}

// ---------------------------------------------------------------------------
// 2. per merge: chunk prefix, break step P and the side that ran out
// ---------------------------------------------------------------------------
// zc of every chunk from the global prefix of chunk zero counts (sums wrap
// modulo 2^32, but every merge's own prefix stays below 2^32)
// (and clears the bucket counters for the insertion-loop kernels)
__device__ __forceinline__ void zc_body(const PlanArgs& pa, uint64_t c) {
  if (c < (uint64_t)kBitsParts) pa.bits_part[c] = 0;
  if (c < pa.total_buckets) {
    pa.bcnt[c] = 0;
    pa.bfill[c] = 0;
  }
  if (c >= pa.total_chunks) return;
  const HbmLevel& lv = pa.lev[level_of_chunk(pa, c)];
  const uint64_t first = c - (uint32_t)(c - lv.chunk_base) % lv.cpm;
  pa.zc[c] = pa.zg[c] - pa.zg[first];
}
__global__ void __launch_bounds__(256) zc_kernel(PlanArgs pa) { zc_body(pa, (uint64_t)blockIdx.x * 256 + threadIdx.x); }

// ---------------------------------------------------------------------------
// BalancedShuffle (Section 2): the word of each merge is the side labels
// Algorithm 2 leaves when it merges 0^n1 1^n2 -- label t is coin flip t for
// t < P, the side that is left for t >= P (B if A ran out, else A), and
// then the insertion loop permutes the labels as it permutes elements.  The
// plan writes those labels (one bit per slot, at the slot's chunk and bit
// position), lets the insertion-loop resolution overwrite the slots it
// moves, and counts the zeros again; the pass reads the labels.
// ---------------------------------------------------------------------------
// The label of slot x before the insertion loop.
__device__ __forceinline__ uint32_t bal_label0(const PlanArgs& pa, uint32_t L, uint32_t m, uint32_t P,
                                               uint32_t side, uint32_t x) {
  if (x >= P) return side == 0 ? 1u : 0u;
  const W4 f = flip_block(x >> kGranLog, m, L, Key{pa.key0, pa.key1});
  return (pick(f, (x >> 5) & 3) >> (x & 31)) & 1u;
}

// Word of slot t of merge m (level lv) in the label array.
__device__ __forceinline__ uint64_t bal_word(const HbmLevel& lv, uint32_t m, uint32_t t) {
  return ((lv.chunk_base + (uint64_t)m * lv.cpm + (t >> kChunkLog)) << 10) + ((t >> 5) & 1023u);
}

__device__ __forceinline__ void bal_set(const PlanArgs& pa, const HbmLevel& lv, uint32_t m, uint32_t t, uint32_t v) {
  uint32_t* w = pa.lab + bal_word(lv, m, t);
  const uint32_t bit = 1u << (t & 31);
  if (v) atomicOr(w, bit);
  else atomicAnd(w, ~bit);
}

// One workgroup per chunk: the labels before the insertion loop.
__global__ void __launch_bounds__(256) bal_words_kernel(PlanArgs pa) {
  const uint64_t chunk = blockIdx.x;
  const HbmLevel& lv = pa.lev[level_of_chunk(pa, chunk)];
  const uint32_t rel = (uint32_t)(chunk - lv.chunk_base);
  const uint32_t m = rel / lv.cpm;
  const uint32_t ch = rel - m * lv.cpm;
  const uint64_t gm = lv.merge_base + m;
  const uint32_t P = pa.P[gm];
  const uint32_t fill = pa.side[gm] == 0 ? ~0u : 0u;
  const uint32_t g = (ch << kChunkGranLog) + threadIdx.x;
  const W4 f = flip_block(g, m, lv.L, Key{pa.key0, pa.key1});
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t t0 = (g << kGranLog) + 32u * k;  // slot of bit 0
    uint32_t w = f.w[k];
    if (t0 + 32 > P) {
      const uint32_t keep = P > t0 ? (1u << (P - t0)) - 1u : 0u;  // bits below P
      w = (w & keep) | (fill & ~keep);
    }
    pa.lab[(chunk << 10) + 4u * threadIdx.x + k] = w;
  }
}

// Zeros per granule and per chunk of the final labels.
__global__ void __launch_bounds__(256) bal_count_kernel(PlanArgs pa) {
  __shared__ uint32_t tmp[8];
  const uint64_t chunk = blockIdx.x;
  const uint32_t* w = pa.lab + (chunk << 10) + 4u * threadIdx.x;
  const uint32_t z = 128u - (uint32_t)(__popc(w[0]) + __popc(w[1]) + __popc(w[2]) + __popc(w[3]));
  uint32_t total;
  const uint32_t ex = block_excl_scan<256>(z, tmp, &total);
  pa.zloc[(chunk << kChunkGranLog) + threadIdx.x] = (uint16_t)ex;
  if (threadIdx.x == 0) pa.ctot[chunk] = total;
}

__global__ void __launch_bounds__(256) bal_zc_kernel(PlanArgs pa) {
  const uint64_t c = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= pa.total_chunks) return;
  const HbmLevel& lv = pa.lev[level_of_chunk(pa, c)];
  const uint64_t first = c - (uint32_t)(c - lv.chunk_base) % lv.cpm;
  pa.zc[c] = pa.zg[c] - pa.zg[first];
}

// Per merge (one thread each): the chunk holding the (n1+1)-th zero and the
// one holding the (n2+1)-th one by binary search over the chunk prefixes,
// the flip inside it, and so the break step P and the side that ran out.
__device__ __forceinline__ uint64_t break_body(const PlanArgs& pa, uint64_t gm) {
  uint64_t used = 0;
  if (gm < pa.total_merges) {
    const int l = level_of_merge(pa, gm);
    const HbmLevel& lv = pa.lev[l];
    const uint32_t m = (uint32_t)(gm - lv.merge_base);
    const MergeGeom g = merge_geom(pa, lv.L, m);
    const uint64_t cb = lv.chunk_base + (uint64_t)m * lv.cpm;
    uint32_t lo = 0, hi = lv.cpm - 1;
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (pa.zc[cb + mid] <= g.n1) lo = mid; else hi = mid - 1;
    }
    uint32_t resA = kNone32;
    {
      const uint32_t z0 = pa.zc[cb + lo];
      if (z0 <= g.n1 && g.n1 < z0 + pa.ctot[cb + lo]) resA = locate_in_chunk(pa, cb + lo, lo, m, lv.L, g.n1 - z0, 0);
    }
    lo = 0;
    hi = lv.cpm - 1;
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (((uint64_t)mid << kChunkLog) - pa.zc[cb + mid] <= g.n2) lo = mid; else hi = mid - 1;
    }
    uint32_t resB = kNone32;
    {
      const uint64_t o0 = ((uint64_t)lo << kChunkLog) - pa.zc[cb + lo];
      const uint64_t ov = (1ull << kChunkLog) - pa.ctot[cb + lo];
      if (o0 <= g.n2 && g.n2 < o0 + ov) resB = locate_in_chunk(pa, cb + lo, lo, m, lv.L, (uint32_t)(g.n2 - o0), 1);
    }
    const uint32_t P = resA < resB ? resA : resB;
    pa.P[gm] = P;
    pa.side[gm] = resA < resB ? 0 : 1;
    pa.kcnt[gm] = g.N - P;
    used = (uint64_t)P + 1;
  }
  return used;
}
__global__ void __launch_bounds__(256) plan_break_kernel(PlanArgs pa) {
  __shared__ uint64_t red[4];
  const uint64_t used = break_body(pa, (uint64_t)blockIdx.x * 256 + threadIdx.x);
  const uint64_t t = block_sum_u64<256>(used, red);
  if (threadIdx.x == 0 && t) atomicAdd(pa.bits, (unsigned long long)t);
}

__device__ __forceinline__ uint32_t tail_draw(const PlanArgs& pa, uint32_t L, uint32_t m, uint32_t i,
                                              uint32_t* bits) {
  const Key key{pa.key0, pa.key1};
  const W4 db = draw_block(i >> 2, m, L, key);
  const Draw r = fdr_draw((uint64_t)i + 1, pick(db, i & 3), L, m, i, key);
  *bits += r.bits;
  return r.v;
}

// A tail workgroup's share of one merge: its part w of the merge's wpm parts,
// worked by `lanes` threads (the workgroup, or one wave when the level puts
// one merge on each wave); `act` is false for a wave past the level's last
// merge (its k is 0 and it reads the last merge's fields).
struct TailWg {
  const HbmLevel* lv;
  int l;
  uint32_t m, w, lanes, lane;
  bool act;
  MergeGeom g;
  uint32_t P, k;
  uint64_t gm, bb;
};

__device__ __forceinline__ TailWg tail_wg(const PlanArgs& pa, uint64_t wg) {
  TailWg t;
  const int l = level_of_wg(pa, wg);
  t.l = l;
  t.lv = &pa.lev[l];
  // workgroups of one level number fewer than 2^32: a 32-bit division
  const uint32_t rel = (uint32_t)(wg - t.lv->wg_base);
  if (t.lv->mpw > 1) {
    t.m = rel * t.lv->mpw + (threadIdx.x >> 6);
    t.w = 0;
    t.lanes = 64;
    t.lane = threadIdx.x & 63;
  } else {
    t.m = rel / t.lv->wpm;
    t.w = rel - t.m * t.lv->wpm;
    t.lanes = 256;
    t.lane = threadIdx.x;
  }
  t.act = t.m < t.lv->nmerge;
  if (!t.act) t.m = t.lv->nmerge - 1;
  t.g = merge_geom(pa, t.lv->L, t.m);
  t.gm = t.lv->merge_base + t.m;
  t.P = pa.P[t.gm];
  t.k = t.act ? t.g.N - t.P : 0u;
  t.bb = t.lv->bucket_base + (uint64_t)t.m * t.lv->bpm;
  return t;
}

// ---------------------------------------------------------------------------
// 3. insertion-loop draws: count target entries per bucket (and the bits)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void tail_count_body(const PlanArgs& pa, uint64_t wg, uint64_t* red) {
  const TailWg t = tail_wg(pa, wg);
  uint32_t bits = 0;
  for (uint32_t d = t.w * t.lanes + t.lane; d < t.k; d += t.lv->wpm * t.lanes) {
    const uint32_t i = t.P + d;
    const uint32_t j = tail_draw(pa, t.lv->L, t.m, i, &bits);
    if (j != i) atomicAdd(&pa.bcnt[t.bb + (j >> t.lv->blog)], 1u);
  }
  // one of kBitsParts partial counters: tens of thousands of workgroups
  // adding to one address would serialize on it
  const uint64_t s = block_sum_u64<256>(bits, red);
  if (threadIdx.x == 0 && s) atomicAdd(&pa.bits_part[wg % kBitsParts], (unsigned long long)s);
}
__global__ void __launch_bounds__(256) tail_count_kernel(PlanArgs pa) {
  __shared__ uint64_t red[4];
  tail_count_body(pa, blockIdx.x, red);
}

// ---------------------------------------------------------------------------
// 4. exclusive scans (3 phases): counts -> offsets, total at out[count]
// ---------------------------------------------------------------------------
constexpr int kScanPer = 2048;  // items per workgroup

__global__ void __launch_bounds__(256) scan_reduce_kernel(const uint32_t* __restrict__ in, uint64_t count,
                                                          uint32_t* __restrict__ part) {
  __shared__ uint32_t tmp[8];
  const uint64_t base = (uint64_t)blockIdx.x * kScanPer;
  uint32_t s = 0;
  for (int k = 0; k < kScanPer / 256; ++k) {
    const uint64_t i = base + (uint64_t)k * 256 + threadIdx.x;
    if (i < count) s += in[i];
  }
  uint32_t tot;
  block_excl_scan<256>(s, tmp, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(1024) scan_top_kernel(uint32_t* part, uint32_t nparts, uint32_t* out_end,
                                                        uint64_t cap, uint32_t* status, uint32_t flag) {
  __shared__ uint32_t tmp[20];
  uint32_t running = 0;
  for (uint32_t b = 0; b < nparts; b += 1024) {
    const uint32_t idx = b + threadIdx.x;
    const uint32_t v = idx < nparts ? part[idx] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan<1024>(v, tmp, &tot);
    if (idx < nparts) part[idx] = running + ex;
    running += tot;
  }
  if (threadIdx.x == 0) {
    *out_end = running;
    if ((uint64_t)running > cap) atomicOr(status, flag);
  }
}

__global__ void __launch_bounds__(256) scan_down_kernel(const uint32_t* __restrict__ in, uint64_t count,
                                                        const uint32_t* __restrict__ part,
                                                        uint32_t* __restrict__ out) {
  __shared__ uint32_t tmp[8];
  constexpr int kPer = kScanPer / 256;
  const uint64_t base = (uint64_t)blockIdx.x * kScanPer + (uint64_t)threadIdx.x * kPer;
  uint32_t v[kPer];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    v[k] = base + k < count ? in[base + k] : 0u;
    s += v[k];
  }
  const uint32_t ex = block_excl_scan<256>(s, tmp, nullptr);
  uint32_t run = part[blockIdx.x] + ex;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    if (base + k < count) out[base + k] = run;
    run += v[k];
  }
}

// The same scan by one workgroup, for short arrays (one launch instead of three).
constexpr uint64_t kScanOneMax = 65536;
template <int NT>
__device__ __forceinline__ void block_scan_all(const uint32_t* __restrict__ in, uint64_t count,
                                               uint32_t* __restrict__ out, uint64_t cap, uint32_t* status,
                                               uint32_t flag, uint32_t* tmp) {
  constexpr int K = 8;
  uint32_t running = 0;
  for (uint64_t b0 = 0; b0 < count; b0 += NT * K) {
    const uint64_t base = b0 + (uint64_t)threadIdx.x * K;
    uint32_t v[K];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      v[k] = base + k < count ? in[base + k] : 0u;
      sum += v[k];
    }
    uint32_t tot;
    uint32_t run = running + block_excl_scan<NT>(sum, tmp, &tot);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (base + k < count) out[base + k] = run;
      run += v[k];
    }
    running += tot;
  }
  if (threadIdx.x == 0) {
    out[count] = running;
    if ((uint64_t)running > cap) atomicOr(status, flag);
  }
}
__global__ void __launch_bounds__(1024) scan_one_kernel(const uint32_t* __restrict__ in, uint64_t count,
                                                        uint32_t* __restrict__ out, uint64_t cap, uint32_t* status,
                                                        uint32_t flag) {
  __shared__ uint32_t tmp[20];
  block_scan_all<1024>(in, count, out, cap, status, flag, tmp);
}

static void launch_scan(const uint32_t* in, uint64_t count, uint32_t* part, uint32_t* out, uint64_t cap,
                        uint32_t* status, uint32_t flag, hipStream_t st) {
  if (count <= kScanOneMax) {
    hipLaunchKernelGGL(scan_one_kernel, dim3(1), dim3(1024), 0, st, in, count, out, cap, status, flag);
    return;
  }
  const uint32_t nparts = (uint32_t)((count + kScanPer - 1) / kScanPer);
  hipLaunchKernelGGL(scan_reduce_kernel, dim3(nparts), dim3(256), 0, st, in, count, part);
  hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(1024), 0, st, part, nparts, out + count, cap, status, flag);
  hipLaunchKernelGGL(scan_down_kernel, dim3(nparts), dim3(256), 0, st, in, count, part, out);
}

// ---------------------------------------------------------------------------
// 5. insertion-loop draws again: scatter the target entries into buckets
// ---------------------------------------------------------------------------
__device__ __forceinline__ void tail_scatter_body(const PlanArgs& pa, uint64_t wg, uint64_t* red) {
  if (wg == 0) {
    // the count kernel's partial bit counters, added once
    static_assert(kBitsParts == 256, "one counter per thread");
    const uint64_t s = block_sum_u64<256>(pa.bits_part[threadIdx.x], red);
    if (threadIdx.x == 0 && s) atomicAdd(pa.bits, (unsigned long long)s);
  }
  const TailWg t = tail_wg(pa, wg);
  uint32_t bits = 0;
  for (uint32_t d = t.w * t.lanes + t.lane; d < t.k; d += t.lv->wpm * t.lanes) {
    const uint32_t i = t.P + d;
    const uint32_t j = tail_draw(pa, t.lv->L, t.m, i, &bits);
    if (j == i) continue;
    const uint64_t b = t.bb + (j >> t.lv->blog);
    const uint64_t slot = (uint64_t)pa.boff[b] + atomicAdd(&pa.bfill[b], 1u);
    if (slot < pa.pool_cap) {
      pa.pool_x[slot] = j;
      pa.pool_step[slot] = i;
    }
  }
}
__global__ void __launch_bounds__(256) tail_scatter_kernel(PlanArgs pa) {
  __shared__ uint64_t red[4];
  tail_scatter_body(pa, blockIdx.x, red);
}

// Largest step s' < below among the steps that target slot y (y's own step excluded).
__device__ __forceinline__ uint32_t max_target(const PlanArgs& pa, uint64_t bb, uint32_t blog, uint32_t y,
                                               uint32_t below) {
  const uint64_t b = bb + (y >> blog);
  const uint64_t lo = pa.boff[b];
  uint64_t hi = lo + pa.bcnt[b];
  if (hi > pa.pool_cap) hi = pa.pool_cap;
  uint32_t best = kNone32;
  for (uint64_t e = lo; e < hi; ++e) {
    const uint32_t x = pa.pool_x[e];
    const uint32_t st = pa.pool_step[e];
    if (x == y && st < below && (best == kNone32 || st > best)) best = st;
  }
  return best;
}

// The printed Merge listing's placement (in-place swaps).  A one at step t
// swaps slot t with slot n1 + (ones before t), the next B element; a zero
// leaves slot t alone.  So a slot p >= n1, once its B element has left, holds
// what slot t_{p-n1} held at that swap (t_r = step of the r-th one, r from
// 0), and the element a zero at step t keeps, or that slot t >= P holds at
// the break when B ran out, is A[f(t)]: f(q) = q for q < n1, else
// f(t_{q-n1}), with t_{q-n1} < q.  Everything else (the B slots, the break,
// the insertion loop) is the same as for the stable interleave.

// Step of the r-th one flip (r from 0) of merge m of level lv.
__device__ __forceinline__ uint32_t nth_one(const PlanArgs& pa, const HbmLevel& lv, uint32_t m, uint32_t r) {
  const uint64_t cb = lv.chunk_base + (uint64_t)m * lv.cpm;
  uint32_t lo = 0, hi = lv.cpm - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (((uint64_t)mid << kChunkLog) - pa.zc[cb + mid] <= r) lo = mid;
    else hi = mid - 1;
  }
  const uint32_t o0 = (uint32_t)(((uint64_t)lo << kChunkLog) - pa.zc[cb + lo]);
  return locate_in_chunk(pa, cb + lo, lo, m, lv.L, r - o0, 1);
}

// f(q) above.  Every step lowers q; a step that would not (only a broken
// plan could give one) sets status bit 2 and ends the chain.
__device__ __forceinline__ uint32_t r1_a_source(const PlanArgs& pa, const HbmLevel& lv, uint32_t m, uint32_t n1,
                                                uint32_t q) {
  while (q >= n1) {
    const uint32_t nq = nth_one(pa, lv, m, q - n1);
    if (nq >= q) {
      atomicOr(pa.status, 4u);
      return 0u;
    }
    q = nq;
  }
  return q;
}

// Merge-relative input offset of C0[src] (the array before the insertion
// loop); z0 = zeros of the merge before src's granule when src < P.
__device__ __forceinline__ uint32_t c0_offset_z(const PlanArgs& pa, const HbmLevel& lv, uint32_t m,
                                                const MergeGeom& g, uint32_t P, uint32_t side, uint32_t src,
                                                uint32_t z0) {
  if (src >= P) {
    if (side == 0) return src;
    return pa.placement ? r1_a_source(pa, lv, m, g.n1, src) : src - g.n2;
  }
  const uint32_t gi = src >> kGranLog;
  const W4 f = flip_block(gi, m, lv.L, Key{pa.key0, pa.key1});
  const uint32_t wsel = (src >> 5) & 3;
  uint32_t z = z0;
  for (uint32_t w = 0; w < wsel; ++w) z += 32u - (uint32_t)__popc(f.w[w]);
  const uint32_t word = pick(f, wsel);
  const uint32_t bit = src & 31;
  z += (uint32_t)__popc(~word & ((1u << bit) - 1u));
  if ((word >> bit) & 1u) return g.n1 + (src - z);
  return pa.placement ? r1_a_source(pa, lv, m, g.n1, src) : z;
}

// The same, reading the granule's zero count from the plan tables.
__device__ __forceinline__ uint32_t c0_offset(const PlanArgs& pa, const HbmLevel& lv, uint32_t m,
                                              const MergeGeom& g, uint32_t P, uint32_t side, uint32_t src) {
  uint32_t z0 = 0;
  if (src < P) {
    const uint64_t cglob = lv.chunk_base + (uint64_t)m * lv.cpm + (src >> kChunkLog);
    z0 = pa.zc[cglob] + pa.zloc[(cglob << kChunkGranLog) + ((src >> kGranLog) & 255)];
  }
  return c0_offset_z(pa, lv, m, g, P, side, src, z0);
}

// ---------------------------------------------------------------------------
// 6. resolve every touched slot: where its final value comes from
// ---------------------------------------------------------------------------
__device__ __forceinline__ void tail_resolve_body(const PlanArgs& pa, uint64_t wg) {
  const TailWg t = tail_wg(pa, wg);
  const HbmLevel& lv = *t.lv;
  const uint32_t side = pa.side[t.gm];
  const uint64_t toff = pa.toff[t.gm];
  // slots P..N-1, one per step
  for (uint32_t d = t.w * t.lanes + t.lane; d < t.k; d += lv.wpm * t.lanes) {
    const uint32_t x = t.P + d;
    uint32_t out = kNone32;
    if (max_target(pa, t.bb, lv.blog, x, kNone32) == kNone32) {
      // no later step targets x: it keeps what its own step fetched from j_x
      uint32_t dummy = 0;
      uint32_t s = x;
      uint32_t y = tail_draw(pa, lv.L, t.m, x, &dummy);
      uint32_t src;
      for (;;) {
        const uint32_t q = max_target(pa, t.bb, lv.blog, y, s);
        if (q != kNone32) { src = q; break; }      // last earlier step writing y
        if (y >= t.P && y < s) {                   // y's own step wrote it
          s = y;
          y = tail_draw(pa, lv.L, t.m, y, &dummy);
          continue;
        }
        src = y;                                   // untouched since C0
        break;
      }
      if (pa.placement == 2) bal_set(pa, lv, t.m, x, bal_label0(pa, lv.L, t.m, t.P, side, src));
      else out = c0_offset(pa, lv, t.m, t.g, t.P, side, src);
    }
    if (toff + d < pa.tail_cap) pa.tail_src[toff + d] = out;
  }
  // target entries: final if theirs is the last step targeting the slot
  const uint64_t lo = pa.boff[t.bb];
  uint64_t hi = t.act ? pa.boff[t.bb + lv.bpm] : lo;
  if (hi > pa.pool_cap) hi = pa.pool_cap;
  for (uint64_t e = lo + (uint64_t)t.w * t.lanes + t.lane; e < hi; e += (uint64_t)lv.wpm * t.lanes) {
    const uint32_t x = pa.pool_x[e];
    const uint32_t st = pa.pool_step[e];
    uint32_t out = kNone32;
    if (max_target(pa, t.bb, lv.blog, x, kNone32) == st) {
      if (pa.placement == 2) bal_set(pa, lv, t.m, x, bal_label0(pa, lv.L, t.m, t.P, side, st));
      else out = c0_offset(pa, lv, t.m, t.g, t.P, side, st);
    }
    pa.pool_src[e] = out;
  }
}
__global__ void __launch_bounds__(256) tail_resolve_kernel(PlanArgs pa) { tail_resolve_body(pa, blockIdx.x); }

// ---------------------------------------------------------------------------
// 7. trace every resolved source down to the input of its fused pass
// ---------------------------------------------------------------------------
// The source of slot pos's final value at level lev[l], merge m, as an offset
// into the output of the level below (relative to the merge's first element).
// (every table read the three cases may need is issued first, together:
// the merge's break and side, pos's bucket range and granule counts; then
// the bucket's first entries and pos's tail slot)
__device__ __forceinline__ uint32_t final_source(const PlanArgs& pa, int l, uint32_t m, uint32_t pos) {
  const HbmLevel& lv = pa.lev[l];
  const uint64_t gm = lv.merge_base + m;
  const MergeGeom g = merge_geom(pa, lv.L, m);
  const uint64_t b = lv.bucket_base + (uint64_t)m * lv.bpm + (pos >> lv.blog);
  const uint64_t cglob = lv.chunk_base + (uint64_t)m * lv.cpm + (pos >> kChunkLog);
  const uint32_t P = pa.P[gm];
  const uint32_t side = pa.side[gm];
  const uint64_t toff = pa.toff[gm];
  const uint64_t lo = pa.boff[b];
  const uint32_t cnt = pa.bcnt[b];
  const uint32_t z0 = pa.zc[cglob] + pa.zloc[(cglob << kChunkGranLog) + ((pos >> kGranLog) & 255)];
  uint64_t hi = lo + cnt;
  if (hi > pa.pool_cap) hi = pa.pool_cap;
  for (uint64_t e = lo; e < hi; ++e)
    if (pa.pool_x[e] == pos && pa.pool_src[e] != kNone32) return pa.pool_src[e];
  if (pos >= P) {
    const uint64_t t = toff + (pos - P);
    if (t < pa.tail_cap && pa.tail_src[t] != kNone32) return pa.tail_src[t];
  }
  return c0_offset_z(pa, lv, m, g, P, side, pos, z0);
}

__device__ __forceinline__ uint32_t trace_to_input(const PlanArgs& pa, int l, uint32_t m, uint32_t off) {
  if (off == kNone32) return kNone32;
  const uint64_t s0 = merge_geom(pa, pa.lev[l].L, m).s;
  uint64_t abs = s0 + off;
  while (!pa.lev[l].group_bottom) {
    const MergeGeom g = merge_geom(pa, pa.lev[l].L, m);
    const uint32_t child = abs < g.s + g.n1 ? 2 * m : 2 * m + 1;
    l -= 1;
    const uint64_t cs = merge_geom(pa, pa.lev[l].L, child).s;
    abs = cs + final_source(pa, l, child, (uint32_t)(abs - cs));
    m = child;
  }
  return (uint32_t)(abs - s0);
}

__device__ __forceinline__ void trace_body(const PlanArgs& pa, uint64_t wg) {
  const TailWg t = tail_wg(pa, wg);
  const int l = t.l;
  const uint64_t toff = pa.toff[t.gm];
  for (uint32_t d = t.w * t.lanes + t.lane; d < t.k; d += t.lv->wpm * t.lanes) {
    if (toff + d >= pa.tail_cap) break;
    pa.tail_xsrc[toff + d] = trace_to_input(pa, l, t.m, pa.tail_src[toff + d]);
  }
  const uint64_t lo = pa.boff[t.bb];
  uint64_t hi = t.act ? pa.boff[t.bb + t.lv->bpm] : lo;
  if (hi > pa.pool_cap) hi = pa.pool_cap;
  for (uint64_t e = lo + (uint64_t)t.w * t.lanes + t.lane; e < hi; e += (uint64_t)t.lv->wpm * t.lanes)
    pa.pool_xsrc[e] = trace_to_input(pa, l, t.m, pa.pool_src[e]);
}

// ---------------------------------------------------------------------------
// 8. fused passes: boundary records of every tile
// ---------------------------------------------------------------------------
// Slots the coin-flip loop of merge m (level lev[l]) filled from A before slot u.
__device__ __forceinline__ uint32_t rank_at(const PlanArgs& pa, int l, uint32_t m, uint32_t u) {
  const HbmLevel& lv = pa.lev[l];
  const uint64_t gm = lv.merge_base + m;
  const uint32_t P = pa.P[gm];
  if (u >= P) {
    const MergeGeom g = merge_geom(pa, lv.L, m);
    return pa.side[gm] == 0 ? g.n1 : u - g.n2;
  }
  const uint64_t cg = lv.chunk_base + (uint64_t)m * lv.cpm + (u >> kChunkLog);
  uint32_t z = pa.zc[cg] + pa.zloc[(cg << kChunkGranLog) + ((u >> kGranLog) & 255)];
  if (u & 127u) {
    const W4 f = flip_block(u >> kGranLog, m, lv.L, Key{pa.key0, pa.key1});
    const uint32_t wsel = (u >> 5) & 3;
    for (uint32_t w = 0; w < wsel; ++w) z += 32u - (uint32_t)__popc(pick(f, w));
    z += (uint32_t)__popc(~pick(f, wsel) & ((1u << (u & 31)) - 1u));
  }
  return z;
}

// One thread per boundary record: the window tree at slot b*T of top merge M
// (node 0 = the top window's start; a node's children start at its rank in
// the left half and at its slot minus its rank in the right half).
__device__ __forceinline__ void bounds_body(const PlanArgs& pa, uint64_t idx) {
  if (idx >= pa.total_bnd) return;
  int g = (int)pa.ngroup - 1;
  while (g > 0 && pa.grp[g].bnd_first > idx) --g;
  const GroupInfo& gi = pa.grp[g];
  const uint64_t local = idx - gi.bnd_first;
  const uint32_t M = (uint32_t)(local / (gi.tpm + 1));
  const uint32_t b = (uint32_t)(local % (gi.tpm + 1));
  const int lt = (int)(gi.lf + gi.lam - 1);
  const MergeGeom gt = merge_geom(pa, pa.lev[lt].L, M);
  const int nodes = (1 << gi.lam) - 1;
  constexpr int KN = (1 << kGroupMax) - 1;
  uint32_t u[KN], ra[KN];
  u[0] = (uint32_t)min((uint64_t)b * gi.T, (uint64_t)gt.N);
#pragma unroll
  for (int k = 0; k < KN; ++k) {
    if (k < nodes) {
      const int d = 31 - __clz(k + 1);
      const int l = lt - d;
      const uint32_t m = (M << d) + (uint32_t)(k - ((1 << d) - 1));
      ra[k] = rank_at(pa, l, m, u[k]);
      if (2 * k + 2 < KN && 2 * k + 2 < nodes) {
        u[2 * k + 1] = ra[k];
        u[2 * k + 2] = u[k] - ra[k];
      }
    }
  }
  uint32_t* rec = pa.bnd + idx * kBndStride;
#pragma unroll
  for (int k = 0; k < KN; ++k)
    if (k < nodes) {
      rec[2 * k] = u[k];
      rec[2 * k + 1] = ra[k];
    }
}

// ---------------------------------------------------------------------------
// 9. one merge level with the listing's placement: every slot gathers its
//    value before the insertion loop (the patch kernel then applies the loop)
// ---------------------------------------------------------------------------
template <typename E>
__global__ void __launch_bounds__(256) merge_r1_kernel(PlanArgs pa, int l, const void* vin, void* vout) {
  const HbmLevel& lv = pa.lev[l];
  const uint32_t bpm = (lv.nmax + 255) / 256;  // workgroups per merge
  const uint32_t m = blockIdx.x / bpm;
  const uint32_t t = (blockIdx.x % bpm) * 256 + threadIdx.x;
  const MergeGeom g = merge_geom(pa, lv.L, m);
  if (t >= g.N) return;
  const uint64_t gm = lv.merge_base + m;
  const uint32_t src = c0_offset(pa, lv, m, g, pa.P[gm], pa.side[gm], t);
  const E* in = reinterpret_cast<const E*>(vin);
  E* out = reinterpret_cast<E*>(vout);
  out[g.s + t] = in[g.s + (src < g.N ? src : t)];
}

void launch_merge_r1(const PlanArgs& pa, int l, const void* in, void* out, uint32_t eb, hipStream_t st) {
  const HbmLevel& lv = pa.lev[l];
  const dim3 grid((uint32_t)((uint64_t)lv.nmerge * ((lv.nmax + 255) / 256)));
  if (eb == 4) hipLaunchKernelGGL(merge_r1_kernel<uint32_t>, grid, dim3(256), 0, st, pa, l, in, out);
  else if (eb == 8) hipLaunchKernelGGL(merge_r1_kernel<uint64_t>, grid, dim3(256), 0, st, pa, l, in, out);
  else hipLaunchKernelGGL(merge_r1_kernel<uint4>, grid, dim3(256), 0, st, pa, l, in, out);
}

// ---------------------------------------------------------------------------
// host launcher
// ---------------------------------------------------------------------------
// The trace (one workgroup per insertion-loop workgroup) and the boundary
// records (one thread each) in one launch.
__global__ void __launch_bounds__(256) trace_bounds_kernel(PlanArgs pa) {
  if (blockIdx.x < pa.total_tail_wgs) trace_body(pa, blockIdx.x);
  else bounds_body(pa, (blockIdx.x - pa.total_tail_wgs) * 256 + threadIdx.x);
}

// The plans of many arrays, one launch per stage of launch_plan: job j of a
// stage owns workgroups [pre[j], pre[j+1]) (or workgroup j when the stage
// takes one per array).
enum PlanStage {
  kStCount, kStScanZ, kStZc, kStBreak, kStScanK, kStTailCount, kStScanB, kStScatter, kStResolve, kStTrace, kStages
};

template <int S>
__global__ void __launch_bounds__(256) plan_multi_kernel(const PlanArgs* __restrict__ pas,
                                                         const uint32_t* __restrict__ pre, uint32_t njobs) {
  __shared__ uint32_t tmp[8];
  __shared__ uint64_t red[4];
  constexpr bool kPerArray = S == kStScanZ || S == kStScanK || S == kStScanB;
  uint32_t j = blockIdx.x, u = 0;
  if (!kPerArray) {
    uint32_t lo = 0, hi = njobs;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (pre[mid] <= blockIdx.x) lo = mid;
      else hi = mid;
    }
    j = lo;
    u = blockIdx.x - pre[lo];
  }
  const PlanArgs& pa = pas[j];
  if constexpr (S == kStCount) {
    plan_count_body(pa, u, tmp);
  } else if constexpr (S == kStScanZ) {
    block_scan_all<256>(pa.ctot, pa.total_chunks, pa.zg, ~0ull, pa.status, 0u, tmp);
  } else if constexpr (S == kStZc) {
    zc_body(pa, (uint64_t)u * 256 + threadIdx.x);
  } else if constexpr (S == kStBreak) {
    const uint64_t t = block_sum_u64<256>(break_body(pa, (uint64_t)u * 256 + threadIdx.x), red);
    if (threadIdx.x == 0 && t) atomicAdd(pa.bits, (unsigned long long)t);
  } else if constexpr (S == kStScanK) {
    block_scan_all<256>(pa.kcnt, pa.total_merges, pa.toff, pa.tail_cap, pa.status, 2u, tmp);
  } else if constexpr (S == kStTailCount) {
    tail_count_body(pa, u, red);
  } else if constexpr (S == kStScanB) {
    block_scan_all<256>(pa.bcnt, pa.total_buckets, pa.boff, pa.pool_cap, pa.status, 1u, tmp);
  } else if constexpr (S == kStScatter) {
    tail_scatter_body(pa, u, red);
  } else if constexpr (S == kStResolve) {
    tail_resolve_body(pa, u);
  } else {
    if (u < pa.total_tail_wgs) trace_body(pa, u);
    else bounds_body(pa, (u - pa.total_tail_wgs) * 256 + threadIdx.x);
  }
}

// pre[k]: per-job workgroup prefixes (njobs + 1 entries) and units[k] their
// totals, for k = 0 chunks, 1 zc blocks, 2 break blocks, 3 insertion-loop
// workgroups, 4 trace and boundary-record workgroups.
void launch_plan_multi(const PlanArgs* pas, uint32_t njobs, const uint32_t* const* pre, const uint32_t* units,
                       hipStream_t st) {
  if (!njobs) return;
  const dim3 b(256);
  auto go = [&](auto kern, uint32_t grid, const uint32_t* p) {
    if (grid) hipLaunchKernelGGL(kern, dim3(grid), b, 0, st, pas, p, njobs);
  };
  go(plan_multi_kernel<kStCount>, units[0], pre[0]);
  go(plan_multi_kernel<kStScanZ>, njobs, nullptr);
  go(plan_multi_kernel<kStZc>, units[1], pre[1]);
  go(plan_multi_kernel<kStBreak>, units[2], pre[2]);
  go(plan_multi_kernel<kStScanK>, njobs, nullptr);
  go(plan_multi_kernel<kStTailCount>, units[3], pre[3]);
  go(plan_multi_kernel<kStScanB>, njobs, nullptr);
  go(plan_multi_kernel<kStScatter>, units[3], pre[3]);
  go(plan_multi_kernel<kStResolve>, units[3], pre[3]);
  go(plan_multi_kernel<kStTrace>, units[4], pre[4]);
}

void launch_plan(const PlanArgs& pa, hipStream_t st) {
  if (pa.nlev == 0) return;
  const uint64_t count_wgs = (pa.total_chunks + 4 * kCountChunksPerWave - 1) / (4 * kCountChunksPerWave);
  hipLaunchKernelGGL(plan_count_kernel, dim3((uint32_t)count_wgs), dim3(256), 0, st, pa);
  launch_scan(pa.ctot, pa.total_chunks, pa.part, pa.zg, ~0ull, pa.status, 0u, st);
  hipLaunchKernelGGL(zc_kernel, dim3((uint32_t)((std::max(pa.total_chunks, pa.total_buckets) + 255) / 256)), dim3(256),
                     0, st, pa);
  hipLaunchKernelGGL(plan_break_kernel, dim3((uint32_t)((pa.total_merges + 255) / 256)), dim3(256), 0, st, pa);
  launch_scan(pa.kcnt, pa.total_merges, pa.part, pa.toff, pa.tail_cap, pa.status, 2u, st);
  hipLaunchKernelGGL(tail_count_kernel, dim3((uint32_t)pa.total_tail_wgs), dim3(256), 0, st, pa);
  launch_scan(pa.bcnt, pa.total_buckets, pa.part, pa.boff, pa.pool_cap, pa.status, 1u, st);
  hipLaunchKernelGGL(tail_scatter_kernel, dim3((uint32_t)pa.total_tail_wgs), dim3(256), 0, st, pa);
  if (pa.placement == 2)
    hipLaunchKernelGGL(bal_words_kernel, dim3((uint32_t)pa.total_chunks), dim3(256), 0, st, pa);
  hipLaunchKernelGGL(tail_resolve_kernel, dim3((uint32_t)pa.total_tail_wgs), dim3(256), 0, st, pa);
  if (pa.placement == 2) {
    // the passes rank slots among the final labels
    hipLaunchKernelGGL(bal_count_kernel, dim3((uint32_t)pa.total_chunks), dim3(256), 0, st, pa);
    launch_scan(pa.ctot, pa.total_chunks, pa.part, pa.zg, ~0ull, pa.status, 0u, st);
    hipLaunchKernelGGL(bal_zc_kernel, dim3((uint32_t)((pa.total_chunks + 255) / 256)), dim3(256), 0, st, pa);
  }
  if (pa.tail_xsrc)
    hipLaunchKernelGGL(trace_bounds_kernel, dim3((uint32_t)(pa.total_tail_wgs + (pa.total_bnd + 255) / 256)), dim3(256),
                       0, st, pa);
}

}  // namespace ms
