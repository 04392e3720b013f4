// ms_kernels_group.hip -- LAM consecutive HBM merge levels in one pass.
//
// A workgroup produces T output slots [t0, t1) of one merge M of the top
// level of the group.  By the coin-flip loop's stable interleave (Algorithm
// 2) those slots come from one contiguous window of each half of M's input:
// [r0(t0), r0(t1)) of the left half and [t0 - r0(t0), t1 - r0(t1)) of the
// right half, r0(t) counting the zero flips before slot t (slots past the
// break step P take the side that is left, in order).  Each of these windows
// is itself the output window of a merge one level down, so the tile defines
// a binary tree of windows whose 2^LAM leaves are contiguous runs of the pass
// input.  Laid out in tree order, a window occupies the same LDS range as its
// two children, so every level is one interleave from one LDS buffer into the
// other.  The insertion loop's slots of every level inside the tile are then
// overwritten with their final values, fetched from the pass input at the
// offsets the plan traced down to it.
#include <stdlib.h>

#include <algorithm>

#include "ms_device.hpp"
#include "ms_plan.hpp"

namespace ms {

struct Win {
  uint32_t m, L, u0, u1, ra0, ra1, off, bo, P, side, n1, n2, g0, wb, toff;
  uint64_t s;
};

// One tile of one fused pass (tile = top merge * tpm + tile within it).
template <typename E, int T, int LAM, int NT>
__device__ __forceinline__ void group_body(const GroupArgs& a, uint32_t tile) {
  constexpr int NODES = (1 << LAM) - 1;
  constexpr int NB = NODES / 2 + 1;  // bottom windows
  // flip words of every window: at most T/32 + 8 per window and level
  constexpr int NWORD = LAM * (T / 32) + 8 * NODES + 8 * LAM;
  constexpr int KW = (NWORD + NT - 1) / NT;
  constexpr int PT = T / NT;  // staged elements per thread
  constexpr int PK = 2;        // patches per thread fetched ahead of the levels
  constexpr uint32_t NONE = 0xFFFFFFFFu;
  using R = typename RegOf<E>::type;
  // windows start at multiples of 4 slots (each input run's region is
  // rounded up to 4), so every group of 4 slots lies in one window
  constexpr int TB = T + 4 * (1 << LAM);
  __shared__ __align__(16) E buf[2][TB];
  __shared__ __align__(16) uint32_t words[NWORD];
  // zeros before each flip word: 16 bits suffice, which keeps the 4-level
  // tile within a quarter of the CU's LDS (four workgroups per CU)
  static_assert(32 * NWORD < 65536, "flip-word prefix must fit 16 bits");
  __shared__ uint16_t wpre[NWORD];
  __shared__ uint32_t tmp[NT / 64 + 1];
  __shared__ __align__(16) uint32_t hot[NODES][8];
  __shared__ Win win[NODES + 1];
  __shared__ uint32_t rec[2][2 * NODES];  // boundary records at both tile edges
  __shared__ uint32_t rs[2 * NB + 1];     // first element of each staged run in run order (+ end)
  __shared__ uint32_t rl[2 * NB];         // its LDS slot
  __shared__ uint32_t rsrc[2 * NB];       // its first element in the pass input, from the top merge's
  __shared__ uint32_t lgroups[LAM];       // groups of 4 slots per level
  // insertion-loop slots of the tile: per window, a range of the dense
  // per-step array (slots >= P) and a range of target entries (its buckets)
  __shared__ uint32_t pcnt[2 * NODES];
  __shared__ uint64_t pbase[2 * NODES];
  const int tid = threadIdx.x;
  const Key key{a.key0, a.key1};
  const E* X = reinterpret_cast<const E*>(a.X);
  const R* XR = reinterpret_cast<const R*>(a.X);
  E* Z = reinterpret_cast<E*>(a.Z);
  const uint32_t M = tile / a.tpm;
  const uint32_t b = tile - M * a.tpm;

  // 1. boundary records, and per window the break step, side and first step
  if (tid < 4 * NODES) {
    const uint32_t e = tid >= 2 * NODES ? 1u : 0u;
    const uint32_t w = tid - e * 2 * NODES;
    rec[e][w] = a.bnd[((uint64_t)M * (a.tpm + 1) + b + e) * kBndStride + w];
  } else if (tid >= 128 && tid < 128 + NODES) {
    const int k = tid - 128;
    const int d = 31 - __clz(k + 1);
    const int li = LAM - 1 - d;
    const uint32_t m = (M << d) + (uint32_t)(k - ((1 << d) - 1));
    const uint64_t gm = a.merge_base[li] + m;
    win[k].P = a.P[gm];
    win[k].side = a.side[gm];
    win[k].toff = a.toff[gm];
  }
  __syncthreads();
  if (rec[0][0] >= rec[1][0]) return;  // the top merge ends before this tile

  // 2. the window tree (one thread per window)
  uint64_t bq_lo = 0, bq_hi = 0;  // the window's buckets of target entries (threads < NODES)
  if (tid < NODES) {
    const int k = tid;
    const int d = 31 - __clz(k + 1);
    const int li = LAM - 1 - d;
    const uint32_t idx = (uint32_t)(k - ((1 << d) - 1));
    Win& w = win[k];
    w.m = (M << d) + idx;
    w.L = a.L[li];
    const uint64_t i0 = (uint64_t)w.m << w.L;
    const uint64_t s0 = bound(a.n, i0, a.c);
    const uint64_t mid = bound(a.n, i0 + (1ull << (w.L - 1)), a.c);
    const uint64_t e0 = bound(a.n, i0 + (1ull << w.L), a.c);
    w.s = s0;
    w.n1 = (uint32_t)(mid - s0);
    w.n2 = (uint32_t)(e0 - mid);
    const uint32_t u0 = rec[0][2 * k], u1 = rec[1][2 * k];
    w.u0 = u0;
    w.u1 = u1;
    w.ra0 = rec[0][2 * k + 1];
    w.ra1 = rec[1][2 * k + 1];
    w.g0 = u0 >> kGranLog;
    // LDS layout: every window's region is the union of the regions of the
    // 2^LAM input runs below it, each run rounded up to 4 slots; a window
    // starts where its left child does and its right child after the left
    // child's region
    auto region = [&](int node) -> uint32_t {
      const int dn = 31 - __clz(node + 1);
      const int first = ((node + 1) << (LAM - 1 - dn)) - 1;
      uint32_t S = 0;
      for (int q = first; q < first + (1 << (LAM - 1 - dn)); ++q) {
        const uint32_t la = rec[1][2 * q + 1] - rec[0][2 * q + 1], ln = rec[1][2 * q] - rec[0][2 * q];
        S += ((la + 3u) & ~3u) + ((ln - la + 3u) & ~3u);
      }
      return S;
    };
    uint32_t off = 0, node = 0;
    for (int j = d; j-- > 0;) {
      if ((idx >> j) & 1u) {
        off += region(2 * node + 1);
        node = 2 * node + 2;
      } else {
        node = 2 * node + 1;
      }
    }
    w.off = off;
    w.bo = d == LAM - 1 ? ((rec[1][2 * k + 1] - rec[0][2 * k + 1] + 3u) & ~3u) : region(2 * k + 1);
    // flip words: nodes in breadth-first order, whole granules per window
    uint32_t wb = 0;
    for (int j = 0; j < k; ++j) {
      const uint32_t a0 = rec[0][2 * j], a1 = rec[1][2 * j];
      wb += a1 > a0 ? 4 * (((a1 + 127) >> kGranLog) - (a0 >> kGranLog)) : 0u;
    }
    w.wb = wb;
    if (k >= NODES / 2) {
      // a bottom window reads one run of each half of its merge's input
      const uint32_t j = (uint32_t)(k - NODES / 2);
      const uint64_t sTop = bound(a.n, (uint64_t)M << a.L[LAM - 1], a.c);
      const uint32_t rel = (uint32_t)(s0 - sTop);
      // runs in tree order: their element counts add up to the tile's length
      uint32_t before = 0;
      for (int q = NODES / 2; q < k; ++q) before += rec[1][2 * q] - rec[0][2 * q];
      const uint32_t la = w.ra1 - w.ra0;
      rs[2 * j] = before;
      rs[2 * j + 1] = before + la;
      rl[2 * j] = off;
      rl[2 * j + 1] = off + w.bo;
      rsrc[2 * j] = rel + w.ra0;
      rsrc[2 * j + 1] = rel + w.n1 + (u0 - w.ra0);
      if (k == NODES - 1) rs[2 * j + 2] = rec[1][0] - rec[0][0];
    }
    if (k == NODES - 1) win[NODES].wb = wb + (u1 > u0 ? 4 * (((u1 + 127) >> kGranLog) - w.g0) : 0u);
    // insertion-loop slots: steps max(u0, P) .. u1 - 1, and the target entries
    // of the buckets that cover [u0, u1)
    const uint32_t P = w.P;
    const uint32_t x0 = max(u0, P), x1 = max(u1, P);
    uint64_t sb = (uint64_t)w.toff + (x0 - P);
    uint32_t sc = x1 - x0;
    if (sb >= a.tail_cap) sc = 0;
    else if (sb + sc > a.tail_cap) sc = (uint32_t)(a.tail_cap - sb);
    if (u1 > u0) {
      const uint64_t bb = a.bucket_base[li] + (uint64_t)w.m * a.bpm[li];
      bq_lo = bb + (u0 >> a.blog[li]);
      bq_hi = bb + ((u1 - 1) >> a.blog[li]) + 1;
    }
    pcnt[k] = sc;
    pbase[k] = sb;
  }
  __syncthreads();
  // the tile's length and its merge's start are the same in every lane:
  // scalar registers hold them
  const uint32_t len = uniform_u32(win[0].u1 - win[0].u0);
  const uint64_t sM = uniform_u64((uint32_t)(win[0].s >> 32), (uint32_t)win[0].s);

  // 3. loads: the 2^LAM runs of the pass input, and the first PK * NT
  //    insertion-loop patches (they land after the flips are counted)
  R v[PT];
  uint32_t sl[PT];  // LDS slot of each staged element (TB = none)
  {
    int r = 0;
    uint32_t si[PT];
#pragma unroll
    for (int i = 0; i < PT; ++i) {
      const uint32_t p = tid + NT * i;
      si[i] = 0;
      sl[i] = TB;
      if (p < len) {
        while (p >= rs[r + 1]) ++r;
        si[i] = rsrc[r] + (p - rs[r]);
        sl[i] = rl[r] + (p - rs[r]);
      }
    }
#pragma unroll
    for (int i = 0; i < PT; ++i) v[i] = XR[sM + si[i]];
  }
  // the bucket offsets of the target entries are in flight with the runs
  uint32_t boff_lo = 0, boff_hi = 0;
  if (tid < NODES && bq_hi > bq_lo) {
    boff_lo = a.boff[bq_lo];
    boff_hi = a.boff[bq_hi];
  }
  uint32_t stot = 0;
#pragma unroll
  for (int r = 0; r < NODES; ++r) stot += pcnt[r];
  // patch e of the ranges from rbeg on: its level (bits 16..), LDS slot
  // (bits 0..15) and pass-input offset, or NONE.  Ranges 0..NODES-1 are the
  // windows' insertion steps, NODES..2*NODES-1 their target entries.
  auto patch_at = [&](int rbeg, uint32_t e, uint32_t& meta) -> uint64_t {
    int r = rbeg;
    uint32_t start = 0;
    while (e >= start + pcnt[r]) {
      start += pcnt[r];
      ++r;
    }
    const int k = r < NODES ? r : r - NODES;
    const Win& w = win[k];
    const uint64_t idx = pbase[r] + (e - start);
    uint32_t x, xs;
    if (r < NODES) {
      x = max(w.u0, w.P) + (e - start);
      xs = a.tail_xsrc[idx];
    } else {
      x = a.pool_x[idx];
      xs = a.pool_xsrc[idx];
    }
    meta = NONE;
    if (xs == NONE || xs >= w.n1 + w.n2 || x < w.u0 || x >= w.u1) return 0;
    const int d = 31 - __clz(k + 1);
    meta = ((uint32_t)(LAM - 1 - d) << 16) | (w.off + (x - w.u0));
    return w.s + xs;
  };
  uint32_t pm[2 * PK];
  R pv[2 * PK];
#pragma unroll
  for (int i = 0; i < PK; ++i) {
    pm[i] = NONE;
    const uint32_t e = tid + NT * i;
    if (e < stot) {
      const uint64_t src = patch_at(0, e, pm[i]);
      if (pm[i] != NONE) pv[i] = XR[src];
    }
  }

  // 4. coin flips of every window of every level
  const uint32_t nwords = win[NODES].wb;
  for (uint32_t fb = tid; fb < nwords / 4; fb += NT) {
    int k = 0;
    while (k + 1 < NODES && 4 * fb >= win[k + 1].wb) ++k;
    const Win& w = win[k];
    const W4 f = flip_block(w.g0 + (fb - w.wb / 4), w.m, w.L, key);
    *reinterpret_cast<uint4*>(&words[4 * fb]) = make_uint4(f.w[0], f.w[1], f.w[2], f.w[3]);
  }
  __syncthreads();
  // zeros per word, scanned over all windows of all levels
  {
    uint32_t zl[KW];
    uint32_t zs = 0;
#pragma unroll
    for (int k = 0; k < KW; ++k) {
      const uint32_t wi = tid * KW + k;
      zl[k] = wi < nwords ? 32u - (uint32_t)__popc(words[wi]) : 0u;
      zs += zl[k];
    }
    uint32_t run = block_excl_scan<NT>(zs, tmp, nullptr);
#pragma unroll
    for (int k = 0; k < KW; ++k) {
      const uint32_t wi = tid * KW + k;
      if (wi < NWORD) wpre[wi] = (uint16_t)run;
      run += zl[k];
    }
  }
  // the staged runs land in LDS; the target-entry ranges are known now
#pragma unroll
  for (int i = 0; i < PT; ++i)
    if (sl[i] < (uint32_t)TB) reinterpret_cast<R*>(buf[0])[sl[i]] = v[i];
  if (tid < NODES) {
    const uint64_t hi = min((uint64_t)boff_hi, a.pool_cap);
    pcnt[NODES + tid] = hi > boff_lo ? (uint32_t)(hi - boff_lo) : 0u;
    pbase[NODES + tid] = boff_lo;
  }
  __syncthreads();
  uint32_t ptot = 0;
#pragma unroll
  for (int r = NODES; r < 2 * NODES; ++r) ptot += pcnt[r];
#pragma unroll
  for (int i = 0; i < PK; ++i) {
    pm[PK + i] = NONE;
    const uint32_t e = tid + NT * i;
    if (e < ptot) {
      const uint64_t src = patch_at(NODES, e, pm[PK + i]);
      if (pm[PK + i] != NONE) pv[PK + i] = XR[src];
    }
  }
  // per window, what the interleave needs.  Group q of the level (4 slots)
  // lies in window k from gpre = the groups of the windows before it on its
  // level; its LDS slot is s0 = off + 4 (q - gpre) and its merge slot
  // t0 = u0 + 4 (q - gpre), both one multiply-add from 4q.  Before the break
  // step, with zp = the wpre-based zero count before slot t (zeros in
  // [u0, t) plus zbase), a zero flip takes A at off + zp - zbase and a one
  // takes B at (off + la4 - u0 + zbase) + t - zp; from the break step on, t
  // maps to t + pdelta.  lim = min(u1, P): a group of 4 slots below it takes
  // the short path.
  if (tid < NODES) {
    const Win& w = win[tid];
    const int d = 31 - __clz(tid + 1);
    const uint32_t la4 = w.bo;  // the B input starts la4 slots after the window
    const uint32_t wbase = w.wb - 4 * w.g0;
    const uint32_t w0 = wbase + (w.u0 >> 5);
    const uint32_t zbase =
        w.u1 > w.u0 ? wpre[w0] + (uint32_t)__popc(~words[w0] & ((1u << (w.u0 & 31)) - 1u)) : 0u;
    const uint32_t pdelta = w.side == 0 ? w.off + la4 - w.n1 - w.u0 + w.ra0 : w.off - w.n2 - w.ra0;
    uint32_t gpre = 0;
    for (int q = (1 << d) - 1; q < tid; ++q) gpre += (win[q].u1 - win[q].u0 + 3u) >> 2;
    *reinterpret_cast<uint4*>(&hot[tid][0]) = make_uint4(w.u0 - 4 * gpre, min(w.u1, w.P), wbase, w.off - zbase);
    *reinterpret_cast<uint4*>(&hot[tid][4]) =
        make_uint4(w.off - 4 * gpre, w.off + la4 - w.u0 + zbase, pdelta, gpre);
    if (tid == (2 << d) - 2) lgroups[LAM - 1 - d] = gpre + ((w.u1 - w.u0 + 3u) >> 2);
  }
  __syncthreads();

  // 5. the levels, bottom up, each one interleave from one LDS buffer into
  //    the other (4 slots of one window per thread and step), then its
  //    insertion-loop slots
#pragma unroll
  for (int li = 0; li < LAM; ++li) {
    const int d = LAM - 1 - li;
    const int kf = (1 << d) - 1;
    const E* src = buf[li & 1];
    E* dst = buf[(li + 1) & 1];
    const uint32_t ng = lgroups[li];
    for (uint32_t g = tid; g < ng; g += NT) {
      int k = kf;
#pragma unroll
      for (int q = 1; q < (1 << d); ++q) k += g >= hot[kf + q][7] ? 1 : 0;
      const uint4 h0 = *reinterpret_cast<const uint4*>(&hot[k][0]);
      const uint4 h1 = *reinterpret_cast<const uint4*>(&hot[k][4]);
      const uint32_t s0 = 4 * g + h1.x;
      const uint32_t t0 = 4 * g + h0.x;
      const uint32_t wi = min(h0.z + (t0 >> 5), (uint32_t)NWORD - 2);
      const uint32_t wlo = words[wi], whi = words[wi + 1];
      const uint32_t zp = wpre[wi] + (uint32_t)__popc(~wlo & ((1u << (t0 & 31)) - 1u));
      const uint32_t bits4 = (uint32_t)((((uint64_t)whi << 32) | wlo) >> (t0 & 31));
      uint32_t fr[4];
      if (t0 + 4 <= h0.y) {
        // four slots of the window before the break step: with o_j the ones
        // among the first j flips, slot j takes B at bb + o_j or A at
        // ab + j - o_j
        // x = bb + o_j and w = ab - o_j, moved by the all-ones mask of each
        // 1 flip; the slot picks x or w + j through that mask (kept opaque so
        // that it stays a bit select instead of a compare and a select)
        uint32_t w = h0.w + zp, x = h1.y + t0 - zp;
        asm volatile("" : "+v"(w), "+v"(x));
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          uint32_t m = 0u - ((bits4 >> j) & 1u);
          asm volatile("" : "+v"(m));
          fr[j] = (x & m) | ((w + j) & ~m);
          x -= m;
          w += m;
        }
      } else {
        const uint32_t P = win[k].P;
        uint32_t z = zp;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const uint32_t t = t0 + j;
          const uint32_t bit = (bits4 >> j) & 1u;
          const uint32_t rk = bit ? h1.y + t - z : h0.w + z;
          fr[j] = min(t < P ? rk : t + h1.z, (uint32_t)TB - 1);
          z += bit ^ 1u;
        }
      }
      if constexpr (sizeof(E) == 4) {
        uint4 o;
        o.x = *reinterpret_cast<const uint32_t*>(&src[fr[0]]);
        o.y = *reinterpret_cast<const uint32_t*>(&src[fr[1]]);
        o.z = *reinterpret_cast<const uint32_t*>(&src[fr[2]]);
        o.w = *reinterpret_cast<const uint32_t*>(&src[fr[3]]);
        *reinterpret_cast<uint4*>(&dst[s0]) = o;
      } else {
        const R* srcR = reinterpret_cast<const R*>(src);
        R* dstR = reinterpret_cast<R*>(dst);
        const R a0 = srcR[fr[0]], a1 = srcR[fr[1]], a2 = srcR[fr[2]], a3 = srcR[fr[3]];
        dstR[s0] = a0;
        dstR[s0 + 1] = a1;
        dstR[s0 + 2] = a2;
        dstR[s0 + 3] = a3;
      }
    }
    __syncthreads();
    // insertion-loop slots of this level inside the tile
#pragma unroll
    for (int i = 0; i < 2 * PK; ++i)
      if (pm[i] != NONE && (pm[i] >> 16) == (uint32_t)li && (pm[i] & 0xFFFFu) < (uint32_t)TB)
        reinterpret_cast<R*>(dst)[pm[i] & 0xFFFFu] = pv[i];
    for (uint32_t e = NT * PK + tid; e < stot; e += NT) {
      uint32_t meta;
      const uint64_t srcx = patch_at(0, e, meta);
      if (meta != NONE && (meta >> 16) == (uint32_t)li && (meta & 0xFFFFu) < (uint32_t)TB)
        dst[meta & 0xFFFFu] = X[srcx];
    }
    for (uint32_t e = NT * PK + tid; e < ptot; e += NT) {
      uint32_t meta;
      const uint64_t srcx = patch_at(NODES, e, meta);
      if (meta != NONE && (meta >> 16) == (uint32_t)li && (meta & 0xFFFFu) < (uint32_t)TB)
        dst[meta & 0xFFFFu] = X[srcx];
    }
    __syncthreads();
  }

  // 6. store the top window
  const E* fin = buf[LAM & 1];
  E* out = Z + sM + win[0].u0;
  for (uint32_t o = 4 * tid; o < len; o += 4 * NT) {
    const uint32_t cnt = min(4u, len - o);
    if (cnt == 4 && sizeof(E) == 4 && ((uintptr_t)(out + o) & 15) == 0) {
      *reinterpret_cast<uint4*>(out + o) = *reinterpret_cast<const uint4*>(&fin[o]);
    } else {
#pragma unroll
      for (uint32_t k = 0; k < 4; ++k)
        if (k < cnt) out[o + k] = fin[o + k];
    }
  }
}

// Workgroups are dealt to the 8 XCDs round robin; give each XCD a
// contiguous eighth of the tiles so that the tiles of one merge share an L2,
// which then also serves most insertion-loop fetches within the merge.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t ntiles) {
  const uint32_t q = ntiles >> 3, r = ntiles & 7u;
  const uint32_t x = blockIdx.x & 7u, i = blockIdx.x >> 3;
  return x * q + min(x, r) + i;
}

// The 4-level tiles of 4- and 8-byte elements are asked to fit 64 VGPRs (8
// waves per SIMD, as their LDS allows); the others fit by themselves or are
// bound by their VGPRs.
template <typename E, int T, int LAM, int NT>
constexpr int kGroupWaves = LAM == 4 && sizeof(E) <= 8 && NT == 512 ? 8 : 1;

template <typename E, int T, int LAM, int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(kGroupWaves<E, T, LAM, NT>)))
group_kernel(GroupArgs a) {
  if (blockIdx.x >= a.ntiles) return;
  group_body<E, T, LAM, NT>(a, xcd_tile(a.ntiles));
}

// The same pass of many arrays in one launch: job j owns tiles
// [tpre[j], tpre[j+1]) of the ntiles = tpre[njobs] tiles.
template <typename E, int T, int LAM, int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(kGroupWaves<E, T, LAM, NT>)))
group_multi_kernel(const GroupArgs* __restrict__ jobs,
                                                         const uint32_t* __restrict__ tpre, uint32_t njobs,
                                                         uint32_t ntiles) {
  if (blockIdx.x >= ntiles) return;
  const uint32_t tile = xcd_tile(ntiles);
  uint32_t lo = 0, hi = njobs;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (tpre[mid] <= tile) lo = mid;
    else hi = mid;
  }
  group_body<E, T, LAM, NT>(jobs[lo], tile - tpre[lo]);
}

// Slots per tile for 4-byte elements: 4096 with 512 threads (the default:
// measured faster) or 2048 with 256 threads (MS_GROUP_TILE=2048).  A tuning
// knob only: the permutation does not depend on it.  8-byte elements take
// 2048 slots with 512 threads (8 waves per SIMD; measured faster than 256),
// 16-byte elements 1024 slots with 256 threads (512 measured much slower:
// at 78-94 VGPRs the larger workgroup fits fewer times per CU).
static int group_tile_u32() {
  static const int t = [] {
    const char* e = getenv("MS_GROUP_TILE");
    return e && atoi(e) == 2048 ? 2048 : 4096;
  }();
  return t;
}

int group_tile(uint32_t eb) { return eb == 4 ? group_tile_u32() : eb == 8 ? 2048 : 1024; }

template <typename E, int T, int NT>
static void launch_group_t(const GroupArgs& a, int lam, uint64_t tiles, hipStream_t st) {
  const dim3 g((uint32_t)tiles), b(NT);
  if (lam == 1) hipLaunchKernelGGL((group_kernel<E, T, 1, NT>), g, b, 0, st, a);
  else if (lam == 2) hipLaunchKernelGGL((group_kernel<E, T, 2, NT>), g, b, 0, st, a);
  else if (lam == 3) hipLaunchKernelGGL((group_kernel<E, T, 3, NT>), g, b, 0, st, a);
  else hipLaunchKernelGGL((group_kernel<E, T, 4, NT>), g, b, 0, st, a);
}

template <typename E, int T, int NT>
static void launch_group_multi_t(const GroupArgs* jobs, const uint32_t* tpre, uint32_t njobs, uint32_t ntiles,
                                 int lam, hipStream_t st) {
  const dim3 g(ntiles), b(NT);
  if (lam == 1) hipLaunchKernelGGL((group_multi_kernel<E, T, 1, NT>), g, b, 0, st, jobs, tpre, njobs, ntiles);
  else if (lam == 2) hipLaunchKernelGGL((group_multi_kernel<E, T, 2, NT>), g, b, 0, st, jobs, tpre, njobs, ntiles);
  else if (lam == 3) hipLaunchKernelGGL((group_multi_kernel<E, T, 3, NT>), g, b, 0, st, jobs, tpre, njobs, ntiles);
  else hipLaunchKernelGGL((group_multi_kernel<E, T, 4, NT>), g, b, 0, st, jobs, tpre, njobs, ntiles);
}

void launch_group_multi(const GroupArgs* jobs, const uint32_t* tpre, uint32_t njobs, uint32_t ntiles, int lam,
                        uint32_t eb, hipStream_t st) {
  if (!ntiles) return;
  if (eb == 4) {
    if (group_tile_u32() == 2048) launch_group_multi_t<uint32_t, 2048, 256>(jobs, tpre, njobs, ntiles, lam, st);
    else launch_group_multi_t<uint32_t, 4096, 512>(jobs, tpre, njobs, ntiles, lam, st);
  } else if (eb == 8) {
    launch_group_multi_t<uint64_t, 2048, 512>(jobs, tpre, njobs, ntiles, lam, st);
  } else {
    launch_group_multi_t<uint4, 1024, 256>(jobs, tpre, njobs, ntiles, lam, st);
  }
}

void launch_group(const GroupArgs& a, int lam, uint32_t eb, uint64_t grid, hipStream_t st) {
  if (eb == 4) {
    if (group_tile_u32() == 2048) launch_group_t<uint32_t, 2048, 256>(a, lam, grid, st);
    else launch_group_t<uint32_t, 4096, 512>(a, lam, grid, st);
  } else if (eb == 8) {
    launch_group_t<uint64_t, 2048, 512>(a, lam, grid, st);
  } else {
    launch_group_t<uint4, 1024, 256>(a, lam, grid, st);
  }
}

}  // namespace ms
