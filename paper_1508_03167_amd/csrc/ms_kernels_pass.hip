// ms_kernels_pass.hip -- LAM consecutive HBM merge levels in one pass over the array.
//
// A workgroup produces T output slots [u0, u1) of one merge M of the pass's
// top level.  By the stable interleave of the coin-flip loop (Algorithm 2),
// those slots come from one contiguous window of each half of M's input:
// [r(u0), r(u1)) of the left half and [u0 - r(u0), u1 - r(u1)) of the right
// half, r(u) counting the zero flips before slot u (from the break step P on,
// the side that is left, in order).  Each of those windows is the output
// window of a merge one level down, so the tile defines a binary tree of
// windows whose 2^LAM leaves are contiguous runs of the pass input.  The
// plan's boundary records give every node's window start and rank at both
// tile edges.
//
// Layout.  At each level of the pass, every window occupies LDS positions
// that agree with its merge slots modulo 32: window k of level li holds merge
// slot u at position D_k + u, D_k a multiple of 32.  So the 32 slots of one
// coin-flip word are 32 consecutive positions, and one table entry per word
// holds all a slot needs:
//   fw  the flip word, with every flip from the break step P on replaced by
//       the side that is left (1 when A ran out: the rest comes from B; 0
//       when B ran out), which makes the interleave's rank rule exact to the
//       end of the merge;
//   ZA  the position, one level down, of the A element the first zero flip
//       of the word would take, less the zeros before the word's first slot;
//   OB  the same for B and the ones
// (ZA and OB are positions below 2^16 and share one 32-bit word).  A slot at
// bit s of its word then reads, one level down, position
// ZA + (zeros of fw below s) on a 0 flip and OB + (ones of fw below s) on a
// 1 flip.  Positions outside the windows (the ends of a window's first and
// last word) compute positions within 31 of a real window below them and are
// never read by the level above, so the level buffers carry 32 guard
// positions at each end and nothing is clamped.
//
// Everything above depends only on (n, cutoff, seed), so the plan builds it
// once per tile (pass_desc_kernel: the window tree, the flips, their zero
// counts, the table, the staged runs' layout and the insertion-loop ranges)
// into a tile descriptor.  The pass itself (pass_kernel) loads its
// descriptor, stages the runs, runs the levels bottom up -- each one
// interleave from one LDS buffer into the other, then the level's
// insertion-loop slots (Algorithm 2, second loop) overwritten with their
// final values, fetched from the pass input at the offsets the plan traced
// down to it -- and stores the top window.
#include <stdlib.h>

#include <algorithm>
#include <type_traits>

#include "ms_device.hpp"
#include "ms_plan.hpp"

namespace ms {

template <int T, int LAM>
struct DescShape {
  static constexpr int NODES = (1 << LAM) - 1;
  static constexpr int NB = 1 << (LAM - 1);  // bottom windows
  static constexpr int NRUN = 1 << LAM;      // staged runs of the pass input
  // flip words of every window: at most T/32 + 2 per level plus one per window
  static constexpr int NE = LAM * (T / 32) + 2 * NODES + LAM + 2;
  // positions per level buffer: the words of the widest level plus 32 guard
  // positions at each end (also holds the staged runs, each padded to whole
  // 16-byte vectors)
  static constexpr int BUF = T + 64 * NB + 64;
  static_assert(BUF < 65536, "positions fit 16 bits");
};

// A window's record in the descriptor: what the insertion-loop patches need.
enum { dU0, dU1, dP, dD, dN, dLi, dSrel, dDbase, dDcnt, dPlo, dPcnt, dPad, kDN };

template <int T, int LAM>
struct __align__(16) TileDesc {
  using S = DescShape<T, LAM>;
  uint32_t len;            // slots of the tile (0: the top merge ends before it)
  uint32_t u0;             // its first slot in the top merge (a multiple of T)
  uint32_t sM_lo, sM_hi;   // the top merge's first element
  uint32_t dep_tb[LAM + 1];          // first table entry of each depth (top first) and the end
  uint32_t run_base[S::NRUN];        // LDS position of each run's first vector
  uint32_t run_vpre[S::NRUN + 1];    // vectors before each run
  uint32_t run_grel[S::NRUN];        // each run's first vector (element index relative to sMa:
                                     // sM rounded down to a whole 16-byte vector)
  uint32_t node[S::NODES][kDN];      // windows, breadth first
  uint2 tab[S::NE];                  // (fw, ZA | OB << 16)
};

template <int T, int LAM>
constexpr uint32_t desc_words() { return (uint32_t)(sizeof(TileDesc<T, LAM>) / 4); }

// Working fields of a window while its descriptor is built.
enum {
  // the four read together when the table entries are finished come first
  kZ0, kCA, kCB, kWt,
  kU0, kU1, kRa0, kRa1, kP, kSide, kM, kL, kTb, kD, kBlk, kZf, kToff, kN, kLi, kRes, kNF
};

// Entry li (< LAM, different per lane) of a per-level argument array: a
// select over the LAM entries, which stay scalar, rather than a vector load
// from the argument memory with its own wait.
__device__ __forceinline__ uint32_t scalar_of(uint32_t v) { return uniform_u32(v); }
__device__ __forceinline__ uint64_t scalar_of(uint64_t v) { return uniform_u64((uint32_t)(v >> 32), (uint32_t)v); }
template <int LAM, typename T>
__device__ __forceinline__ T level_pick(const T (&v)[kGroupMax], int li) {
  T x = scalar_of(v[0]);
#pragma unroll
  for (int i = 1; i < LAM; ++i) {
    const T y = scalar_of(v[i]);
    x = li == i ? y : x;
  }
  return x;
}

// The descriptor of one tile (tile = top merge * tpm + tile within it), by
// NTB threads, into global memory at out.
template <typename E, int T, int LAM, int NTB>
__device__ __forceinline__ void desc_body(const GroupArgs& a, uint32_t tile, uint32_t* out) {
  using S = DescShape<T, LAM>;
  constexpr int NODES = S::NODES, NRUN = S::NRUN, NE = S::NE;
  constexpr int VE = 16 / (int)sizeof(E) > 0 ? 16 / (int)sizeof(E) : 1;
  constexpr int KW = (NE + NTB - 1) / NTB;  // table entries per thread in the scan
  constexpr uint32_t DW4 = desc_words<T, LAM>() / 4;
  static_assert(kNF % 4 == 0, "window rows are whole 16-byte vectors");
  __shared__ TileDesc<T, LAM> td;
  __shared__ __align__(16) uint32_t nd[NODES][kNF];
  __shared__ uint32_t rec[2][2 * NODES];  // boundary records at both tile edges
  __shared__ uint32_t tmp[NTB / 64 + 1];
  __shared__ uint32_t nblk_tot;
  const int tid = threadIdx.x;
  const Key key{a.key0, a.key1};
  const uint32_t M = tile / a.tpm;
  const uint32_t b = tile - M * a.tpm;
  const uint32_t ve = a.vec_ok ? (uint32_t)VE : 1u;

  // 1. boundary records, and per window the break step, side and first step
  if (tid < 4 * NODES) {
    const uint32_t e = tid >= 2 * NODES ? 1u : 0u;
    const uint32_t w = tid - e * 2 * NODES;
    rec[e][w] = a.bnd[((uint64_t)M * (a.tpm + 1) + b + e) * kBndStride + w];
  }
  // (the merges' break step, side and tail offset by the second wave, beside
  // the first wave's boundary-record loads)
  constexpr int ND0 = 64;
  static_assert(4 * NODES <= 64 && ND0 + NODES <= NTB, "the set-up loads fit the first two waves");
  if (tid >= ND0 && tid < ND0 + NODES) {
    const int k = tid - ND0;
    const int d = 31 - __clz(k + 1);
    const int li = LAM - 1 - d;
    const uint32_t m = (M << d) + (uint32_t)(k - ((1 << d) - 1));
    const uint64_t gm = level_pick<LAM>(a.merge_base, li) + m;
    nd[k][kP] = a.P[gm];
    nd[k][kSide] = a.side[gm];
    nd[k][kToff] = a.toff[gm];
  }
  __syncthreads();
  if (rec[0][0] >= rec[1][0]) {
    // the top merge ends before this tile
    if (tid == 0) out[0] = 0u;
    return;
  }

  // 2. the window tree, one lane of wave 0 per window: table entries and
  //    flip blocks by prefix over the windows (breadth first, so each
  //    level's windows are consecutive), positions, staged runs, and the
  //    insertion-loop ranges (their bucket offsets are loaded here and used
  //    after the table is built, so the loads overlap the flips)
  uint64_t p_lo = 0, p_hi = 0;
  bool p_any = false;
  if (tid < 64) {
    const int k = tid;
    const bool act = k < NODES;
    const int d = 31 - __clz(k + 1);
    const int li = LAM - 1 - d;
    const uint32_t idx = (uint32_t)(k - ((1 << d) - 1));
    uint32_t u0 = 0, u1 = 0, ra0 = 0, ra1 = 0, m = 0, L = 0, n1 = 0, n2 = 0;
    uint64_t s0 = 0;
    if (act) {
      u0 = rec[0][2 * k];
      u1 = rec[1][2 * k];
      ra0 = rec[0][2 * k + 1];
      ra1 = rec[1][2 * k + 1];
      m = (M << d) + idx;
      L = level_pick<LAM>(a.L, li);
      const uint64_t i0 = (uint64_t)m << L;
      s0 = bound(a.n, i0, a.c);
      const uint64_t mid = bound(a.n, i0 + (1ull << (L - 1)), a.c);
      const uint64_t e0 = bound(a.n, i0 + (1ull << L), a.c);
      n1 = (uint32_t)(mid - s0);
      n2 = (uint32_t)(e0 - mid);
    }
    const uint64_t sM = __shfl(s0, 0, 64);
    // element offsets in the descriptor are relative to sM rounded down to
    // a whole vector, which no run's aligned start lies below
    const uint64_t sMa = sM - sM % ve;
    const bool ne = act && u1 > u0;
    const uint32_t nw = ne ? ((u1 - 1) >> 5) - (u0 >> 5) + 1 : 0u;
    const uint32_t nblk = ne ? ((u1 - 1) >> 7) - (u0 >> 7) + 1 : 0u;
    const uint32_t tb = wave_incl_scan(nw) - nw;
    const uint32_t blk = wave_incl_scan(nblk) - nblk;
    const uint32_t lb = __shfl(tb, (1 << d) - 1, 64);  // first entry of this window's level
    const uint32_t D = 32u * (tb - lb + 1u) - 32u * (u0 >> 5);
    // staged runs: the A and B run of each bottom window, in window order,
    // each in a region of whole 16-byte vectors starting at its run's
    // element modulo VE (so the loads are aligned 16-byte copies)
    const bool bot = act && d == LAM - 1;
    const uint64_t gA = s0 + ra0, gB = s0 + n1 + (u0 - ra0);
    const uint32_t lenA = ra1 - ra0, lenB = (u1 - ra1) - (u0 - ra0);
    const uint32_t offA = (uint32_t)(gA % ve), offB = (uint32_t)(gB % ve);
    const uint32_t regA = bot && lenA ? (offA + lenA + ve - 1) / ve * ve : 0u;
    const uint32_t regB = bot && lenB ? (offB + lenB + ve - 1) / ve * ve : 0u;
    const uint32_t rpre = wave_incl_scan(regA + regB) - (regA + regB);  // 0 up to the first bottom window
    const uint32_t baseA = 32u + rpre, baseB = baseA + regA;
    uint32_t CA = baseA + offA - ra0, CB = baseB + offB - (u0 - ra0);
    // an upper window reads its children's positions
    const uint32_t Dl = __shfl(D, min(2 * k + 1, 63), 64), Dr = __shfl(D, min(2 * k + 2, 63), 64);
    if (!bot) {
      CA = Dl;
      CB = Dr;
    }
    if (act) {
      const uint32_t P = nd[k][kP];
      nd[k][kZ0] = 0u;
      nd[k][kCA] = CA;
      nd[k][kCB] = CB;
      nd[k][kWt] = (u0 >> 5) - tb;  // the word of table entry e is kWt + e
      nd[k][kU0] = u0;
      nd[k][kU1] = u1;
      nd[k][kRa0] = ra0;
      nd[k][kM] = m;
      nd[k][kL] = L;
      nd[k][kTb] = tb;
      nd[k][kBlk] = blk;
      nd[k][kZf] = 0u;
      if (k == (1 << d) - 1) td.dep_tb[d] = tb;
      if (k == NODES - 1) {
        td.dep_tb[LAM] = tb + nw;
        nblk_tot = blk + nblk;
      }
      if (bot) {
        const uint32_t j = (uint32_t)(k - NODES / 2);
        td.run_base[2 * j] = baseA;
        td.run_base[2 * j + 1] = baseB;
        td.run_grel[2 * j] = (uint32_t)(gA - offA - sMa);
        td.run_grel[2 * j + 1] = (uint32_t)(gB - offB - sMa);
        td.run_vpre[2 * j] = rpre / ve;
        td.run_vpre[2 * j + 1] = (rpre + regA) / ve;
        if (k == NODES - 1) td.run_vpre[NRUN] = (rpre + regA + regB) / ve;
      }
      // insertion-loop slots: steps max(u0, P) .. u1 - 1 (a dense range of
      // the per-step arrays), and the target entries of the buckets that
      // cover [u0, u1)
      const uint32_t x0 = max(u0, P), x1 = max(u1, P);
      const uint64_t sb = (uint64_t)nd[k][kToff] + (x0 - P);
      uint32_t sc = x1 - x0;
      if (sb >= a.tail_cap) sc = 0;
      else if (sb + sc > a.tail_cap) sc = (uint32_t)(a.tail_cap - sb);
      if (u1 > u0) {
        const uint64_t bb = level_pick<LAM>(a.bucket_base, li) + (uint64_t)m * level_pick<LAM>(a.bpm, li);
        const uint32_t blg = level_pick<LAM>(a.blog, li);
        p_lo = a.boff[bb + (u0 >> blg)];
        p_hi = a.boff[bb + ((u1 - 1) >> blg) + 1];
        p_any = true;
      }
      uint32_t* r = td.node[k];
      r[dU0] = u0;
      r[dU1] = u1;
      r[dP] = P;
      r[dD] = D;
      r[dN] = n1 + n2;
      r[dLi] = (uint32_t)li;
      r[dSrel] = (uint32_t)(s0 - sMa);
      r[dDbase] = (uint32_t)sb;
      r[dDcnt] = sc;
      r[dPad] = 0u;
      if (k == 0) {
        td.len = u1 - u0;
        td.u0 = u0;
        td.sM_lo = (uint32_t)sM;
        td.sM_hi = (uint32_t)(sM >> 32);
      }
    }
  }
  __syncthreads();

  // 3. coin flips of every window, words inside the window only, with the
  //    flips from the break step on replaced by the side that is left
  const uint32_t nblk = nblk_tot;
  for (uint32_t fb = tid; fb < nblk; fb += NTB) {
    // the last window whose first block is at most fb (windows without
    // blocks share their prefix with the next one, so the last is not empty)
    int k = 0;
#pragma unroll
    for (int h = (NODES + 1) / 2; h >= 1; h >>= 1) k += (k + h < NODES && fb >= nd[k + h][kBlk]) ? h : 0;
    const uint32_t u0 = nd[k][kU0], u1 = nd[k][kU1];
    const uint32_t g = (u0 >> 7) + (fb - nd[k][kBlk]);
    const W4 f = flip_block(g, nd[k][kM], nd[k][kL], key);
    const uint32_t P = nd[k][kP], side = nd[k][kSide];
    const uint32_t w0 = u0 >> 5, w1 = (u1 - 1) >> 5;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const uint32_t w = 4 * g + (uint32_t)e;
      if (w < w0 || w > w1) continue;
      uint32_t fw = f.w[e];
      const uint32_t t0 = 32u * w;
      if (t0 + 32u > P) {
        // flips at slots >= P: the side that is left
        const uint32_t hi = t0 >= P ? 0xFFFFFFFFu : ~((1u << (P - t0)) - 1u);
        fw = side == 0 ? (fw | hi) : (fw & ~hi);
      }
      td.tab[nd[k][kTb] + (w - w0)] = make_uint2(fw, (uint32_t)k);
      if (w == w0) nd[k][kZf] = (uint32_t)__popc(~fw & ((1u << (u0 & 31)) - 1u));
    }
  }
  __syncthreads();

  // 4. zeros per word, scanned over all table entries; the first entry of
  //    each window fixes the window's base
  const uint32_t nent = td.dep_tb[LAM];
  uint32_t zl[KW];
  {
    uint32_t zs = 0;
#pragma unroll
    for (int q = 0; q < KW; ++q) {
      const uint32_t e = tid * KW + q;
      zl[q] = e < nent ? 32u - (uint32_t)__popc(td.tab[e].x) : 0u;
      zs += zl[q];
    }
    uint32_t run = block_excl_scan<NTB>(zs, tmp, nullptr);
#pragma unroll
    for (int q = 0; q < KW; ++q) {
      const uint32_t e = tid * KW + q;
      const uint32_t z = zl[q];
      zl[q] = run;  // zeros over all entries before e
      run += z;
      if (e < nent) {
        const uint32_t k = td.tab[e].y;
        if (e == nd[k][kTb]) nd[k][kZ0] = nd[k][kRa0] - nd[k][kZf] - zl[q];
      }
    }
  }
  __syncthreads();
  // 5. each entry's ZA and OB
#pragma unroll
  for (int q = 0; q < KW; ++q) {
    const uint32_t e = tid * KW + q;
    if (e < nent) {
      const uint32_t k = td.tab[e].y;
      const uint4 c = *reinterpret_cast<const uint4*>(&nd[k][kZ0]);  // (Z0, CA, CB, Wt)
      const uint32_t z = c.x + zl[q];  // zeros of the merge before the word's first slot
      const uint32_t w = c.w + e;
      const uint32_t za = c.y + z, ob = c.z + 32u * w - z;
      td.tab[e].y = (za & 0xFFFFu) | (ob << 16);
    }
  }
  __syncthreads();
  // the windows' target-entry ranges, from the loads issued in step 2
  if (tid < NODES) {
    const uint64_t hi = min(p_hi, a.pool_cap);
    td.node[tid][dPlo] = p_any ? (uint32_t)p_lo : 0u;
    td.node[tid][dPcnt] = p_any && hi > p_lo ? (uint32_t)(hi - p_lo) : 0u;
  }
  __syncthreads();
  // 6. out
  const uint4* src = reinterpret_cast<const uint4*>(&td);
  uint4* dst = reinterpret_cast<uint4*>(out);
  for (uint32_t i = tid; i < DW4; i += NTB) dst[i] = src[i];
}

// slots per thread and step in the 4-byte levels
constexpr uint32_t kPassGroup4 = 4;

// One tile of one fused pass, from its descriptor.
template <typename E, int T, int LAM, int NT>
__device__ __forceinline__ void pass_body(const GroupArgs& a, uint32_t tile) {
  using S = DescShape<T, LAM>;
  constexpr int NODES = S::NODES, NRUN = S::NRUN, BUF = S::BUF;
  constexpr int VE = 16 / (int)sizeof(E) > 0 ? 16 / (int)sizeof(E) : 1;  // elements per 16 bytes
  constexpr int MAXV = T / VE + 2 * NRUN + 2;                           // staged 16-byte vectors
  constexpr int PV = (MAXV + NT - 1) / NT;
  constexpr uint32_t DW4 = desc_words<T, LAM>() / 4;
  constexpr int PK = 2;  // insertion-loop patches per thread fetched ahead of the levels, per kind
  constexpr uint32_t NONE = 0xFFFFFFFFu;
  static_assert(NRUN * VE <= 64 * S::NB, "staged run padding fits the guard space");
  using R = typename RegOf<E>::type;
  __shared__ __align__(16) E buf[2][BUF];
  __shared__ TileDesc<T, LAM> td;
  __shared__ uint32_t pcnt[2 * NODES];  // insertion-loop patches: per window a dense range
  __shared__ uint32_t pbase[2 * NODES];  //   and a range of target entries
  const int tid = threadIdx.x;

  // 1. the descriptor
  {
    const uint4* src = reinterpret_cast<const uint4*>(a.desc + (uint64_t)tile * a.desc_words);
    uint4* dst = reinterpret_cast<uint4*>(&td);
    for (uint32_t i = tid; i < DW4; i += NT) dst[i] = src[i];
  }
  __syncthreads();
  const uint32_t len = uniform_u32(td.len);
  if (len == 0) return;  // the top merge ends before this tile
  const uint64_t sM = uniform_u64(td.sM_hi, td.sM_lo);
  const uint32_t u0top = uniform_u32(td.u0);
  const uint64_t sMa = a.vec_ok ? sM - sM % VE : sM;
  const E* X = reinterpret_cast<const E*>(a.X);
  const E* XM = X + sMa;
  E* Z = reinterpret_cast<E*>(a.Z);
  if (tid < 2 * NODES) {
    const int k = tid < NODES ? tid : tid - NODES;
    pcnt[tid] = tid < NODES ? td.node[k][dDcnt] : td.node[k][dPcnt];
    pbase[tid] = tid < NODES ? td.node[k][dDbase] : td.node[k][dPlo];
  }

  // 2. staging loads: the runs' 16-byte vectors (element loads for arrays
  //    that are not 16-byte aligned), held in registers until they land
  const uint32_t nvec = td.run_vpre[NRUN];
  uint4 sv[PV];
  uint32_t spos[PV];  // LDS position of each loaded vector, BUF = none
  if (a.vec_ok) {
#pragma unroll
    for (int i = 0; i < PV; ++i) {
      const uint32_t v = tid + NT * i;
      spos[i] = BUF;
      if (v < nvec) {
        int r = 0;
#pragma unroll
        for (int h = NRUN / 2; h >= 1; h >>= 1) r += v >= td.run_vpre[r + h] ? h : 0;
        const uint32_t rel = v - td.run_vpre[r];
        const uint64_t g = sMa + td.run_grel[r] + (uint64_t)rel * VE;
        spos[i] = td.run_base[r] + rel * VE;
        if (g + VE <= a.n) {
          sv[i] = *reinterpret_cast<const uint4*>(X + g);
        } else {
          // the array's last vector: only its elements below n exist
          E tmpv[VE];
#pragma unroll
          for (int e = 0; e < VE; ++e) tmpv[e] = g + e < a.n ? X[g + e] : E();
          sv[i] = *reinterpret_cast<const uint4*>(tmpv);
        }
      }
    }
  }
  __syncthreads();  // pcnt, pbase
  uint32_t stot = 0, ptot = 0;
#pragma unroll
  for (int r = 0; r < NODES; ++r) {
    stot += pcnt[r];
    ptot += pcnt[NODES + r];
  }
  // patch e of the ranges from rbeg on: its range, and in `start` the
  // patches of the range's predecessors.  Ranges 0..NODES-1 are the windows'
  // insertion steps, NODES..2*NODES-1 their target entries.
  auto locate = [&](int rbeg, uint32_t e, uint32_t& start) -> int {
    int r = rbeg;
    start = 0;
    while (e >= start + pcnt[r]) {
      start += pcnt[r];
      ++r;
    }
    return r;
  };
  // a patch of range r with target slot x and source xs: its level (bits
  // 16..) and LDS position (bits 0..15), or NONE, and in `src` its
  // pass-input element relative to sMa
  auto patch_meta = [&](int r, uint32_t x, uint32_t xs, uint32_t& src) -> uint32_t {
    const uint32_t* nr = td.node[r < NODES ? r : r - NODES];
    src = 0;
    if (xs == NONE || xs >= nr[dN] || x < nr[dU0] || x >= nr[dU1]) return NONE;
    src = nr[dSrel] + xs;
    return (nr[dLi] << 16) | (nr[dD] + x);
  };
  // patch e's target (an insertion step's own slot) and source index loads;
  // tl: a target entry (its range is NODES or above)
  auto patch_fetch = [&](bool tl, int r, uint32_t e, uint32_t start, uint32_t& x, uint32_t& xs) {
    const uint64_t idx = (uint64_t)pbase[r] + (e - start);
    if (!tl) {
      x = max(td.node[r][dU0], td.node[r][dP]) + (e - start);
      xs = a.tail_xsrc[idx];
    } else {
      x = a.pool_x[idx];
      xs = a.pool_xsrc[idx];
    }
  };
  auto patch_at = [&](int rbeg, uint32_t e, uint32_t& meta) -> uint32_t {
    uint32_t start, x, xs, src;
    const int r = locate(rbeg, e, start);
    patch_fetch(rbeg != 0, r, e, start, x, xs);
    meta = patch_meta(r, x, xs, src);
    return src;
  };
  // the first PK patches of each kind per thread, fetched ahead of the
  // levels: every index load issued before any is used, then the values
  uint32_t pm[2 * PK];
  R pv[2 * PK];
  {
    uint32_t px[2 * PK], pxs[2 * PK];
    int pr[2 * PK];
#pragma unroll
    for (int i = 0; i < 2 * PK; ++i) {
      const bool tl = i >= PK;
      const uint32_t e = tid + NT * (uint32_t)(i % PK);
      pr[i] = -1;
      if (e < (tl ? ptot : stot)) {
        uint32_t start;
        pr[i] = locate(tl ? NODES : 0, e, start);
        patch_fetch(tl, pr[i], e, start, px[i], pxs[i]);
      }
    }
#pragma unroll
    for (int i = 0; i < 2 * PK; ++i) {
      // every thread loads, element 0 of the merge when it has no patch (no
      // branch around the load, so nothing waits for it before its use)
      uint32_t src = 0;
      pm[i] = NONE;
      if (pr[i] >= 0) pm[i] = patch_meta(pr[i], px[i], pxs[i], src);
      pv[i] = reinterpret_cast<const R*>(XM)[src];
    }
  }
  // the staged runs land in LDS
  if (a.vec_ok) {
#pragma unroll
    for (int i = 0; i < PV; ++i)
      if (spos[i] < (uint32_t)BUF) *reinterpret_cast<uint4*>(&buf[0][spos[i]]) = sv[i];
  } else {
    // element loads: the regions are the runs themselves
    for (uint32_t v = tid; v < nvec; v += NT) {
      int r = 0;
#pragma unroll
      for (int h = NRUN / 2; h >= 1; h >>= 1) r += v >= td.run_vpre[r + h] ? h : 0;
      const uint32_t rel = v - td.run_vpre[r];
      buf[0][td.run_base[r] + rel] = XM[td.run_grel[r] + rel];
    }
  }
  __syncthreads();

  // 3. the levels, bottom up: one interleave from one buffer into the other
  //    (4 slots of one flip word per thread and step), then the insertion
  //    loop's slots of the level
#pragma unroll
  for (int li = 0; li < LAM; ++li) {
    const E* src = buf[li & 1];
    E* dst = buf[(li + 1) & 1];
    const R* srcR = reinterpret_cast<const R*>(src);
    R* dstR = reinterpret_cast<R*>(dst);
    // level li is depth LAM-1-li of the tree (breadth first: the top first)
    const uint32_t e0 = uniform_u32(td.dep_tb[LAM - 1 - li]);
    const uint32_t ne = uniform_u32(td.dep_tb[LAM - li]) - e0;
    if constexpr (sizeof(E) == 4) {
      // groups of GS consecutive slots per thread (GPW groups to a flip
      // word): one entry read and one pair of counts per group.  The lanes
      // of a wave read A and B near 64 / GS * (lane) words apart, so fewer
      // slots per group spread a read over more LDS banks.
      constexpr uint32_t GS = kPassGroup4, GPW = 32u / GS;
      const uint32_t* src4 = reinterpret_cast<const uint32_t*>(src);
      for (uint32_t q = tid; q < GPW * ne; q += NT) {
        const uint2 t = td.tab[e0 + q / GPW];
        const uint32_t G = 32u + GS * q;
        const uint32_t sh = GS * (q % GPW);
        const uint32_t lo = (1u << sh) - 1u;
        // byte offsets of the next A and B sources (the zeros before the
        // group are its offset in the word less the ones)
        const uint32_t ones = (uint32_t)__popc(t.x & lo);
        uint32_t za = 4u * ((t.y & 0xFFFFu) + sh - ones);
        uint32_t ob = 4u * ((t.y >> 16) + ones);
        const uint32_t bg = t.x >> sh;
        const char* srcb = reinterpret_cast<const char*>(src4);
        uint32_t v[GS];
#pragma unroll
        for (int j = 0; j < (int)GS; ++j) {
          // all ones on a 1 flip: take B at ob, else A at za (the mask kept
          // opaque so that the choice stays one bit select)
          uint32_t msk = (uint32_t)__builtin_amdgcn_sbfe((int)bg, (uint32_t)j, 1u);
          asm volatile("" : "+v"(msk));
          const uint32_t m4 = msk << 2;
          v[j] = *reinterpret_cast<const uint32_t*>(srcb + ((ob & msk) | (za & ~msk)));
          za += 4u + m4;
          ob -= m4;
        }
        if constexpr (GS == 2) {
          *reinterpret_cast<uint2*>(&dst[G]) = make_uint2(v[0], v[1]);
        } else {
          uint4* d4 = reinterpret_cast<uint4*>(&dst[G]);
#pragma unroll
          for (int h = 0; h < (int)GS / 4; ++h) d4[h] = make_uint4(v[4 * h], v[4 * h + 1], v[4 * h + 2], v[4 * h + 3]);
        }
      }
    } else
    for (uint32_t q = tid; q < 8u * ne; q += NT) {
      const uint2 t = td.tab[e0 + (q >> 3)];
      const uint32_t G = 32u + 4u * q;
      const uint32_t s = G & 31u;
      const uint32_t lo = (1u << s) - 1u;
      uint32_t za = (t.y & 0xFFFFu) + (uint32_t)__popc(~t.x & lo);
      uint32_t ob = (t.y >> 16) + (uint32_t)__popc(t.x & lo);
      const uint32_t b4 = t.x >> s;
      uint32_t fr[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        // all ones on a 1 flip: take B at ob, else A at za
        const uint32_t msk = (uint32_t)__builtin_amdgcn_sbfe((int)b4, (uint32_t)j, 1u);
        fr[j] = (ob & msk) | (za & ~msk);
        za += 1u + msk;
        ob -= msk;
      }
      const R a0 = srcR[fr[0]], a1 = srcR[fr[1]], a2 = srcR[fr[2]], a3 = srcR[fr[3]];
      dstR[G] = a0;
      dstR[G + 1] = a1;
      dstR[G + 2] = a2;
      dstR[G + 3] = a3;
    }
    __syncthreads();
    // insertion-loop slots of this level inside the tile
#pragma unroll
    for (int i = 0; i < 2 * PK; ++i)
      if (pm[i] != NONE && (pm[i] >> 16) == (uint32_t)li) dstR[pm[i] & 0xFFFFu] = pv[i];
    for (uint32_t e = NT * PK + tid; e < stot; e += NT) {
      uint32_t meta;
      const uint32_t srcx = patch_at(0, e, meta);
      if (meta != NONE && (meta >> 16) == (uint32_t)li) dst[meta & 0xFFFFu] = XM[srcx];
    }
    for (uint32_t e = NT * PK + tid; e < ptot; e += NT) {
      uint32_t meta;
      const uint32_t srcx = patch_at(NODES, e, meta);
      if (meta != NONE && (meta >> 16) == (uint32_t)li) dst[meta & 0xFFFFu] = XM[srcx];
    }
    __syncthreads();
  }

  // 4. store the top window: its slots u0.. sit at positions 32.. (u0 is a
  //    multiple of T, hence of 32)
  const E* fin = buf[LAM & 1] + 32;
  E* out = Z + sM + u0top;
  const bool vout = a.vec_ok && ((sM + u0top) % VE) == 0;
  if (vout) {
    for (uint32_t o = VE * tid; o < len; o += VE * NT) {
      if (o + VE <= len) {
        *reinterpret_cast<uint4*>(out + o) = *reinterpret_cast<const uint4*>(&fin[o]);
      } else {
        for (uint32_t k = o; k < len; ++k) out[k] = fin[k];
      }
    }
  } else {
    for (uint32_t o = tid; o < len; o += NT) out[o] = fin[o];
  }
}

// Workgroups are dealt to the 8 XCDs round robin; give each XCD a
// contiguous eighth of the tiles so that the tiles of one merge share an L2,
// which then also serves most insertion-loop fetches within the merge.
__device__ __forceinline__ uint32_t xcd_tile_of(uint32_t ntiles) {
  const uint32_t q = ntiles >> 3, r = ntiles & 7u;
  const uint32_t x = blockIdx.x & 7u, i = blockIdx.x >> 3;
  return x * q + min(x, r) + i;
}

// Threads of a descriptor build (measured at 2^30: 128 builds a tile's
// descriptor with the least time beside the leaf kernel; 64 and 256 take
// 0.3 ms more per shuffle, 512 0.9 ms)
constexpr int kDescThreads = 128;

template <typename E, int T, int LAM, int NT>
__global__ void __launch_bounds__(NT) pass_kernel(GroupArgs a) {
  if (blockIdx.x >= a.ntiles) return;
  pass_body<E, T, LAM, NT>(a, xcd_tile_of(a.ntiles));
}

template <typename E, int T, int LAM>
__global__ void __launch_bounds__(kDescThreads) pass_desc_kernel(GroupArgs a) {
  if (blockIdx.x >= a.ntiles) return;
  desc_body<E, T, LAM, kDescThreads>(a, blockIdx.x, a.desc + (uint64_t)blockIdx.x * a.desc_words);
}

// The same pass of many arrays in one launch: job j owns tiles
// [tpre[j], tpre[j+1]) of the ntiles = tpre[njobs] tiles.
__device__ __forceinline__ uint32_t job_of(const uint32_t* __restrict__ tpre, uint32_t njobs, uint32_t tile) {
  uint32_t lo = 0, hi = njobs;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (tpre[mid] <= tile) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <typename E, int T, int LAM, int NT>
__global__ void __launch_bounds__(NT) pass_multi_kernel(const GroupArgs* __restrict__ jobs,
                                                        const uint32_t* __restrict__ tpre, uint32_t njobs,
                                                        uint32_t ntiles) {
  if (blockIdx.x >= ntiles) return;
  const uint32_t tile = xcd_tile_of(ntiles);
  const uint32_t j = job_of(tpre, njobs, tile);
  pass_body<E, T, LAM, NT>(jobs[j], tile - tpre[j]);
}

template <typename E, int T, int LAM>
__global__ void __launch_bounds__(kDescThreads) pass_desc_multi_kernel(const GroupArgs* __restrict__ jobs,
                                                                       const uint32_t* __restrict__ tpre,
                                                                       uint32_t njobs, uint32_t ntiles) {
  if (blockIdx.x >= ntiles) return;
  const uint32_t j = job_of(tpre, njobs, blockIdx.x);
  const GroupArgs& a = jobs[j];
  const uint32_t tile = blockIdx.x - tpre[j];
  desc_body<E, T, LAM, kDescThreads>(a, tile, a.desc + (uint64_t)tile * a.desc_words);
}

// Tile shapes (slots per tile, threads per workgroup) per element size; the
// first is the default, MS_PASS_TILE=<slots> picks another.  4-byte arrays of
// 2^26 elements or more take 8192-slot tiles of 1024 threads: half the tiles
// of the default, so half the descriptors for the plan to build (measured at
// 2^30: 27.3 against 27.9 ms per shuffle, the passes themselves 6 % slower).
// A tuning choice only: the permutation does not depend on it.
struct TileShape {
  int T, NT;
};
static const TileShape kShapes4[] = {{3584, 512}, {4096, 512}, {2048, 256}, {8192, 1024}, {7168, 1024}};
static const TileShape kShapes8[] = {{2048, 512}, {1792, 512}, {1024, 256}, {4096, 1024}};
static const TileShape kShapes16[] = {{1024, 256}, {640, 256}, {512, 128}, {2048, 512}};
constexpr uint64_t kBigTileN = 1ull << 26;

static int shape_count(uint32_t eb) { return eb == 4 ? (int)(sizeof kShapes4 / sizeof kShapes4[0]) : 4; }
static const TileShape* shapes_of(uint32_t eb) { return eb == 4 ? kShapes4 : eb == 8 ? kShapes8 : kShapes16; }

// The tile of a pass over an array of n elements of eb bytes.
int pass_group_tile(uint32_t eb, uint64_t n) {
  static const int want = [] {
    const char* e = getenv("MS_PASS_TILE");
    return e ? atoi(e) : 0;
  }();
  const TileShape* t = shapes_of(eb);
  for (int i = 0; i < shape_count(eb); ++i)
    if (t[i].T == want) return t[i].T;
  if (eb == 4 && n >= kBigTileN) return 8192;
  return t[0].T;
}

static TileShape shape_of(uint32_t eb, uint32_t T) {
  const TileShape* t = shapes_of(eb);
  for (int i = 0; i < shape_count(eb); ++i)
    if ((uint32_t)t[i].T == T) return t[i];
  return t[0];
}

// Calls f.template go<E, T, LAM, NT>() for the element size's selected shape.
template <typename E, int T, int NT, typename F>
static void with_lam(int lam, F& f) {
  if (lam == 1) f.template go<E, T, 1, NT>();
  else if (lam == 2) f.template go<E, T, 2, NT>();
  else if (lam == 3) f.template go<E, T, 3, NT>();
  else f.template go<E, T, 4, NT>();
}

template <typename F>
static void with_shape(uint32_t eb, uint32_t T, int lam, F& f) {
  const TileShape sh = shape_of(eb, T);
  if (eb == 4) {
    if (sh.T == 4096) with_lam<uint32_t, 4096, 512>(lam, f);
    else if (sh.T == 2048) with_lam<uint32_t, 2048, 256>(lam, f);
    else if (sh.T == 8192) with_lam<uint32_t, 8192, 1024>(lam, f);
    else if (sh.T == 7168) with_lam<uint32_t, 7168, 1024>(lam, f);
    else with_lam<uint32_t, 3584, 512>(lam, f);
  } else if (eb == 8) {
    if (sh.T == 1792) with_lam<uint64_t, 1792, 512>(lam, f);
    else if (sh.T == 1024) with_lam<uint64_t, 1024, 256>(lam, f);
    else if (sh.T == 4096) with_lam<uint64_t, 4096, 1024>(lam, f);
    else with_lam<uint64_t, 2048, 512>(lam, f);
  } else {
    if (sh.T == 640) with_lam<uint4, 640, 256>(lam, f);
    else if (sh.T == 512) with_lam<uint4, 512, 128>(lam, f);
    else if (sh.T == 2048) with_lam<uint4, 2048, 512>(lam, f);
    else with_lam<uint4, 1024, 256>(lam, f);
  }
}

struct DescWordsF {
  uint32_t w = 0;
  template <typename E, int T, int LAM, int NT>
  void go() { w = desc_words<T, LAM>(); }
};

struct LaunchPassF {
  const GroupArgs* a;
  uint64_t grid;
  hipStream_t st;
  bool desc;
  template <typename E, int T, int LAM, int NT>
  void go() {
    if (desc) hipLaunchKernelGGL((pass_desc_kernel<E, T, LAM>), dim3((uint32_t)grid), dim3(kDescThreads), 0, st, *a);
    else hipLaunchKernelGGL((pass_kernel<E, T, LAM, NT>), dim3((uint32_t)grid), dim3(NT), 0, st, *a);
  }
};

struct LaunchPassMultiF {
  const GroupArgs* jobs;
  const uint32_t* tpre;
  uint32_t njobs, ntiles;
  hipStream_t st;
  bool desc;
  template <typename E, int T, int LAM, int NT>
  void go() {
    if (desc)
      hipLaunchKernelGGL((pass_desc_multi_kernel<E, T, LAM>), dim3(ntiles), dim3(kDescThreads), 0, st, jobs, tpre,
                         njobs, ntiles);
    else
      hipLaunchKernelGGL((pass_multi_kernel<E, T, LAM, NT>), dim3(ntiles), dim3(NT), 0, st, jobs, tpre, njobs, ntiles);
  }
};

uint32_t pass_desc_words(uint32_t eb, uint32_t T, int lam) {
  DescWordsF f;
  with_shape(eb, T, lam, f);
  return f.w;
}

void launch_pass_group(const GroupArgs& a, int lam, uint32_t eb, uint32_t T, uint64_t grid, hipStream_t st) {
  LaunchPassF f{&a, grid, st, false};
  with_shape(eb, T, lam, f);
}

void launch_pass_desc(const GroupArgs& a, int lam, uint32_t eb, uint32_t T, uint64_t grid, hipStream_t st) {
  LaunchPassF f{&a, grid, st, true};
  with_shape(eb, T, lam, f);
}

// (batched arrays hold at most 2^21 elements: the default tile)
void launch_pass_group_multi(const GroupArgs* jobs, const uint32_t* tpre, uint32_t njobs, uint32_t ntiles, int lam,
                             uint32_t eb, hipStream_t st) {
  if (!ntiles) return;
  LaunchPassMultiF f{jobs, tpre, njobs, ntiles, st, false};
  with_shape(eb, (uint32_t)pass_group_tile(eb, 0), lam, f);
}

void launch_pass_desc_multi(const GroupArgs* jobs, const uint32_t* tpre, uint32_t njobs, uint32_t ntiles, int lam,
                            uint32_t eb, hipStream_t st) {
  if (!ntiles) return;
  LaunchPassMultiF f{jobs, tpre, njobs, ntiles, st, true};
  with_shape(eb, (uint32_t)pass_group_tile(eb, 0), lam, f);
}

}  // namespace ms
