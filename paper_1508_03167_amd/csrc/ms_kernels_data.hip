// ms_kernels_data.hip -- the kernels that move elements.
//
//   leaf_kernel   one workgroup per super-block of 2^lds_levels leaves:
//                 Fisher-Yates of every leaf (Algorithm 1) in LDS, then the
//                 first lds_levels merge levels (Algorithm 2) in LDS.
//   merge_pass    one HBM level: every output slot t of a merge takes, by the
//                 coin-flip loop's stable interleave, A[r0(t)] on a 0 flip and
//                 B[t - r0(t)] on a 1 flip, r0(t) = zeros among flips 0..t-1;
//                 slots from the break step P on take the side that is left,
//                 in order.  A and B runs are staged through LDS.
//   patch         the same level's insertion-loop slots, resolved by the plan.
//
// Fisher-Yates in parallel.  Algorithm 1 runs r = b-1 down to 1 with
// swap(T[r], T[j_r]), j_r <= r.  Slot r is final after step r and receives
// what slot j_r held just before step r.  A slot x < r has been written since
// the start only by steps r' > r that target it (j_r' = x), the latest being
// the smallest such r', which left what slot r' held just before step r'.  So
// with up(x) = min{r' > x : j_r' = x} and top() following up() to its end:
//   F[r] = T0[top(nxt(r))] if nxt(r) = min{r' > r : j_r' = j_r} exists,
//          T0[j_r] otherwise;     F[0] = T0[top(0)].
// The steps that target a slot are chained in increasing order by atomic
// exchanges on the slot's LDS word, so up() and nxt() come straight from the
// exchanges' return values; top() is found by pointer jumping.
//
// Insertion loop in LDS.  A merge's tail steps i = P..N-1 run as groups of
// 64 steps on one wave: within a group each lane resolves its step against
// the earlier lanes of the group (the latest earlier lane targeting the same
// slot, else the lane whose own step filled that slot, else the value before
// the group), then every touched slot is written once.
#include "ms_device.hpp"
#include "ms_plan.hpp"

namespace ms {

constexpr int kLeafMaxMerges = 64;  // at most 2^6 leaves per super-block


template <typename E>
__device__ __forceinline__ E ident_value(uint64_t i);
template <>
__device__ __forceinline__ uint32_t ident_value<uint32_t>(uint64_t i) { return (uint32_t)i; }
template <>
__device__ __forceinline__ uint64_t ident_value<uint64_t>(uint64_t i) { return i; }
template <>
__device__ __forceinline__ uint4 ident_value<uint4>(uint64_t i) {
  return make_uint4((uint32_t)i, (uint32_t)(i >> 32), 0u, 0u);
}

template <int SCAP>
struct MergeAux {
  static constexpr int kWords = SCAP / 32 + 8 * kLeafMaxMerges + 8;
  uint32_t words[kWords];
  uint32_t wpre[kWords];
};

__device__ __forceinline__ uint32_t get16(uint32_t packed, int half) { return (packed >> (16 * half)) & 0xFFFFu; }

// Runs body(i, x, w, ok) for the slots x = lt + tpl * i (i < SPT) of the
// thread's leaf, without branches: ok tells whether slot x exists (x < b), w
// is the word of slot x if it does and the spare word `dummy` otherwise, so
// that a body that addresses its own slot through w and guards everything
// else by ok runs straight through.  The opaque copy of lt keeps the
// compiler from computing every slot's address once and holding it across
// phases.
template <int SPT, typename Body, int I0 = 0, int I1 = SPT>
__device__ __forceinline__ void for_slots(uint32_t lt, uint32_t tpl, uint32_t lb, uint32_t b, uint32_t dummy,
                                          Body&& body) {
  uint32_t x0 = lt;
  asm volatile("" : "+v"(x0));
#pragma unroll
  for (int i = I0; i < I1; ++i) {
    const uint32_t x = x0 + tpl * (uint32_t)i;
    const bool ok = x < b;
    body(i, x, ok ? lb + x : dummy, ok);
  }
}

// The same over the slots in two halves, each read completely before it is
// written (half the registers of reading every slot first).
template <int SPT, typename Read, typename Write>
__device__ __forceinline__ void for_slots_rw(uint32_t lt, uint32_t tpl, uint32_t lb, uint32_t b, uint32_t dummy,
                                             Read&& rd, Write&& wr) {
  constexpr int H = (SPT + 1) / 2;
  for_slots<SPT, Read&, 0, H>(lt, tpl, lb, b, dummy, rd);
  for_slots<SPT, Write&, 0, H>(lt, tpl, lb, b, dummy, wr);
  for_slots<SPT, Read&, H, SPT>(lt, tpl, lb, b, dummy, rd);
  for_slots<SPT, Write&, H, SPT>(lt, tpl, lb, b, dummy, wr);
}

__device__ __forceinline__ uint32_t set16(uint32_t packed, int half, uint32_t v) {
  return half ? (packed & 0xFFFFu) | (v << 16) : (packed & 0xFFFF0000u) | (v & 0xFFFFu);
}

// Fisher-Yates of every leaf of the super-block at once (Algorithm 1 per leaf).
// Before the elements are loaded, the LDS data region holds one 32-bit word
// per super-block slot: first the slot's draw, then a 16-bit list head
// (later up()) and the step's 16-bit link (later nxt(), or its draw when no
// later step targets the same slot).  For the draws each thread owns blocks
// of 4 consecutive steps of one leaf (the steps whose draws share one Philox
// block); for everything else it owns the slots x = lt + tpl * i of its leaf,
// so that the lanes of a wave touch consecutive LDS words.  It returns,
// packed two per register, the leaf-relative source F of each of those
// slots.
template <int BPT, int SPT, int NT>
__device__ __forceinline__ void leaf_fy_sources(uint16_t* head, uint32_t lb, uint32_t b, uint32_t dummy, uint32_t u,
                                                uint32_t lt, uint32_t tpl, Key key, uint32_t* bits, uint32_t* status,
                                                uint32_t (&F)[(SPT + 1) / 2]) {
  constexpr uint32_t NONE = 0xFFFFu;
  uint16_t* const half = head;  // the lists' words, as 16-bit halves
#define HED(y) half[2 * (y)]
#define LNK(y) half[2 * (y) + 1]
  // 1. the draws j_r, r = 1..b-1, of this thread's blocks (r = 4g..4g+3,
  //    g = lt + tpl*k).  The primary words go to the data region first (one
  //    word per slot); then each lane runs the Fast Dice Roller of its draws
  //    one after the other, so that a wave waits for the lane with the most
  //    rounds in total rather than for the slowest lane of every draw.  The
  //    result replaces the word.
  uint32_t* W = reinterpret_cast<uint32_t*>(head);
  {
    // The first round of every draw as its block comes out of Philox (it
    // takes the top bitlen(r) bits of the word and ends unless they exceed
    // r): the word gets the result, or the raw word if the draw stays open;
    // the open draws then run to the end one after the other per lane.
    constexpr uint32_t QN = 4 * BPT;
    static_assert(QN <= 64, "open draws are tracked in a 64-bit mask");
    uint64_t open = 0;
    uint32_t nb = 0;
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
      const uint32_t g = lt + tpl * k;
      if (4 * g < b) {
        const W4 db = draw_block(g, u, 0, key);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const uint32_t r = 4 * g + e;
          const bool ok = r >= 1 && r < b;
          const uint32_t bk = 32 - __clz(r | 1u);
          const uint32_t x = db.w[e] >> (32 - bk);
          const bool first = x <= r;
          W[ok ? lb + r : dummy] = first ? x : db.w[e];
          nb += ok && first ? bk : 0u;
          open |= (uint64_t)(ok && !first) << (4 * k + e);
        }
      }
    }
    *bits += nb;
    if (open) {
      uint32_t r = 0, w = 0, v = 0, c = 0, used = 0, left = 0, kk = 0, bk = 0;
      auto next = [&]() {
        const uint32_t q = (uint32_t)__builtin_ctzll(open);
        open &= open - 1;
        r = 4 * (lt + tpl * (q >> 2)) + (q & 3u);
        w = W[lb + r];
        bk = 32 - __clz(r);
        kk = r + 1;
        // state after the rejected first round
        v = (1u << bk) - kk;
        c = (w >> (32 - bk)) - kk;
        used = bk;
        left = 32 - bk;
      };
      next();
#pragma unroll 1
      for (;;) {
        bool done = true;
        uint32_t res = 0;
        int jump = (int)bk - (32 - __clz(v));
        if ((v << jump) <= kk - 1) jump += 1;
        if (jump > (int)left) {
          const Draw d = fdr_draw_slow((uint64_t)kk, w, 0, u, r, key);
          res = d.v;
          used = d.bits;
        } else {
          const uint32_t x = (w >> (left - jump)) & ((1u << jump) - 1u);
          left -= jump;
          used += (uint32_t)jump;
          v <<= jump;
          c = (c << jump) | x;
          if (c < kk) {
            res = c;
          } else {
            v -= kk;
            c -= kk;
            done = false;
          }
        }
        if (done) {
          W[lb + r] = res;
          *bits += used;
          if (!open) break;
          next();
        }
      }
    }
  }
  __syncthreads();
  // 2. up(x) = least step > x targeting x, nxt(r) = least step > r
  //    targeting j_r.  One 32-bit word per super-block slot y: the high half
  //    holds j_y while the steps are pushed onto their slots' lists, the low
  //    half the head of y's list.  A push of step r is an atomic exchange of
  //    word j_r that keeps its high half, so the old head comes back.  The
  //    steps of a leaf are pushed in increasing order (each wave of the leaf
  //    takes one contiguous range of steps, the waves one after the other,
  //    a wave's lanes in step order; the LDS applies one wave's exchanges of
  //    one address in lane order), so the head a push returns is the
  //    previous step targeting the same slot: its nxt() is the pushed step,
  //    and the first push onto slot y gives up(y) (the second one when the
  //    first is step y itself).  No list is walked.  Pushes per lane: at most
  //    ceil(ceil(b / ranges) / lanes) <= SCAP / NT + 1 <= 4 * BPT, since a
  //    leaf holds at most SCAP / 2^lds_levels + 1 slots.
  // (each thread rewrites the words of its own slots: j_r, none for step 0)
  // Every loop below runs straight through: a lane whose slot or step does
  // not exist works on the spare word `dummy` (its two halves as HED/LNK)
  // and its results are not used.
  {
    uint32_t v[SPT];
    for_slots_rw<SPT>(lt, tpl, lb, b, dummy, [&](int i, uint32_t, uint32_t w, bool) { v[i] = W[w]; },
                      [&](int i, uint32_t r, uint32_t w, bool) { W[w] = ((r >= 1 ? v[i] : NONE) << 16) | NONE; });
  }
  __syncthreads();
  constexpr int ITER = 4 * BPT;  // pushes per lane, at most
  const uint32_t lpp = tpl < 64 ? tpl : 64u;  // lanes pushing one range
  const uint32_t wpl = tpl / lpp;             // ranges (waves) per leaf
  const uint32_t wl = lt / lpp, li = lt % lpp;
  const uint32_t span = (((b + wpl - 1) / wpl + lpp - 1) / lpp) * lpp;
  const uint32_t r0 = wl * span + li;
  const uint32_t r1 = min(b, (wl + 1) * span);
  uint32_t OLD[(ITER + 1) / 2];  // per pushed step, packed two per register: the head it replaced
  for (uint32_t ph = 0; ph < wpl; ++ph) {
    if (wl == ph) {
      // in halves of the steps: every target first, then every target's
      // high half (no push changes a high half), then the exchanges, which
      // the LDS applies in program order
      constexpr int H = (ITER + 1) / 2;
#pragma unroll
      for (int h0 = 0; h0 < ITER; h0 += H) {
        uint32_t wy[H], xv[H];
#pragma unroll
        for (int t = 0; t < H; ++t) {
          const uint32_t r = r0 + lpp * (h0 + t);
          const bool ok = h0 + t < ITER && r >= 1 && r < r1;
          const uint32_t y = W[ok ? lb + r : dummy] >> 16;
          wy[t] = ok ? lb + y : dummy;
        }
#pragma unroll
        for (int t = 0; t < H; ++t) xv[t] = (W[wy[t]] & 0xFFFF0000u) | (r0 + lpp * (h0 + t));
#pragma unroll
        for (int t = 0; t < H; ++t) {
          if (h0 + t >= ITER) break;
          const uint32_t r = r0 + lpp * (h0 + t);
          const bool ok = r >= 1 && r < r1;
          const uint32_t x = atomicExch(&W[wy[t]], xv[t]) & 0xFFFFu;
          const uint32_t old = ok ? x : NONE;
          if ((h0 + t) & 1) OLD[(h0 + t) >> 1] |= old << 16;
          else OLD[(h0 + t) >> 1] = old;
        }
      }
    }
    __syncthreads();
  }
  // The first push onto slot y sets up(y), unless it is step y itself: then
  // the second push (if any) does.  A pushed step's link starts as its own
  // target j_r with bit 15 set (no later step on its slot: its source is
  // j_r; j_r = r marks a self push); the step pushed next onto the same slot
  // then makes itself the link.
  constexpr uint32_t NOLATER = 0x8000u;
  {
    // (every target is read before the first write; the writes touch the
    // heads of targets and the links of this lane's own steps)
    constexpr int H = (ITER + 1) / 2;
#pragma unroll
    for (int h0 = 0; h0 < ITER; h0 += H) {
      uint32_t y[H];
#pragma unroll
      for (int k = 0; k < H; ++k) {
        const int t = h0 + k;
        const uint32_t r = r0 + lpp * t;
        y[k] = t < ITER ? W[r >= 1 && r < r1 ? lb + r : dummy] >> 16 : 0u;
      }
#pragma unroll
      for (int k = 0; k < H; ++k) {
        const int t = h0 + k;
        if (t >= ITER) break;
        const uint32_t r = r0 + lpp * t;
        const bool ok = r >= 1 && r < r1;
        const uint32_t old = get16(OLD[t >> 1], t & 1);
        HED(ok && old == NONE ? lb + y[k] : dummy) = (uint16_t)(r != y[k] ? r : NONE);
        LNK(ok ? lb + r : dummy) = (uint16_t)(y[k] | NOLATER);
      }
    }
  }
  __syncthreads();
  {
    // Each old step is the predecessor of exactly one pushed step, so its
    // word is this lane's alone here: all of them are read, then written.
    // Pushes onto one slot came in increasing step order; a lane that sees
    // otherwise reports it (bit 3), the lists are then unordered.
    bool unordered = false;
    constexpr int H = (ITER + 1) / 2;
#pragma unroll
    for (int h0 = 0; h0 < ITER; h0 += H) {
      uint32_t wv[H];
#pragma unroll
      for (int k = 0; k < H; ++k) {
        const int t = h0 + k;
        if (t >= ITER) break;
        const uint32_t r = r0 + lpp * t;
        const uint32_t old = get16(OLD[t >> 1], t & 1);
        const bool ok = r >= 1 && r < r1 && old != NONE;
        wv[k] = W[ok ? lb + old : dummy];
      }
#pragma unroll
      for (int k = 0; k < H; ++k) {
        const int t = h0 + k;
        if (t >= ITER) break;
        const uint32_t r = r0 + lpp * t;
        const uint32_t old = get16(OLD[t >> 1], t & 1);
        const bool ok = r >= 1 && r < r1 && old != NONE;
        unordered |= ok && old > r;
        const uint32_t lk = wv[k] >> 16, hd = wv[k] & 0xFFFFu;
        // head (low half) and link (high half) of the old step's word
        W[ok ? lb + old : dummy] = (r << 16) | (lk == (old | NOLATER) ? r : hd);
      }
    }
    if (unordered) atomicOr(status, 8u);
  }
  __syncthreads();
  // 4. top() of every slot: the end of its chain of up() links (NONE if it
  //    has no up()), then F[r] = top(nxt(r)) or j_r, F[0] = top(0).  F
  //    first takes each slot's link (nxt(x), or j_x with bit 15 set), which
  //    frees the link halves; the head halves keep the up() links, which
  //    nothing changes from here on, so every lane follows the chains of its
  //    own slots with no barrier: two steps for every slot at once (most
  //    chains are that short), then the rest one slot at a time, writing
  //    top() to the slot's link half.
  static_assert(SPT <= 64, "live slots are tracked in a 64-bit mask");
#pragma unroll
  for (int i = 0; i < (SPT + 1) / 2; ++i) F[i] = 0u;
  for_slots<SPT>(lt, tpl, lb, b, dummy, [&](int i, uint32_t x, uint32_t w, bool) {
    const uint32_t l = LNK(w);
    F[i >> 1] = set16(F[i >> 1], i & 1, x >= 1 ? l : 0u);
  });
  __syncthreads();
  {
    uint64_t live = 0;
    {
      // in two halves of the slots, each: every head, then every head's
      // head, then the links
      uint32_t t[SPT], tt[SPT];
      auto rd1 = [&](int i, uint32_t, uint32_t w, bool) { t[i] = HED(w); };
      auto rd2 = [&](int i, uint32_t, uint32_t, bool ok) { tt[i] = HED(ok && t[i] != NONE ? lb + t[i] : dummy); };
      auto wr = [&](int i, uint32_t, uint32_t w, bool ok) {
        const bool two = ok && t[i] != NONE && tt[i] != NONE;
        LNK(w) = (uint16_t)(two ? tt[i] : t[i]);
        live |= (uint64_t)two << i;
      };
      constexpr int H = (SPT + 1) / 2;
      for_slots<SPT, decltype(rd1)&, 0, H>(lt, tpl, lb, b, dummy, rd1);
      for_slots<SPT, decltype(rd2)&, 0, H>(lt, tpl, lb, b, dummy, rd2);
      for_slots<SPT, decltype(wr)&, 0, H>(lt, tpl, lb, b, dummy, wr);
      for_slots<SPT, decltype(rd1)&, H, SPT>(lt, tpl, lb, b, dummy, rd1);
      for_slots<SPT, decltype(rd2)&, H, SPT>(lt, tpl, lb, b, dummy, rd2);
      for_slots<SPT, decltype(wr)&, H, SPT>(lt, tpl, lb, b, dummy, wr);
    }
    while (live) {
      const int q = __builtin_ctzll(live);
      live &= live - 1;
      const uint32_t x = lb + lt + tpl * (uint32_t)q;
      uint32_t cur = LNK(x);
      for (;;) {
        const uint32_t nx = HED(lb + cur);
        if (nx == NONE) break;
        cur = nx;
      }
      LNK(x) = (uint16_t)cur;
    }
  }
  __syncthreads();
  // the link half of x's word now holds the end of x's up() chain, or NONE
  // if x has no up().  Step x's link: a later step on its slot, or its own
  // target with bit 15 set; slot 0 starts from itself.  A slot that does not
  // exist gets source 0.
  for_slots<SPT>(lt, tpl, lb, b, dummy, [&](int i, uint32_t, uint32_t, bool ok) {
    const uint32_t lk = get16(F[i >> 1], i & 1);
    const uint32_t top = LNK(lb + (lk & ~NOLATER));
    uint32_t f = (lk & NOLATER) ? lk & ~NOLATER : (top != NONE ? top : lk);
    F[i >> 1] = set16(F[i >> 1], i & 1, ok ? f : 0u);
  });
  __syncthreads();
#undef HED
#undef LNK
}

// Insertion loop of one merge [s0, s0+N) in LDS by one wave, groups of 64
// steps.  `seen` is a zeroed bitmap over the super-block's slots.  A group
// whose targets all lie below the group and are pairwise distinct touches
// disjoint slots, so its swaps commute and run at once; other groups resolve
// their steps against each other lane by lane.
template <typename E>
__device__ __forceinline__ void lds_merge_tail(E* data, uint32_t* seen, uint32_t* dup, uint32_t s0, uint32_t N, uint32_t P,
                                               uint32_t L, uint32_t gm, Key key, uint32_t* bits) {
  const int lane = threadIdx.x & 63;
  for (uint32_t i0 = P; i0 < N; i0 += 64) {
    const uint32_t i = i0 + lane;
    const bool act = i < N;
    uint32_t j = kNone32;
    if (act) {
      const W4 db = draw_block(i >> 2, gm, L, key);
      const Draw dr = fdr_draw((uint64_t)i + 1, pick(db, i & 3), L, gm, i, key);
      j = dr.v;
      *bits += dr.bits;
    }
    bool clash = act && j >= i0;
    if (act && j < i0) {
      const uint32_t bit = 1u << ((s0 + j) & 31);
      const uint32_t old = atomicOr(&seen[(s0 + j) >> 5], bit);
      clash = (old & bit) != 0;
    }
    const bool any_clash = __any(clash);
    if (act && j < i0) atomicAnd(&seen[(s0 + j) >> 5], ~(1u << ((s0 + j) & 31)));
    if (!any_clash) {
      E ai, aj;
      if (act) {
        ai = data[s0 + i];
        aj = data[s0 + j];
      }
      if (act) {
        data[s0 + i] = aj;
        data[s0 + j] = ai;
      }
      continue;
    }
    // Only lanes that target a slot of the group, or share their target with
    // another lane, can depend on one another: a lane that found its
    // target's bit already set marks the slot in `dup`, which tells the first
    // lane on that slot too.  Those lanes are the only ones scanned.
    const uint32_t bit = 1u << ((s0 + j) & 31);
    const bool later_dup = act && j < i0 && clash;
    if (later_dup) atomicOr(&dup[(s0 + j) >> 5], bit);
    const bool first_dup = act && j < i0 && !clash && (dup[(s0 + j) >> 5] & bit) != 0;
    const uint64_t S = __ballot(act && (j >= i0 || later_dup || first_dup));
    if (later_dup) atomicAnd(&dup[(s0 + j) >> 5], ~bit);
    int candY = -1, tgtLater = -1;
    bool lastForJ = true;
    for (uint64_t m = S; m != 0; m &= m - 1) {
      const int q = __builtin_ctzll(m);
      const uint32_t jq = (uint32_t)__builtin_amdgcn_readlane((int)j, q);
      const uint32_t iq = i0 + (uint32_t)q;
      if (q < lane && jq == j && iq != j) candY = q;
      if (q > lane && jq == i) tgtLater = q;
      if (q > lane && jq == j) lastForJ = false;
    }
    // value slot i fetches from slot j at its step: a lane index or a slot
    int ref = -1;
    uint32_t ysrc = j;
    if (candY >= 0) ysrc = i0 + (uint32_t)candY;
    else if (j >= i0 && j < i) ref = (int)(j - i0);
#pragma unroll
    for (int it = 0; it < 6; ++it) {
      const int at = ref >= 0 ? ref : lane;
      const int refq = __shfl(ref, at, 64);
      const uint32_t ysq = __shfl(ysrc, at, 64);
      if (ref >= 0) {
        if (refq < 0) { ysrc = ysq; ref = -1; }
        else ref = refq;
      }
    }
    E ai, vi;
    if (act) {
      ai = data[s0 + i];
      const uint32_t srcI = tgtLater >= 0 ? i0 + (uint32_t)tgtLater : ysrc;
      vi = data[s0 + srcI];
    }
    if (act) {
      data[s0 + i] = vi;
      if (j < i0 && lastForJ) data[s0 + j] = ai;
    }
  }
}

// One super-block sb of 2^lds_levels leaves: Fisher-Yates of each leaf, then
// the merge levels among them, all in LDS.
// Copy cnt elements between global memory and LDS (LDS side 16-byte
// aligned): the whole 16-byte groups of the global side move as 16-byte
// accesses, every load of a thread issued before its first store; the
// ragged ends move element by element.  MAXV bounds the groups per thread.
template <typename E, int NT, int MAXV, bool TO_LDS>
__device__ __forceinline__ void copy_block(E* lds, E* glob, uint32_t cnt) {
  constexpr uint32_t PER = 16 / sizeof(E);
  const uint32_t mis = (uint32_t)((uintptr_t)glob & 15u);
  const uint32_t h = min(cnt, (uint32_t)(((16u - mis) & 15u) / sizeof(E)));
  const uint32_t groups = (cnt - h) / PER;
  const uint32_t tail0 = h + groups * PER;
  // (an opaque copy of the thread index: the load and the store at the two
  // ends of the leaf kernel compute their addresses each, none held between)
  uint32_t tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  if (tid < h) {
    if (TO_LDS) lds[tid] = glob[tid];
    else glob[tid] = lds[tid];
  }
  if (tid < cnt - tail0) {
    if (TO_LDS) lds[tail0 + tid] = glob[tail0 + tid];
    else glob[tail0 + tid] = lds[tail0 + tid];
  }
  uint4* g4 = reinterpret_cast<uint4*>(glob + h);
  uint4 v[MAXV];
  if (TO_LDS) {
#pragma unroll
    for (int k = 0; k < MAXV; ++k) {
      const uint32_t q = tid + NT * k;
      if (q < groups) v[k] = g4[q];
    }
  }
  if (h == 0) {
    uint4* l4 = reinterpret_cast<uint4*>(lds);
#pragma unroll
    for (int k = 0; k < MAXV; ++k) {
      const uint32_t q = tid + NT * k;
      if (q < groups) {
        if (TO_LDS) l4[q] = v[k];
        else v[k] = l4[q];
      }
    }
  } else {
    // the LDS side is off the 16-byte grid: element accesses
#pragma unroll
    for (int k = 0; k < MAXV; ++k) {
      const uint32_t q = tid + NT * k;
      if (q < groups) {
        E* e = reinterpret_cast<E*>(&v[k]);
#pragma unroll
        for (uint32_t c = 0; c < PER; ++c) {
          if (TO_LDS) lds[h + q * PER + c] = e[c];
          else e[c] = lds[h + q * PER + c];
        }
      }
    }
  }
  if (!TO_LDS) {
#pragma unroll
    for (int k = 0; k < MAXV; ++k) {
      const uint32_t q = tid + NT * k;
      if (q < groups) g4[q] = v[k];
    }
  }
}

template <typename E, int SCAP, int NT, bool IDENT>
__device__ __forceinline__ void leaf_body(const LeafArgs& a, const uint64_t sb) {
  constexpr int KW = (MergeAux<SCAP>::kWords + NT - 1) / NT;  // words per thread in scans
  constexpr int KS = (SCAP + NT - 1) / NT;                     // slots per thread
  constexpr int BPT = (SCAP / 4 + kLeafMaxMerges + NT - 1) / NT;  // step blocks per thread
  constexpr int SPT = SCAP / NT + 1;                              // slots of a leaf per thread, at most
  constexpr int MAXV = (int)((SCAP * sizeof(E) / 16 + NT - 1) / NT);  // 16-byte groups per thread
  static_assert(SCAP * sizeof(E) >= 4 * SCAP, "list heads and links live in the data region");
  // past the super-block's slots: 64 spare words, one per lane of a wave,
  // that the straight-line loops address for slots and steps that do not
  // exist (one shared spare word would take all those lanes' writes at one
  // address in one instruction)
  constexpr int kSpare = (int)(256 / sizeof(E));
  __shared__ __align__(16) E data[SCAP + kSpare];
  __shared__ MergeAux<SCAP> maux;
  __shared__ uint32_t tmp[20];
  __shared__ uint32_t mP[kLeafMaxMerges];
  __shared__ uint32_t mb[kLeafMaxMerges + 1];
  __shared__ uint32_t mmid[kLeafMaxMerges];
  __shared__ uint64_t red[NT / 64];

  const int tid = threadIdx.x;
  const Key key{a.key0, a.key1};
  const uint32_t Lam = a.lds_levels;
  const uint64_t base = bound(a.n, sb << Lam, a.c);
  const uint32_t cnt = (uint32_t)(bound(a.n, (sb + 1) << Lam, a.c) - base);
  const E* in = reinterpret_cast<const E*>(a.in);
  E* out = reinterpret_cast<E*>(a.out);
  uint32_t bits = 0;

  // leaves: tpl threads per leaf
  const uint32_t nleaf = 1u << Lam;
  const uint32_t tpl = NT >> Lam;
  const uint32_t lf = tid / tpl, lt = tid % tpl;
  const uint64_t u = (sb << Lam) + lf;
  const uint32_t lb = (uint32_t)(bound(a.n, u, a.c) - base);
  const uint32_t b = (uint32_t)(bound(a.n, u + 1, a.c) - bound(a.n, u, a.c));
  uint16_t* head = reinterpret_cast<uint16_t*>(data);
  uint32_t F[(SPT + 1) / 2];
  // this lane's spare word (lists use one word per slot)
  const uint32_t dummy = (uint32_t)(SCAP * sizeof(E) / 4) + (uint32_t)(tid & 63);
  leaf_fy_sources<BPT, SPT, NT>(head, lb, b, dummy, (uint32_t)u, lt, tpl, key, &bits, a.status, F);
  (void)nleaf;

  if (IDENT) {
    for (uint32_t i = tid; i < cnt; i += NT) data[i] = ident_value<E>(base + i);
  } else {
    copy_block<E, NT, MAXV, true>(data, const_cast<E*>(in) + base, cnt);
  }
  __syncthreads();
  {
    using R = typename RegOf<E>::type;
    R* dataR = reinterpret_cast<R*>(data);
    R val[SPT];
    // (a slot that does not exist has source 0 and writes the lane's spare
    // element)
    const uint32_t spare = SCAP + (uint32_t)(tid % kSpare);
    for_slots<SPT>(lt, tpl, lb, b, spare, [&](int i, uint32_t, uint32_t, bool) {
      val[i] = dataR[lb + get16(F[i >> 1], i & 1)];
    });
    __syncthreads();
    for_slots<SPT>(lt, tpl, lb, b, spare, [&](int i, uint32_t, uint32_t w, bool) { dataR[w] = val[i]; });
    __syncthreads();
  }

  // merge levels inside the super-block
  for (uint32_t L = 1; L <= Lam; ++L) {
    const uint32_t nm = 1u << (Lam - L);
    if (tid < (int)nm) {
      const uint64_t gm = (sb << (Lam - L)) + tid;
      const uint64_t i0 = gm << L;
      mb[tid] = (uint32_t)(bound(a.n, i0, a.c) - base);
      mmid[tid] = (uint32_t)(bound(a.n, i0 + (1ull << (L - 1)), a.c) - base);
      mP[tid] = kNone32;
    }
    if (tid == 0) mb[nm] = cnt;
    __syncthreads();
    uint32_t nmax = 0;
    for (uint32_t mm = 0; mm < nm; ++mm) nmax = max(nmax, mb[mm + 1] - mb[mm]);
    const uint32_t nblk = (nmax + 1 + 127) / 128;  // flips 0..N
    const uint32_t W = 4 * nblk;
    for (uint32_t fb = tid; fb < nm * nblk; fb += NT) {
      const uint32_t mm = fb / nblk, g = fb % nblk;
      const uint32_t gm = (uint32_t)((sb << (Lam - L)) + mm);
      const W4 f = flip_block(g, gm, L, key);
#pragma unroll
      for (int e = 0; e < 4; ++e) maux.words[mm * W + 4 * g + e] = f.w[e];
    }
    __syncthreads();
    // exclusive prefix of zeros over all words (flat)
    const uint32_t nw = nm * W;
    uint32_t zloc[KW];
    uint32_t zs = 0;
#pragma unroll
    for (int k = 0; k < KW; ++k) {
      const uint32_t w = tid * KW + k;
      zloc[k] = w < nw ? 32u - (uint32_t)__popc(maux.words[w]) : 0u;
      zs += zloc[k];
    }
    uint32_t run = block_excl_scan<NT>(zs, tmp, nullptr);
#pragma unroll
    for (int k = 0; k < KW; ++k) {
      const uint32_t w = tid * KW + k;
      if (w < nw) maux.wpre[w] = run;
      run += zloc[k];
    }
    __syncthreads();
    // break step: the (n1+1)-th zero or the (n2+1)-th one, whichever first
    for (uint32_t w = tid; w < nw; w += NT) {
      const uint32_t mm = w / W, wl = w % W;
      const uint32_t N = mb[mm + 1] - mb[mm];
      if (32 * wl > N) continue;
      const uint32_t n1 = mmid[mm] - mb[mm], n2 = mb[mm + 1] - mmid[mm];
      const uint32_t zp = maux.wpre[w] - maux.wpre[mm * W];
      const uint32_t op = 32 * wl - zp;
      const uint32_t word = maux.words[w];
      const uint32_t zw = 32u - (uint32_t)__popc(word), ow = (uint32_t)__popc(word);
      if (zp <= n1 && n1 < zp + zw) atomicMin(&mP[mm], (32 * wl + select_zero(word, (int)(n1 - zp))) * 2 + 0);
      if (op <= n2 && n2 < op + ow) atomicMin(&mP[mm], (32 * wl + select_one(word, (int)(n2 - op))) * 2 + 1);
    }
    __syncthreads();
    if (tid < (int)nm) bits += (mP[tid] >> 1) + 1;
    // stable interleave of A and B: source slot of every output slot (packed
    // two per register), then the values into registers, then back.  The
    // opaque copy of the thread index keeps the compiler from hoisting the
    // per-slot addresses of every level out of the level loop.
    uint32_t tv = (uint32_t)tid;
    asm volatile("" : "+v"(tv));
    // slots go by groups of 4 consecutive slots (group q of this thread:
    // slots 4 * (tid + q * NT) + j); a group inside one merge and before its
    // break step shares one flip word pair: with o_j the ones among its
    // first j flips, slot j takes B at n1 + t0 - r0 + o_j or A at r0 + j - o_j.
    // A thread's groups go up through the slots, so its merge only moves
    // forward: the merge's bounds stay in registers until a group passes
    // its end.
    constexpr int KG = (KS + 3) / 4;
    using R = typename RegOf<E>::type;
    R* dataR = reinterpret_cast<R*>(data);
    R val[4 * KG];
    uint32_t mm = 0, m0 = mb[0], m1 = mb[1], n1 = mmid[0] - mb[0], P = mP[0] >> 1, wb = maux.wpre[0];
#pragma unroll
    for (int q = 0; q < KG; ++q) {
      const uint32_t s0 = 4 * (tv + q * NT);
      uint32_t src[4] = {0u, 0u, 0u, 0u};
      if (s0 < cnt) {
        while (mm + 1 < nm && m1 <= s0) {
          ++mm;
          m0 = m1;
          m1 = mb[mm + 1];
          n1 = mmid[mm] - m0;
          P = mP[mm] >> 1;
          wb = maux.wpre[mm * W];
        }
        const uint32_t t0 = s0 - m0;
        if (s0 + 4 <= m1 && t0 + 4 <= P) {
          const uint32_t w = mm * W + (t0 >> 5);
          const uint32_t wlo = maux.words[w], whi = maux.words[w + 1];
          const uint32_t bp = t0 & 31;
          const uint32_t r0 = maux.wpre[w] - wb + (uint32_t)__popc(~wlo & ((1u << bp) - 1u));
          const uint32_t bits4 = (uint32_t)((((uint64_t)whi << 32) | wlo) >> bp);
          // xb = B's next source and xa + j = A's, moved by the all-ones mask
          // of each 1 flip (kept opaque: a bit select, not compare and select)
          uint32_t xa = m0 + r0, xb = m0 + n1 + t0 - r0;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            uint32_t m = 0u - ((bits4 >> j) & 1u);
            asm volatile("" : "+v"(m));
            src[j] = (xb & m) | ((xa + j) & ~m);
            xb -= m;
            xa += m;
          }
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const uint32_t sj = s0 + j;
            if (sj < cnt) {
              uint32_t k = mm;
              while (k + 1 < nm && mb[k + 1] <= sj) ++k;
              const uint32_t t = sj - mb[k];
              const uint32_t kn1 = mmid[k] - mb[k], kn2 = mb[k + 1] - mmid[k];
              const uint32_t kP = mP[k] >> 1, side = mP[k] & 1;
              uint32_t v;
              if (t < kP) {
                const uint32_t w = k * W + (t >> 5);
                const uint32_t word = maux.words[w];
                const uint32_t bp = t & 31;
                const uint32_t r0 = maux.wpre[w] - maux.wpre[k * W] + (uint32_t)__popc(~word & ((1u << bp) - 1u));
                v = ((word >> bp) & 1u) ? kn1 + (t - r0) : r0;
              } else {
                v = side == 0 ? t : t - kn2;
              }
              src[j] = v + mb[k];
            }
          }
        }
      }
      // the values can be read at once: nothing is written before the barrier
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (s0 + j < cnt) val[4 * q + j] = dataR[src[j]];
    }
    __syncthreads();
    asm volatile("" : "+v"(tv));
#pragma unroll
    for (int q = 0; q < KG; ++q) {
      const uint32_t s0 = 4 * (tv + q * NT);
      if constexpr (sizeof(E) == 4) {
        if (s0 + 4 <= cnt) {
          uint4 o4;
          o4.x = *reinterpret_cast<const uint32_t*>(&val[4 * q]);
          o4.y = *reinterpret_cast<const uint32_t*>(&val[4 * q + 1]);
          o4.z = *reinterpret_cast<const uint32_t*>(&val[4 * q + 2]);
          o4.w = *reinterpret_cast<const uint32_t*>(&val[4 * q + 3]);
          *reinterpret_cast<uint4*>(&data[s0]) = o4;
          continue;
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (s0 + j < cnt) dataR[s0 + j] = val[4 * q + j];
    }
    __syncthreads();
    // insertion loops, one wave per merge; the flip words are dead now and
    // their space holds the slot bitmap
    uint32_t* seen = maux.words;
    uint32_t* dup = maux.wpre;
    for (uint32_t w = tid; w < (cnt + 31) / 32; w += NT) seen[w] = dup[w] = 0u;
    __syncthreads();
    for (uint32_t mm = tid >> 6; mm < nm; mm += NT / 64) {
      const uint32_t gm = (uint32_t)((sb << (Lam - L)) + mm);
      lds_merge_tail<E>(data, seen, dup, mb[mm], mb[mm + 1] - mb[mm], mP[mm] >> 1, L, gm, key, &bits);
    }
    __syncthreads();
  }

  copy_block<E, NT, MAXV, false>(data, out + base, cnt);
  const uint64_t t = block_sum_u64<NT>(bits, red);
  if (tid == 0 && t) atomicAdd(a.bits, (unsigned long long)t);
}

// ---------------------------------------------------------------------------
// HBM merge pass
// ---------------------------------------------------------------------------

template <typename E>
__device__ __forceinline__ void store4(E* dst, const E v[4], uint32_t cnt) {
  if (cnt == 4 && sizeof(E) == 4 && ((uintptr_t)dst & 15) == 0) {
    uint4 w;
    w.x = *reinterpret_cast<const uint32_t*>(&v[0]);
    w.y = *reinterpret_cast<const uint32_t*>(&v[1]);
    w.z = *reinterpret_cast<const uint32_t*>(&v[2]);
    w.w = *reinterpret_cast<const uint32_t*>(&v[3]);
    *reinterpret_cast<uint4*>(dst) = w;
    return;
  }
#pragma unroll
  for (uint32_t e = 0; e < 4; ++e)
    if (e < cnt) dst[e] = v[e];
}

// Copy the run src[0..cnt) into dst[0..cnt): 16-byte loads for the whole
// 16-byte groups inside the run when the base pointer allows, element loads
// for the ragged ends.
template <typename E, bool VEC>
__device__ __forceinline__ void stage_run(E* dst, const E* base, uint64_t first, uint32_t cnt) {
  constexpr uint32_t PER = 16 / sizeof(E) > 0 ? 16 / sizeof(E) : 1;
  if (!VEC || PER == 1) {
    for (uint32_t x = threadIdx.x; x < cnt; x += 256) dst[x] = base[first + x];
    return;
  }
  const uint64_t lo = (first + PER - 1) / PER * PER;          // first aligned element
  const uint64_t hi = (first + cnt) / PER * PER;              // end of the last whole group
  if (hi <= lo) {
    for (uint32_t x = threadIdx.x; x < cnt; x += 256) dst[x] = base[first + x];
    return;
  }
  const uint32_t head = (uint32_t)(lo - first);
  const uint32_t groups = (uint32_t)((hi - lo) / PER);
  const uint32_t tail0 = (uint32_t)(hi - first);
  if (threadIdx.x < head) dst[threadIdx.x] = base[first + threadIdx.x];
  if (threadIdx.x < cnt - tail0) dst[tail0 + threadIdx.x] = base[hi + threadIdx.x];
  const uint4* g = reinterpret_cast<const uint4*>(base + lo);
  for (uint32_t q = threadIdx.x; q < groups; q += 256) {
    const uint4 v = g[q];
    const E* ve = reinterpret_cast<const E*>(&v);
#pragma unroll
    for (uint32_t c = 0; c < PER; ++c) dst[head + q * PER + c] = ve[c];
  }
}

// MODE 0: stage the A and B runs of the tile through LDS with element loads;
// MODE 1: the same with 16-byte loads; MODE 2: gather straight from HBM.
template <typename E, int T, int MODE>
__global__ void __launch_bounds__(256) merge_pass_kernel(PassArgs a) {
  constexpr int NW = T / 32;
  static_assert(NW <= 256, "one word per thread");
  __shared__ E stage[MODE == 2 ? 1 : T];
  __shared__ uint32_t Wd[NW];
  __shared__ uint32_t Zw[NW];
  __shared__ uint32_t tmp[8];
  const int tid = threadIdx.x;
  const uint32_t m = blockIdx.x / a.tpm;
  const uint32_t ti = blockIdx.x % a.tpm;
  const uint64_t i0 = (uint64_t)m << a.L;
  const uint64_t s = bound(a.n, i0, a.c);
  const uint64_t mid = bound(a.n, i0 + (1ull << (a.L - 1)), a.c);
  const uint64_t e = bound(a.n, i0 + (1ull << a.L), a.c);
  const uint32_t n1 = (uint32_t)(mid - s), n2 = (uint32_t)(e - mid), N = (uint32_t)(e - s);
  const uint32_t t0 = ti * (uint32_t)T;
  if (t0 >= N) return;
  const uint32_t t1 = min(t0 + (uint32_t)T, N);
  const uint32_t len = t1 - t0;
  // BalancedShuffle: every slot by its final label (the labels hold the
  // break and the insertion loop)
  const uint32_t P = a.lab ? N : a.P[a.merge_base + m];
  const uint32_t side = a.side[a.merge_base + m];
  const uint64_t cb = a.chunk_base + (uint64_t)m * a.cpm;
  auto r0c = [&](uint32_t t) -> uint32_t {
    if (t < P) {
      const uint64_t ch = cb + (t >> kChunkLog);
      return a.zc[ch] + a.zloc[(ch << kChunkGranLog) + ((t >> kGranLog) & 255)];
    }
    return side == 0 ? n1 : t - n2;
  };
  const uint32_t a0 = r0c(t0), a1 = r0c(t1);
  const uint32_t b0 = t0 - a0, b1 = t1 - a1;
  const uint32_t cntA = a1 - a0, cntB = b1 - b0;
  const E* in = reinterpret_cast<const E*>(a.in);
  E* out = reinterpret_cast<E*>(a.out);
  if (MODE != 2) {
    if (MODE == 1 && a.vec_ok) {
      stage_run<E, true>(stage, in, s + a0, cntA);
      stage_run<E, true>(stage + cntA, in, s + n1 + b0, cntB);
    } else {
      stage_run<E, false>(stage, in, s + a0, cntA);
      stage_run<E, false>(stage + cntA, in, s + n1 + b0, cntB);
    }
  }
  const uint32_t nblk = (len + 127) / 128;
  static_assert((1u << kChunkLog) % (uint32_t)T == 0, "a tile lies inside one chunk");
  if ((uint32_t)tid < nblk) {
    if (a.lab) {
      const uint32_t* lw = a.lab + ((cb + (t0 >> kChunkLog)) << 10) + ((t0 >> 5) & 1023u);
#pragma unroll
      for (int k = 0; k < 4; ++k) Wd[4 * tid + k] = lw[4 * tid + k];
    } else {
      const W4 f = flip_block((t0 >> kGranLog) + tid, m, a.L, Key{a.key0, a.key1});
#pragma unroll
      for (int k = 0; k < 4; ++k) Wd[4 * tid + k] = f.w[k];
    }
  }
  __syncthreads();
  const uint32_t nw = nblk * 4;
  const uint32_t z = (uint32_t)tid < nw ? 32u - (uint32_t)__popc(Wd[tid]) : 0u;
  const uint32_t zx = block_excl_scan<256>(z, tmp, nullptr);
  if ((uint32_t)tid < NW) Zw[tid] = zx;
  __syncthreads();
  const E* inA = in + s + a0;
  const E* inB = in + s + n1 + b0;
  for (uint32_t o = 4 * tid; o < len; o += 1024) {
    const uint32_t wi = o >> 5;
    const uint32_t word = Wd[wi];
    const uint32_t zb = Zw[wi];
    E v[4];
    const uint32_t cnt = min(4u, len - o);
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
      if (k < cnt) {
        const uint32_t tt = o + k;
        const uint32_t t = t0 + tt;
        uint32_t ia, ib;
        bool fromB;
        if (t < P) {
          const uint32_t bp = tt & 31;
          const uint32_t zz = zb + (uint32_t)__popc(~word & ((1u << bp) - 1u));
          fromB = (word >> bp) & 1u;
          ia = zz;
          ib = tt - zz;
        } else {
          fromB = side == 0;
          ia = t - n2 - a0;
          ib = t - n1 - b0;
        }
        if (MODE == 2) v[k] = fromB ? inB[ib] : inA[ia];
        else v[k] = fromB ? stage[cntA + ib] : stage[ia];
      }
    }
    store4<E>(out + s + t0 + o, v, cnt);
  }
}

// ---------------------------------------------------------------------------
// insertion-loop patches of one HBM level
// ---------------------------------------------------------------------------
template <typename E>
__global__ void __launch_bounds__(256) patch_kernel(PlanArgs pa, int l, const void* vin, void* vout) {
  const HbmLevel& lv = pa.lev[l];
  const uint32_t m = blockIdx.x / lv.wpm;
  const uint32_t w = blockIdx.x % lv.wpm;
  const uint64_t i0 = (uint64_t)m << lv.L;
  const uint64_t s = bound(pa.n, i0, pa.c);
  const uint32_t N = (uint32_t)(bound(pa.n, i0 + (1ull << lv.L), pa.c) - s);
  const uint64_t gm = lv.merge_base + m;
  const uint32_t P = pa.P[gm];
  const uint32_t k = N - P;
  const uint64_t toff = pa.toff[gm];
  const E* in = reinterpret_cast<const E*>(vin);
  E* out = reinterpret_cast<E*>(vout);
  for (uint32_t d = w * 256 + threadIdx.x; d < k; d += lv.wpm * 256) {
    if (toff + d >= pa.tail_cap) break;
    const uint32_t src = pa.tail_src[toff + d];
    if (src < N) out[s + P + d] = in[s + src];
  }
  const uint64_t bb = lv.bucket_base + (uint64_t)m * lv.bpm;
  const uint64_t lo = pa.boff[bb];
  uint64_t hi = pa.boff[bb + lv.bpm];
  if (hi > pa.pool_cap) hi = pa.pool_cap;
  for (uint64_t e = lo + (uint64_t)w * 256 + threadIdx.x; e < hi; e += (uint64_t)lv.wpm * 256) {
    const uint32_t src = pa.pool_src[e];
    const uint32_t x = pa.pool_x[e];
    if (src < N && x < N) out[s + x] = in[s + src];
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
template <typename E, int SCAP, int NT, bool IDENT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) leaf_kernel(LeafArgs a) {
  leaf_body<E, SCAP, NT, IDENT>(a, blockIdx.x);
}

// The leaf kernels of many arrays in one launch: job j owns workgroups
// [wpre[j], wpre[j+1]) of the nwg = wpre[njobs] workgroups.
template <typename E, int SCAP, int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4)))
leaf_multi_kernel(const LeafArgs* __restrict__ jobs, const uint32_t* __restrict__ wpre, uint32_t njobs) {
  const uint32_t w = blockIdx.x;
  uint32_t lo = 0, hi = njobs;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (wpre[mid] <= w) lo = mid;
    else hi = mid;
  }
  leaf_body<E, SCAP, NT, false>(jobs[lo], w - wpre[lo]);
}

template <typename E, int SCAP, int NT, bool IDENT>
static void launch_leaf_t(const LeafArgs& a, uint64_t grid, hipStream_t st) {
  hipLaunchKernelGGL((leaf_kernel<E, SCAP, NT, IDENT>), dim3((uint32_t)grid), dim3(NT), 0, st, a);
}

// Super-block size: 64 KiB of elements with 512 threads (two workgroups per
// CU, the default: measured faster), or 128 KiB with 1024 threads (one per
// CU, MS_LEAF_BIG=1).  A tuning knob only: the permutation does not depend on
// it.  16-byte leaves of cutoff + 1 = 4097 records do not fit the default
// 4096-record super-block: the planner takes the 128 KiB one for them.
static bool leaf_small() {
  static bool v = [] {
    const char* e = getenv("MS_LEAF_BIG");
    return !(e && atoi(e) != 0);
  }();
  return v;
}

// Elements per super-block: the default size, or the 128 KiB one (`big`).
int leaf_capacity(uint32_t eb, bool big) {
  const int cap = eb == 4 ? 32768 : eb == 8 ? 16384 : 8192;
  return big ? cap : cap / 2;
}
bool leaf_big_default() { return !leaf_small(); }
int leaf_max_block() { return 4097; }
int leaf_max_levels() { return 6; }

void launch_leaf_multi(const LeafArgs* jobs, const uint32_t* wpre, uint32_t njobs, uint32_t nwg, uint32_t eb,
                       bool big, hipStream_t st) {
  if (!nwg) return;
  const bool sm = !big;
  const dim3 g(nwg);
  if (eb == 4) {
    if (sm) hipLaunchKernelGGL((leaf_multi_kernel<uint32_t, 16384, 512>), g, dim3(512), 0, st, jobs, wpre, njobs);
    else hipLaunchKernelGGL((leaf_multi_kernel<uint32_t, 32768, 1024>), g, dim3(1024), 0, st, jobs, wpre, njobs);
  } else if (eb == 8) {
    if (sm) hipLaunchKernelGGL((leaf_multi_kernel<uint64_t, 8192, 512>), g, dim3(512), 0, st, jobs, wpre, njobs);
    else hipLaunchKernelGGL((leaf_multi_kernel<uint64_t, 16384, 1024>), g, dim3(1024), 0, st, jobs, wpre, njobs);
  } else {
    if (sm) hipLaunchKernelGGL((leaf_multi_kernel<uint4, 4096, 512>), g, dim3(512), 0, st, jobs, wpre, njobs);
    else hipLaunchKernelGGL((leaf_multi_kernel<uint4, 8192, 1024>), g, dim3(1024), 0, st, jobs, wpre, njobs);
  }
}

void launch_leaf(const LeafArgs& a, uint32_t eb, bool ident, bool big, uint64_t grid, hipStream_t st) {
  const bool sm = !big;
  if (eb == 4) {
    if (ident) {
      if (sm) launch_leaf_t<uint32_t, 16384, 512, true>(a, grid, st);
      else launch_leaf_t<uint32_t, 32768, 1024, true>(a, grid, st);
    } else {
      if (sm) launch_leaf_t<uint32_t, 16384, 512, false>(a, grid, st);
      else launch_leaf_t<uint32_t, 32768, 1024, false>(a, grid, st);
    }
  } else if (eb == 8) {
    if (sm) launch_leaf_t<uint64_t, 8192, 512, false>(a, grid, st);
    else launch_leaf_t<uint64_t, 16384, 1024, false>(a, grid, st);
  } else {
    if (sm) launch_leaf_t<uint4, 4096, 512, false>(a, grid, st);
    else launch_leaf_t<uint4, 8192, 1024, false>(a, grid, st);
  }
}

// Merge-pass variants: (tile, mode).  The default is variant 0 of each
// element size; the others are kept for tuning (MS_PASS_VARIANT).
struct PassVariant {
  int tile;
  int mode;
};
static const PassVariant kPassVariants[] = {{4096, 1}, {8192, 1}, {2048, 1}, {8192, 0}, {4096, 2}, {2048, 2}};

int pass_variant() {
  static int v = [] {
    const char* e = getenv("MS_PASS_VARIANT");
    int x = e ? atoi(e) : 0;
    return (x >= 0 && x < (int)(sizeof kPassVariants / sizeof kPassVariants[0])) ? x : 0;
  }();
  return v;
}

int pass_tile(uint32_t eb) {
  const int t = kPassVariants[pass_variant()].tile;
  return eb == 4 ? t : eb == 8 ? t / 2 : t / 4;
}

template <typename E, int T>
static void launch_pass_t(const PassArgs& a, int mode, uint64_t grid, hipStream_t st) {
  if (mode == 0) hipLaunchKernelGGL((merge_pass_kernel<E, T, 0>), dim3((uint32_t)grid), dim3(256), 0, st, a);
  else if (mode == 1) hipLaunchKernelGGL((merge_pass_kernel<E, T, 1>), dim3((uint32_t)grid), dim3(256), 0, st, a);
  else hipLaunchKernelGGL((merge_pass_kernel<E, T, 2>), dim3((uint32_t)grid), dim3(256), 0, st, a);
}

void launch_merge_pass(const PassArgs& a, uint32_t eb, uint64_t grid, hipStream_t st) {
  const PassVariant v = kPassVariants[pass_variant()];
  const int t = pass_tile(eb);
  if (eb == 4) {
    if (t == 8192) launch_pass_t<uint32_t, 8192>(a, v.mode, grid, st);
    else if (t == 4096) launch_pass_t<uint32_t, 4096>(a, v.mode, grid, st);
    else launch_pass_t<uint32_t, 2048>(a, v.mode, grid, st);
  } else if (eb == 8) {
    if (t == 4096) launch_pass_t<uint64_t, 4096>(a, v.mode, grid, st);
    else if (t == 2048) launch_pass_t<uint64_t, 2048>(a, v.mode, grid, st);
    else launch_pass_t<uint64_t, 1024>(a, v.mode, grid, st);
  } else {
    if (t == 2048) launch_pass_t<uint4, 2048>(a, v.mode, grid, st);
    else if (t == 1024) launch_pass_t<uint4, 1024>(a, v.mode, grid, st);
    else launch_pass_t<uint4, 512>(a, v.mode, grid, st);
  }
}

void launch_patch(const PlanArgs& pa, int l, const void* in, void* out, uint32_t eb, hipStream_t st) {
  const uint64_t grid = (uint64_t)pa.lev[l].nmerge * pa.lev[l].wpm;
  if (eb == 4) hipLaunchKernelGGL(patch_kernel<uint32_t>, dim3((uint32_t)grid), dim3(256), 0, st, pa, l, in, out);
  else if (eb == 8) hipLaunchKernelGGL(patch_kernel<uint64_t>, dim3((uint32_t)grid), dim3(256), 0, st, pa, l, in, out);
  else hipLaunchKernelGGL(patch_kernel<uint4>, dim3((uint32_t)grid), dim3(256), 0, st, pa, l, in, out);
}

}  // namespace ms
