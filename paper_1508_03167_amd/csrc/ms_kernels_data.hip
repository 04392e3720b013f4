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
// The lists of steps per target slot are built with LDS atomics.
//
// Insertion loop in LDS.  A merge's tail steps i = P..N-1 run as groups of
// 64 steps on one wave: within a group each lane resolves its step against
// the earlier lanes of the group (the latest earlier lane targeting the same
// slot, else the lane whose own step filled that slot, else the value before
// the group), then every touched slot is written once.
#include "ms_device.hpp"
#include "ms_plan.hpp"

namespace ms {

constexpr int kLeafThreads = 1024;
constexpr int kLeafMaxMerges = 64;  // at most 2^6 leaves per super-block

struct LeafArgs {
  const void* in;
  void* out;
  uint64_t n;
  uint32_t c;
  uint32_t lds_levels;
  uint32_t key0, key1;
  unsigned long long* bits;
};

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

template <int LMAX>
struct FyAux {
  uint32_t head[LMAX];   // list head per target slot; later up() per slot
  uint16_t next[LMAX];   // next step in the same target list
};

template <int SCAP>
struct MergeAux {
  static constexpr int kWords = SCAP / 32 + 8 * kLeafMaxMerges + 8;
  uint32_t words[kWords];
  uint32_t wpre[kWords];
};

template <int SCAP, int LMAX>
union LeafAux {
  FyAux<LMAX> fy;
  MergeAux<SCAP> mg;
};

// Fisher-Yates of one leaf [lb, lb+b) of the LDS array, unit u.
template <typename E, int LMAX>
__device__ __forceinline__ void leaf_fisher_yates(E* data, FyAux<LMAX>& fy, uint32_t lb, uint32_t b, uint32_t u,
                                                  Key key, uint32_t* bits) {
  constexpr int NT = kLeafThreads;
  constexpr int NB = (LMAX + 4 * NT - 1) / (4 * NT);
  const int tid = threadIdx.x;
  for (uint32_t x = tid; x < b; x += NT) fy.head[x] = kNone32;
  __syncthreads();
  uint32_t jr[NB][4];
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const uint32_t g = tid + k * NT;
#pragma unroll
    for (int e = 0; e < 4; ++e) jr[k][e] = kNone32;
    if (4 * g < b) {
      const W4 db = draw_block(g, u, 0, key);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint32_t r = 4 * g + e;
        if (r >= 1 && r < b) {
          const uint32_t j = fdr_draw((uint64_t)r + 1, db.w[e], 0, u, r, key, bits);
          jr[k][e] = j;
          const uint32_t old = atomicExch(&fy.head[j], r);
          fy.next[r] = (uint16_t)(old == kNone32 ? 0xFFFFu : old);
        }
      }
    }
  }
  __syncthreads();
  uint32_t upv[NB][4], nx[NB][4];
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const uint32_t g = tid + k * NT;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const uint32_t x = 4 * g + e;
      upv[k][e] = kNone32;
      nx[k][e] = kNone32;
      if (x < b) {
        uint32_t best = kNone32;
        for (uint32_t p = fy.head[x]; p != kNone32;) {
          if (p > x && p < best) best = p;
          const uint32_t q = fy.next[p];
          p = q == 0xFFFFu ? kNone32 : q;
        }
        upv[k][e] = best;
        if (x >= 1) {
          uint32_t best2 = kNone32;
          for (uint32_t p = fy.head[jr[k][e]]; p != kNone32;) {
            if (p > x && p < best2) best2 = p;
            const uint32_t q = fy.next[p];
            p = q == 0xFFFFu ? kNone32 : q;
          }
          nx[k][e] = best2;
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const uint32_t g = tid + k * NT;
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (4 * g + e < b) fy.head[4 * g + e] = upv[k][e];
  }
  __syncthreads();
  E val[NB][4];
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const uint32_t g = tid + k * NT;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const uint32_t x = 4 * g + e;
      if (x < b) {
        uint32_t src;
        uint32_t t = x == 0 ? 0u : nx[k][e];
        if (x != 0 && t == kNone32) {
          src = jr[k][e];
        } else {
          while (fy.head[t] != kNone32) t = fy.head[t];
          src = t;
        }
        val[k][e] = data[lb + src];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const uint32_t g = tid + k * NT;
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (4 * g + e < b) data[lb + 4 * g + e] = val[k][e];
  }
  __syncthreads();
}

// Insertion loop of one merge [s0, s0+N) in LDS by one wave, groups of 64 steps.
template <typename E>
__device__ __forceinline__ void lds_merge_tail(E* data, uint32_t s0, uint32_t N, uint32_t P, uint32_t L,
                                               uint32_t gm, Key key, uint32_t* bits) {
  const int lane = threadIdx.x & 63;
  for (uint32_t i0 = P; i0 < N; i0 += 64) {
    const uint32_t i = i0 + lane;
    const bool act = i < N;
    uint32_t j = kNone32;
    if (act) {
      const W4 db = draw_block(i >> 2, gm, L, key);
      j = fdr_draw((uint64_t)i + 1, db.w[i & 3], L, gm, i, key, bits);
    }
    int candY = -1, tgtLater = -1;
    bool lastForJ = true;
    const uint32_t nact = (N - i0) < 64u ? (N - i0) : 64u;
    for (uint32_t q = 0; q < nact; ++q) {
      const uint32_t jq = (uint32_t)__builtin_amdgcn_readlane((int)j, (int)q);
      const uint32_t iq = i0 + q;
      if ((int)q < lane && jq == j && iq != j) candY = (int)q;
      if ((int)q > lane && jq == i) tgtLater = (int)q;
      if ((int)q > lane && jq == j) lastForJ = false;
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

template <typename E, int SCAP, int LMAX, bool IDENT>
__global__ void __launch_bounds__(kLeafThreads) leaf_kernel(LeafArgs a) {
  constexpr int NT = kLeafThreads;
  constexpr int KW = (MergeAux<SCAP>::kWords + NT - 1) / NT;  // words per thread in scans
  constexpr int KS = (SCAP + NT - 1) / NT;                     // slots per thread
  __shared__ E data[SCAP];
  __shared__ LeafAux<SCAP, LMAX> aux;
  __shared__ uint32_t tmp[20];
  __shared__ uint32_t mP[kLeafMaxMerges];
  __shared__ uint32_t mb[kLeafMaxMerges + 1];
  __shared__ uint32_t mmid[kLeafMaxMerges];
  __shared__ uint64_t red[16];

  const int tid = threadIdx.x;
  const Key key{a.key0, a.key1};
  const uint32_t Lam = a.lds_levels;
  const uint64_t sb = blockIdx.x;
  const uint64_t base = bound(a.n, sb << Lam, a.c);
  const uint32_t cnt = (uint32_t)(bound(a.n, (sb + 1) << Lam, a.c) - base);
  const E* in = reinterpret_cast<const E*>(a.in);
  E* out = reinterpret_cast<E*>(a.out);
  uint32_t bits = 0;

  for (uint32_t i = tid; i < cnt; i += NT) data[i] = IDENT ? ident_value<E>(base + i) : in[base + i];
  __syncthreads();

  // leaves
  const uint32_t nleaf = 1u << Lam;
  for (uint32_t lf = 0; lf < nleaf; ++lf) {
    const uint64_t u = (sb << Lam) + lf;
    const uint32_t lb = (uint32_t)(bound(a.n, u, a.c) - base);
    const uint32_t b = (uint32_t)(bound(a.n, u + 1, a.c) - bound(a.n, u, a.c));
    leaf_fisher_yates<E, LMAX>(data, aux.fy, lb, b, (uint32_t)u, key, &bits);
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
      for (int e = 0; e < 4; ++e) aux.mg.words[mm * W + 4 * g + e] = f.w[e];
    }
    __syncthreads();
    // exclusive prefix of zeros over all words (flat)
    const uint32_t nw = nm * W;
    uint32_t zloc[KW];
    uint32_t zs = 0;
#pragma unroll
    for (int k = 0; k < KW; ++k) {
      const uint32_t w = tid * KW + k;
      zloc[k] = w < nw ? 32u - (uint32_t)__popc(aux.mg.words[w]) : 0u;
      zs += zloc[k];
    }
    uint32_t run = block_excl_scan<NT>(zs, tmp, nullptr);
#pragma unroll
    for (int k = 0; k < KW; ++k) {
      const uint32_t w = tid * KW + k;
      if (w < nw) aux.mg.wpre[w] = run;
      run += zloc[k];
    }
    __syncthreads();
    // break step: the (n1+1)-th zero or the (n2+1)-th one, whichever first
    for (uint32_t w = tid; w < nw; w += NT) {
      const uint32_t mm = w / W, wl = w % W;
      const uint32_t N = mb[mm + 1] - mb[mm];
      if (32 * wl > N) continue;
      const uint32_t n1 = mmid[mm] - mb[mm], n2 = mb[mm + 1] - mmid[mm];
      const uint32_t zp = aux.mg.wpre[w] - aux.mg.wpre[mm * W];
      const uint32_t op = 32 * wl - zp;
      const uint32_t word = aux.mg.words[w];
      const uint32_t zw = 32u - (uint32_t)__popc(word), ow = (uint32_t)__popc(word);
      if (zp <= n1 && n1 < zp + zw) atomicMin(&mP[mm], (32 * wl + select_zero(word, (int)(n1 - zp))) * 2 + 0);
      if (op <= n2 && n2 < op + ow) atomicMin(&mP[mm], (32 * wl + select_one(word, (int)(n2 - op))) * 2 + 1);
    }
    __syncthreads();
    if (tid < (int)nm) bits += (mP[tid] >> 1) + 1;
    // stable interleave of A and B into registers, then back
    E val[KS];
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const uint32_t s = tid + k * NT;
      if (s < cnt) {
        uint32_t lo = 0, hi = nm - 1;
        while (lo < hi) {
          const uint32_t mid = (lo + hi + 1) >> 1;
          if (mb[mid] <= s) lo = mid; else hi = mid - 1;
        }
        const uint32_t mm = lo;
        const uint32_t t = s - mb[mm];
        const uint32_t n1 = mmid[mm] - mb[mm], n2 = mb[mm + 1] - mmid[mm];
        const uint32_t P = mP[mm] >> 1, side = mP[mm] & 1;
        uint32_t src;
        if (t < P) {
          const uint32_t w = mm * W + (t >> 5);
          const uint32_t word = aux.mg.words[w];
          const uint32_t bp = t & 31;
          const uint32_t r0 = aux.mg.wpre[w] - aux.mg.wpre[mm * W] + (uint32_t)__popc(~word & ((1u << bp) - 1u));
          src = ((word >> bp) & 1u) ? n1 + (t - r0) : r0;
        } else {
          src = side == 0 ? t : t - n2;
        }
        val[k] = data[mb[mm] + src];
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const uint32_t s = tid + k * NT;
      if (s < cnt) data[s] = val[k];
    }
    __syncthreads();
    // insertion loops, one wave per merge
    for (uint32_t mm = tid >> 6; mm < nm; mm += NT / 64) {
      const uint32_t gm = (uint32_t)((sb << (Lam - L)) + mm);
      lds_merge_tail<E>(data, mb[mm], mb[mm + 1] - mb[mm], mP[mm] >> 1, L, gm, key, &bits);
    }
    __syncthreads();
  }

  for (uint32_t i = tid; i < cnt; i += NT) out[base + i] = data[i];
  const uint64_t t = block_sum_u64<NT>(bits, red);
  if (tid == 0 && t) atomicAdd(a.bits, (unsigned long long)t);
}

// ---------------------------------------------------------------------------
// HBM merge pass
// ---------------------------------------------------------------------------
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
};

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

template <typename E, int T>
__global__ void __launch_bounds__(256) merge_pass_kernel(PassArgs a) {
  constexpr int NW = T / 32;
  static_assert(NW <= 256, "one word per thread");
  __shared__ E stage[T];
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
  const uint32_t P = a.P[a.merge_base + m];
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
  for (uint32_t x = tid; x < cntA; x += 256) stage[x] = in[s + a0 + x];
  for (uint32_t x = tid; x < cntB; x += 256) stage[cntA + x] = in[s + n1 + b0 + x];
  const uint32_t nblk = (len + 127) / 128;
  if ((uint32_t)tid < nblk) {
    const W4 f = flip_block((t0 >> kGranLog) + tid, m, a.L, Key{a.key0, a.key1});
#pragma unroll
    for (int k = 0; k < 4; ++k) Wd[4 * tid + k] = f.w[k];
  }
  __syncthreads();
  const uint32_t nw = nblk * 4;
  const uint32_t z = (uint32_t)tid < nw ? 32u - (uint32_t)__popc(Wd[tid]) : 0u;
  const uint32_t zx = block_excl_scan<256>(z, tmp, nullptr);
  if ((uint32_t)tid < NW) Zw[tid] = zx;
  __syncthreads();
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
        if (t < P) {
          const uint32_t bp = tt & 31;
          const uint32_t zz = zb + (uint32_t)__popc(~word & ((1u << bp) - 1u));
          v[k] = ((word >> bp) & 1u) ? stage[cntA + tt - zz] : stage[zz];
        } else {
          v[k] = side == 0 ? stage[cntA + (t - n1 - b0)] : stage[t - n2 - a0];
        }
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
    if (src != kNone32) out[s + P + d] = in[s + src];
  }
  const uint64_t bb = lv.bucket_base + (uint64_t)m * lv.bpm;
  const uint64_t lo = pa.boff[bb];
  uint64_t hi = pa.boff[bb + lv.bpm];
  if (hi > pa.pool_cap) hi = pa.pool_cap;
  for (uint64_t e = lo + (uint64_t)w * 256 + threadIdx.x; e < hi; e += (uint64_t)lv.wpm * 256) {
    const uint32_t src = pa.pool_src[e];
    if (src != kNone32) out[s + pa.pool_x[e]] = in[s + src];
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
template <typename E, int SCAP, bool IDENT>
static void launch_leaf_t(const LeafArgs& a, uint64_t grid, hipStream_t st) {
  hipLaunchKernelGGL((leaf_kernel<E, SCAP, 4097, IDENT>), dim3((uint32_t)grid), dim3(kLeafThreads), 0, st, a);
}

int leaf_capacity(uint32_t eb) { return eb == 4 ? 32768 : eb == 8 ? 16384 : 8192; }
int leaf_max_block() { return 4097; }
int leaf_max_levels() { return 6; }
int pass_tile(uint32_t eb) { return eb == 4 ? 8192 : eb == 8 ? 4096 : 2048; }

void launch_leaf(const LeafArgs& a, uint32_t eb, bool ident, uint64_t grid, hipStream_t st) {
  if (eb == 4) {
    if (ident) launch_leaf_t<uint32_t, 32768, true>(a, grid, st);
    else launch_leaf_t<uint32_t, 32768, false>(a, grid, st);
  } else if (eb == 8) {
    launch_leaf_t<uint64_t, 16384, false>(a, grid, st);
  } else {
    launch_leaf_t<uint4, 8192, false>(a, grid, st);
  }
}

void launch_merge_pass(const PassArgs& a, uint32_t eb, uint64_t grid, hipStream_t st) {
  if (eb == 4) hipLaunchKernelGGL((merge_pass_kernel<uint32_t, 8192>), dim3((uint32_t)grid), dim3(256), 0, st, a);
  else if (eb == 8) hipLaunchKernelGGL((merge_pass_kernel<uint64_t, 4096>), dim3((uint32_t)grid), dim3(256), 0, st, a);
  else hipLaunchKernelGGL((merge_pass_kernel<uint4, 2048>), dim3((uint32_t)grid), dim3(256), 0, st, a);
}

void launch_patch(const PlanArgs& pa, int l, const void* in, void* out, uint32_t eb, hipStream_t st) {
  const uint64_t grid = (uint64_t)pa.lev[l].nmerge * pa.lev[l].wpm;
  if (eb == 4) hipLaunchKernelGGL(patch_kernel<uint32_t>, dim3((uint32_t)grid), dim3(256), 0, st, pa, l, in, out);
  else if (eb == 8) hipLaunchKernelGGL(patch_kernel<uint64_t>, dim3((uint32_t)grid), dim3(256), 0, st, pa, l, in, out);
  else hipLaunchKernelGGL(patch_kernel<uint4>, dim3((uint32_t)grid), dim3(256), 0, st, pa, l, in, out);
}

}  // namespace ms
