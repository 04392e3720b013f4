// ms_device.hpp -- device building blocks of the MergeShuffle HIP path (gfx950).
//
// Random source.  The paper works in the random-bit model (introduction,
// paragraph on the random-bit model): a coin flip costs one fair bit and a
// uniform integer in {0..k-1} is drawn from fair bits by the Fast Dice Roller
// of [Lumbroso13].  The paper names no generator, so bits come from
// Philox-4x32-10 (Salmon et al., SC'11) under a fixed counter layout, keyed by
// the 64-bit seed (key = lo32, hi32):
//   FLIP(L, m, t) -- the t-th coin flip of merge m at level L: bit (t & 31) of
//                    word (t >> 5) & 3 of Philox(t >> 7, m, L, 1 << 28).
//   DRAW(L, u, d) -- the bits of the d-th bounded draw of unit u (leaf block u
//                    at L = 0, merge u at L >= 1): word d & 3 of
//                    Philox(d >> 2, u, L, 2 << 28), most significant bit
//                    first, then Philox(d, u, L, (3 << 28) | j), j = 0, 1, ...,
//                    words x0..x3 in order, each most significant bit first.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ms {

constexpr uint32_t kDomFlip = 1u << 28;
constexpr uint32_t kDomDraw = 2u << 28;
constexpr uint32_t kDomCont = 3u << 28;
constexpr uint32_t kNone32 = 0xFFFFFFFFu;

struct Key {
  uint32_t k0, k1;
};

struct W4 {
  uint32_t w[4];
};

// Philox-4x32-10: ten rounds of two 32x32->64 multiplies, key bumped by the
// Weyl constants between rounds.
__device__ __forceinline__ W4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, Key key) {
  uint32_t k0 = key.k0, k1 = key.k1;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  W4 o;
  o.w[0] = c0; o.w[1] = c1; o.w[2] = c2; o.w[3] = c3;
  return o;
}

// Word i (0..3) of a block, without indexing a private array.
__device__ __forceinline__ uint32_t pick(const W4& x, uint32_t i) {
  const uint32_t lo = (i & 1u) ? x.w[1] : x.w[0];
  const uint32_t hi = (i & 1u) ? x.w[3] : x.w[2];
  return (i & 2u) ? hi : lo;
}

// The 128 coin flips t = 128*g .. 128*g+127 of merge m at level L.
__device__ __forceinline__ W4 flip_block(uint32_t g, uint32_t m, uint32_t L, Key key) {
  return philox(g, m, L, kDomFlip, key);
}

// Primary words of the draws d = 4*g .. 4*g+3 of unit u at level L.
__device__ __forceinline__ W4 draw_block(uint32_t g, uint32_t u, uint32_t L, Key key) {
  return philox(g, u, L, kDomDraw, key);
}

__device__ __forceinline__ int bitlen64(uint64_t x) { return 64 - __clzll(x); }

// A wave-uniform value moved to a scalar register.  The builtin takes and
// returns int: its result goes back to uint32_t here, before any widening,
// so that a value >= 2^31 is not sign-extended into the upper half of a
// 64-bit offset.
__device__ __forceinline__ uint32_t uniform_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ uint64_t uniform_u64(uint32_t hi, uint32_t lo) {
  return ((uint64_t)uniform_u32(hi) << 32) | uniform_u32(lo);
}

// Fast Dice Roller in its jump form: instead of one bit at a time it reads at
// once the d bits after which the range v first reaches k (least d with
// v * 2^d >= k), which is the same bits in the same order with the same
// result as the bit-at-a-time loop.  Returns the value in [0, k) and the
// number of bits consumed.  k <= 2^32.
struct Draw {
  uint32_t v;
  uint32_t bits;
};

__device__ __noinline__ Draw fdr_draw_slow(uint64_t k, uint32_t w0, uint32_t L, uint32_t u, uint32_t d, Key key) {
  uint64_t v = 1, c = 0;
  uint32_t buf = w0;
  int left = 32;
  uint32_t cont_j = 0;
  int cont_idx = 4;
  W4 cw;
  cw.w[0] = cw.w[1] = cw.w[2] = cw.w[3] = 0;
  uint32_t used = 0;
  const int bk = bitlen64(k - 1);
  for (;;) {
    int jump = bk - bitlen64(v);
    if ((v << jump) <= k - 1) jump += 1;
    uint64_t x = 0;
    int need = jump;
    while (need > 0) {
      if (left == 0) {
        if (cont_idx == 4) {
          cw = philox(d, u, L, kDomCont | cont_j, key);
          cont_j += 1;
          cont_idx = 0;
        }
        buf = cw.w[cont_idx];
        cont_idx += 1;
        left = 32;
      }
      const int take = need < left ? need : left;
      const uint32_t part = take == 32 ? buf : ((buf >> (left - take)) & ((1u << take) - 1u));
      x = (x << take) | part;
      left -= take;
      need -= take;
    }
    v <<= jump;
    c = (c << jump) | x;
    used += (uint32_t)jump;
    if (c < k) return Draw{(uint32_t)c, used};
    v -= k;
    c -= k;
  }
}

__device__ __forceinline__ Draw fdr_draw(uint64_t k, uint32_t w0, uint32_t L, uint32_t u, uint32_t d, Key key) {
  if (k <= 1) return Draw{0u, 0u};
  if (k <= (1ull << 31)) {
    // Ranges stay below 2^32: run the loop in 32-bit arithmetic as long as
    // the primary word lasts; restart in the general routine otherwise.
    const uint32_t k32 = (uint32_t)k;
    const int bk = 32 - __clz(k32 - 1);
    uint32_t v = 1, c = 0, used = 0;
    int left = 32;
#pragma unroll 1
    for (;;) {
      int jump = bk - (32 - __clz(v));
      if ((v << jump) <= k32 - 1) jump += 1;
      if (jump > left) break;
      const uint32_t x = jump == 32 ? w0 : ((w0 >> (left - jump)) & ((1u << jump) - 1u));
      left -= jump;
      used += (uint32_t)jump;
      v <<= jump;
      c = (c << jump) | x;
      if (c < k32) return Draw{c, used};
      v -= k32;
      c -= k32;
    }
  }
  return fdr_draw_slow(k, w0, L, u, d, key);
}

// Position (0..31) of the r-th zero bit (r counted from 0) of w, LSB first.
__device__ __forceinline__ int select_zero(uint32_t w, int r) {
  uint32_t z = ~w;
  for (int i = 0; i < r; ++i) z &= z - 1;
  return __ffs(z) - 1;
}

__device__ __forceinline__ int select_one(uint32_t w, int r) {
  uint32_t z = w;
  for (int i = 0; i < r; ++i) z &= z - 1;
  return __ffs(z) - 1;
}

// Register copy of an element: a native 4 x u32 vector for uint4, whose
// wrapper type keeps an array of them out of registers.
typedef uint32_t v4u __attribute__((ext_vector_type(4)));
template <typename E> struct RegOf { using type = E; };
template <> struct RegOf<uint4> { using type = v4u; };

// Leaf / merge bounds of the partition: block i is [n*i >> c, n*(i+1) >> c).
__device__ __host__ __forceinline__ uint64_t bound(uint64_t n, uint64_t i, uint32_t c) {
  return (n * i) >> c;
}

// Wave-level inclusive scan (wave64) of u32.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

// Block-level exclusive scan of u32 over NT threads; tmp holds NT/64 + 1 words.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* tmp, uint32_t* total) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t incl = wave_incl_scan(v);
  if (lane == 63) tmp[wid] = incl;
  __syncthreads();
  if (wid == 0) {
    const uint32_t s = lane < NW ? tmp[lane] : 0u;
    const uint32_t si = wave_incl_scan(s);
    if (lane < NW) tmp[lane] = si - s;
    if (lane == NW - 1) tmp[NW] = si;
  }
  __syncthreads();
  const uint32_t r = tmp[wid] + incl - v;
  if (total) *total = tmp[NW];
  __syncthreads();
  return r;
}

template <int NT>
__device__ __forceinline__ uint64_t block_sum_u64(uint64_t v, uint64_t* tmp) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if (lane == 0) tmp[wid] = v;
  __syncthreads();
  uint64_t t = 0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < NW; ++i) t += tmp[i];
  }
  __syncthreads();
  return t;
}

}  // namespace ms
