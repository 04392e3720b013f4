// ms_api.hip -- host runtime and C ABI of the MergeShuffle library.
//
// The planner turns (n, element size, cutoff) into the level layout of the
// top-level routine (shuffle() listing, Appendix A.2): c levels over q = 2^c leaves, the
// first `lds_levels` merge levels fused into the leaf kernel, the rest as HBM
// passes with their data-independent plan.  Scratch (one array copy for the
// out-of-place HBM levels plus the plan tables) is kept per (device, stream)
// and grown on demand; every launch is enqueued on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "mergeshuffle.h"
#include "ms_plan.hpp"

namespace ms {
void launch_group(const GroupArgs& a, int lam, uint32_t eb, uint64_t grid, hipStream_t st);
int group_tile(uint32_t eb);
void launch_pass_group(const GroupArgs& a, int lam, uint32_t eb, uint32_t T, uint64_t grid, hipStream_t st);
int pass_group_tile(uint32_t eb, uint64_t n);
void launch_pass_group_multi(const GroupArgs* jobs, const uint32_t* tpre, uint32_t njobs, uint32_t ntiles, int lam,
                             uint32_t eb, hipStream_t st);
uint32_t pass_desc_words(uint32_t eb, uint32_t T, int lam);
void launch_pass_desc(const GroupArgs& a, int lam, uint32_t eb, uint32_t T, uint64_t grid, hipStream_t st);
void launch_pass_desc_multi(const GroupArgs* jobs, const uint32_t* tpre, uint32_t njobs, uint32_t ntiles, int lam,
                            uint32_t eb, hipStream_t st);
void launch_plan(const PlanArgs& pa, hipStream_t st);
void launch_plan_multi(const PlanArgs* pas, uint32_t njobs, const uint32_t* const* pre, const uint32_t* units,
                       hipStream_t st);
void launch_leaf_multi(const LeafArgs* jobs, const uint32_t* wpre, uint32_t njobs, uint32_t nwg, uint32_t eb,
                       bool big, hipStream_t st);
void launch_group_multi(const GroupArgs* jobs, const uint32_t* tpre, uint32_t njobs, uint32_t ntiles, int lam,
                        uint32_t eb, hipStream_t st);
void launch_leaf(const LeafArgs& a, uint32_t eb, bool ident, bool big, uint64_t grid, hipStream_t st);
void launch_merge_pass(const PassArgs& a, uint32_t eb, uint64_t grid, hipStream_t st);
void launch_patch(const PlanArgs& pa, int l, const void* in, void* out, uint32_t eb, hipStream_t st);
void launch_merge_r1(const PlanArgs& pa, int l, const void* in, void* out, uint32_t eb, hipStream_t st);
int leaf_capacity(uint32_t eb, bool big);
bool leaf_big_default();
int leaf_max_block();
int leaf_max_levels();
int pass_tile(uint32_t eb);
}  // namespace ms

namespace {

using namespace ms;

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(MS_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr uint64_t kMaxN = (1ull << 32) - (1ull << 16);

// Fused-pass kernel: the word-aligned table pass (default) or the earlier
// window-tree pass (MS_PASS_IMPL=tree), kept for comparison.  The
// permutation does not depend on the choice.
bool pass_tree() {
  static const bool v = [] {
    const char* e = getenv("MS_PASS_IMPL");
    return e && strcmp(e, "tree") == 0;
  }();
  return v;
}
int fused_tile(uint32_t eb, uint64_t n) { return pass_tree() ? group_tile(eb) : pass_group_tile(eb, n); }
void launch_fused(const GroupArgs& a, int lam, uint32_t eb, uint32_t T, uint64_t grid, hipStream_t st) {
  if (pass_tree()) launch_group(a, lam, eb, grid, st);
  else launch_pass_group(a, lam, eb, T, grid, st);
}
void launch_fused_multi(const GroupArgs* jobs, const uint32_t* tpre, uint32_t njobs, uint32_t ntiles, int lam,
                        uint32_t eb, hipStream_t st) {
  if (pass_tree()) launch_group_multi(jobs, tpre, njobs, ntiles, lam, eb, st);
  else launch_pass_group_multi(jobs, tpre, njobs, ntiles, lam, eb, st);
}
constexpr uint32_t kDefaultB = 4096;

// ---------------------------------------------------------------------------
// planner
// ---------------------------------------------------------------------------
struct Layout {
  size_t zloc, ctot, zc, zg, P, side, kcnt, toff, tail_src, bcnt, bfill, boff, part, pool_x, pool_step, pool_src,
      tail_xsrc, pool_xsrc, bnd, desc, bits_part, lab;
  size_t bytes;
};

struct HostPlan {
  uint64_t n = 0;
  uint32_t eb = 4, B = kDefaultB, c = 0, lam = 0, nlev = 0;
  uint64_t q = 1;
  uint64_t pass_tiles = 0;
  bool fused = true;              // HBM levels run as fused groups (else one pass + patch per level)
  bool leaf_big = false;          // 128 KiB leaf super-block (1024 threads)
  uint32_t ngroup = 0;
  uint32_t gfirst[kMaxLevels];    // first HBM level index of each group
  uint32_t glam[kMaxLevels];      // levels in each group
  uint64_t gdesc_first[kMaxLevels];  // first word of each group's tile descriptors (table pass)
  uint32_t gdesc_words[kMaxLevels];  // words per tile descriptor
  PlanArgs pa;
  Layout lay;
};

uint64_t ceil_shift(uint64_t n, uint32_t s) { return (n + (1ull << s) - 1) >> s; }

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// ---------------------------------------------------------------------------
// tuning table: per (element size, floor(log2 n)) the cutoff, the fused
// levels per pass and the leaf shape that calls with MS_CFG_TUNED take
// ---------------------------------------------------------------------------
std::mutex g_tune_mu;
std::map<uint64_t, ms_tune_entry> g_tune;

uint64_t tune_key(uint32_t eb, uint64_t n) {
  uint32_t k = 0;
  while (k < 63 && (n >> (k + 1)) != 0) ++k;
  return ((uint64_t)eb << 32) | k;
}

bool tune_lookup(uint64_t n, uint32_t eb, ms_tune_entry* out) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(tune_key(eb, n));
  if (it == g_tune.end()) return false;
  *out = it->second;
  return true;
}

int make_plan(uint64_t n, uint32_t eb, const ms_config* cfg, HostPlan& hp) {
  ms_config tuned;
  if (cfg && (cfg->flags & MS_CFG_TUNED)) {
    tuned = *cfg;
    ms_tune_entry e;
    if (tune_lookup(n, eb, &e)) {
      tuned.leaf_B = e.leaf_B;
      tuned.levels_per_pass = e.levels_per_pass;
      tuned.flags = (tuned.flags & ~MS_CFG_LEAF_BIG) | (e.flags & MS_CFG_LEAF_BIG);
    }
    cfg = &tuned;
  }
  if (eb != 4 && eb != 8 && eb != 16) return fail(MS_ERR_UNSUPPORTED, "element size %u not in {4,8,16}", eb);
  if (n > kMaxN) return fail(MS_ERR_UNSUPPORTED, "n = %llu exceeds %llu", (unsigned long long)n,
                             (unsigned long long)kMaxN);
  uint32_t B = cfg && cfg->leaf_B ? cfg->leaf_B : kDefaultB;
  if (B + 1 > (uint32_t)leaf_max_block()) return fail(MS_ERR_UNSUPPORTED, "cutoff %u above %d", B, leaf_max_block() - 1);
  memset(&hp.pa, 0, sizeof hp.pa);
  hp.n = n;
  hp.eb = eb;
  hp.B = B;
  uint32_t c = 0;
  while ((n >> c) > B) ++c;
  hp.c = c;
  hp.q = 1ull << c;
  // the default super-block, or the 128 KiB one when a leaf does not fit
  // (16-byte leaves of cutoff + 1 = 4097 records)
  hp.leaf_big = leaf_big_default() || (cfg && (cfg->flags & MS_CFG_LEAF_BIG)) ||
                ceil_shift(n, c) > (uint64_t)leaf_capacity(eb, false);
  const uint64_t scap = (uint64_t)leaf_capacity(eb, hp.leaf_big);
  if (ceil_shift(n, c) > scap) return fail(MS_ERR_UNSUPPORTED, "leaf of %llu elements does not fit in LDS",
                                           (unsigned long long)ceil_shift(n, c));
  uint32_t lam_max = (uint32_t)leaf_max_levels();
  if (cfg && cfg->lds_levels_max && cfg->lds_levels_max < lam_max) lam_max = cfg->lds_levels_max;
  const bool r1 = cfg && (cfg->flags & MS_CFG_PLACEMENT_R1);
  const bool bal = cfg && (cfg->flags & MS_CFG_PLACEMENT_BALANCED);
  if (r1 && bal) return fail(MS_ERR_INVALID, "MS_CFG_PLACEMENT_R1 and MS_CFG_PLACEMENT_BALANCED together");
  if (cfg && (cfg->flags & MS_CFG_HBM_ONLY)) lam_max = 0;  // every merge level as an HBM pass
  if (r1 || bal) lam_max = 0;  // the leaf kernel's merge levels use the stable interleave
  uint32_t lam = 0;
  while (lam < c && lam < lam_max && ceil_shift(n, c - lam - 1) <= scap) ++lam;
  hp.lam = lam;
  hp.nlev = c - lam;
  PlanArgs& pa = hp.pa;
  pa.n = n;
  pa.c = c;
  pa.lds_levels = lam;
  pa.nlev = hp.nlev;
  const uint32_t T = (uint32_t)pass_tile(eb);
  uint64_t chunks = 0, merges = 0, buckets = 0, wgs = 0, cap = 0, tiles = 0;
  for (uint32_t l = 0; l < hp.nlev; ++l) {
    HbmLevel& lv = pa.lev[l];
    const uint32_t L = lam + 1 + l;
    lv.L = L;
    lv.nmerge = (uint32_t)(hp.q >> L);
    const uint64_t nmax = ceil_shift(n, c - L);
    lv.nmax = (uint32_t)nmax;
    lv.cpm = (uint32_t)ceil_shift(nmax + 1, kChunkLog);
    {
      uint32_t bl = 5;
      while (bl < 24 && (double)(1u << (bl + 1)) <= 2.5 * std::sqrt((double)nmax)) ++bl;
      lv.blog = bl;
    }
    lv.bpm = (uint32_t)ceil_shift(nmax, lv.blog);
    lv.tpm = (uint32_t)((nmax + T - 1) / T);
    const double ek = 0.8 * std::sqrt((double)nmax);
    lv.wpm = (uint32_t)std::max(1.0, std::ceil(ek / 1024.0));
    // merges of at most about 256 insertion steps: one to a wave, four to a
    // tail workgroup (most of a workgroup per merge would idle)
    lv.mpw = ek <= 256.0 ? 4u : 1u;
    lv.chunk_base = chunks;
    lv.merge_base = merges;
    lv.bucket_base = buckets;
    lv.wg_base = wgs;
    // insertion-loop steps of this level: about 0.8 sqrt(N) per merge; the
    // bound adds 0.4 sqrt(N) per merge and 14 sqrt(n) for the whole level
    double bnd = 1.2 * (double)lv.nmerge * std::sqrt((double)nmax) + 14.0 * std::sqrt((double)n) + 64.0;
    uint64_t lcap = (uint64_t)std::ceil(bnd);
    if (lcap > n) lcap = n;
    chunks += (uint64_t)lv.nmerge * lv.cpm;
    merges += lv.nmerge;
    buckets += (uint64_t)lv.nmerge * lv.bpm;
    wgs += (uint64_t)(lv.nmerge + lv.mpw - 1) / lv.mpw * lv.wpm;
    cap += lcap;
    tiles = std::max<uint64_t>(tiles, (uint64_t)lv.nmerge * lv.tpm);
  }
  // fused passes: groups of at most lpp consecutive HBM levels, sizes within
  // one; or one streaming pass and one patch kernel per level.  Default: 3,
  // and 4 at 13 or more HBM levels -- for 4-byte elements only when 3 does
  // not divide them (measured: a 4-level pass costs about as much per level
  // as a 3-level one, so fewer passes pay at the large sizes; for 4-byte
  // elements an even split by 3 is as fast, and at fewer levels the 4-level
  // tile's set-up does not pay)
  uint32_t lpp = 3u;
  if (cfg && cfg->levels_per_pass) lpp = cfg->levels_per_pass;
  else if (hp.nlev >= 13 && (eb != 4 || hp.nlev % 3 != 0)) lpp = 4u;
  if (lpp > (uint32_t)kGroupMax) lpp = kGroupMax;
  hp.fused = !(cfg && (cfg->flags & MS_CFG_ONE_LEVEL_PASSES)) && !r1 && !bal;
  pa.placement = r1 ? 1u : bal ? 2u : 0u;
  if (!hp.fused) lpp = 1;
  hp.ngroup = hp.nlev ? (hp.nlev + lpp - 1) / lpp : 0;
  {
    uint32_t l = 0;
    for (uint32_t g = 0; g < hp.ngroup; ++g) {
      const uint32_t sz = hp.nlev / hp.ngroup + (g < hp.nlev % hp.ngroup ? 1u : 0u);
      hp.gfirst[g] = l;
      hp.glam[g] = sz;
      for (uint32_t k = 0; k < sz; ++k) pa.lev[l + k].group_bottom = k == 0 ? 1u : 0u;
      l += sz;
    }
  }
  uint64_t all_bnd = 0, all_desc = 0;
  if (hp.fused) {
    const uint32_t Tg = (uint32_t)fused_tile(eb, n);
    tiles = 0;
    for (uint32_t g = 0; g < hp.ngroup; ++g) {
      const HbmLevel& top = pa.lev[hp.gfirst[g] + hp.glam[g] - 1];
      GroupInfo& gi = pa.grp[g];
      gi.lf = hp.gfirst[g];
      gi.lam = hp.glam[g];
      gi.T = Tg;
      gi.tpm = (top.nmax + Tg - 1) / Tg;
      gi.bnd_first = all_bnd;
      // the table pass reads one descriptor per tile, built by the plan
      hp.gdesc_words[g] = pass_tree() ? 0u : pass_desc_words(eb, Tg, (int)gi.lam);
      hp.gdesc_first[g] = all_desc;
      all_desc += (uint64_t)top.nmerge * gi.tpm * hp.gdesc_words[g];
      for (uint32_t k = 0; k < gi.lam; ++k) {
        pa.lev[gi.lf + k].grp = g;
        pa.lev[gi.lf + k].gli = k;
      }
      const uint64_t t = (uint64_t)top.nmerge * gi.tpm;
      all_bnd += (uint64_t)top.nmerge * (gi.tpm + 1);
      tiles = std::max<uint64_t>(tiles, t);
    }
    pa.ngroup = hp.ngroup;
  }
  pa.total_bnd = all_bnd;
  pa.total_desc = all_desc;
  pa.total_chunks = chunks;
  pa.total_merges = merges;
  pa.total_buckets = buckets;
  pa.total_tail_wgs = wgs;
  // MS_CAP_SCALE=f (0 < f < 1) shrinks both capacities by f: a test knob that
  // makes the overflow path (clamped writes, a status flag) reachable
  if (const char* e = getenv("MS_CAP_SCALE")) {
    const double f = atof(e);
    if (f > 0.0 && f < 1.0) cap = std::max<uint64_t>(1, (uint64_t)((double)cap * f));
  }
  pa.pool_cap = cap;
  pa.tail_cap = cap;
  hp.pass_tiles = tiles;
  Layout& y = hp.lay;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
  y.zloc = take(chunks * 256 * 2);
  y.ctot = take(chunks * 4);
  y.zc = take(chunks * 4);
  y.zg = take((chunks + 1) * 4);
  y.P = take(merges * 4);
  y.side = take(merges);
  y.kcnt = take(merges * 4);
  y.toff = take((merges + 1) * 4);
  y.tail_src = take(cap * 4);
  y.bcnt = take(buckets * 4);
  y.bfill = take(buckets * 4);
  y.boff = take((buckets + 1) * 4);
  y.part = take(((std::max(std::max(buckets, merges), chunks) + 2047) / 2048 + 1) * 4);
  y.pool_x = take(cap * 4);
  y.pool_step = take(cap * 4);
  y.pool_src = take(cap * 4);
  y.tail_xsrc = hp.fused ? take(cap * 4) : 0;
  y.pool_xsrc = hp.fused ? take(cap * 4) : 0;
  y.bnd = hp.fused ? take(all_bnd * kBndStride * 4) : 0;
  y.desc = hp.fused ? take(all_desc * 4) : 0;
  y.bits_part = take(kBitsParts * 8);
  y.lab = bal ? take(chunks * 1024 * 4) : 0;
  y.bytes = hp.nlev ? o : 0;
  return MS_OK;
}

uint64_t scratch_of(const HostPlan& hp) { return (hp.nlev ? hp.n * hp.eb : 0) + hp.lay.bytes; }

// ---------------------------------------------------------------------------
// per-device context and per-stream scratch
// ---------------------------------------------------------------------------
struct Arena {
  std::mutex mu;          // held for a whole call's launch sequence on this stream
  void* data = nullptr;   // array copy
  size_t data_bytes = 0;
  void* plan = nullptr;   // plan tables
  size_t plan_bytes = 0;
  // batched calls: descriptors, plan tables and array copies of one wave of
  // arrays, and two pinned staging buffers for the descriptors (each reused
  // once the copy out of it has run)
  void* wave = nullptr;
  size_t wave_bytes = 0;
  void* stage[2] = {nullptr, nullptr};
  size_t stage_bytes[2] = {0, 0};
  hipEvent_t stage_done[2] = {nullptr, nullptr};
  int stage_next = 0;
  // the plan runs on its own stream (default priority), forked from and
  // joined back into this one, so that it overlaps the leaf kernel
  hipStream_t plan_st = nullptr;
  hipEvent_t plan_fork = nullptr, plan_join = nullptr;
  // the status word of the calls made on this stream (byte 0) and a bit
  // counter for calls without one (byte 64)
  uint32_t* status = nullptr;
  // batched calls on this stream spread their large arrays over these
  // streams (default priority), forked from and joined back into this one;
  // side_mu is held from the fork to the join
  std::mutex side_mu;
  bool side_init = false;
  hipStream_t side[4] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[4] = {};
};

constexpr int kSideStreams = 4;

struct DeviceCtx {
  std::map<hipStream_t, Arena> arenas;
};

std::mutex g_mu;
DeviceCtx g_dev[64];

struct ProfRec {
  int cls;
  hipEvent_t a, b;
};
bool g_prof = false;
std::vector<ProfRec> g_prof_recs;
std::mutex g_prof_mu;

int device_ctx(DeviceCtx** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(MS_ERR_HIP, "device %d out of range", dev);
  *out = &g_dev[dev];
  return MS_OK;
}

// The arena of stream st on the current device (created empty on first use)
// with its status word allocated.
int arena_of(hipStream_t st, Arena** out) {
  DeviceCtx* dc;
  int rc;
  Arena* ar;
  {
    // g_mu, not the arena's own locks: a batched call holds side_mu while
    // its waves look up the same arena
    std::lock_guard<std::mutex> lk(g_mu);
    if ((rc = device_ctx(&dc))) return rc;
    ar = &dc->arenas[st];  // map nodes do not move
    if (!ar->status) {
      if (getenv("MS_FAIL_ALLOC")) return fail(MS_ERR_NOMEM, "status allocation refused (MS_FAIL_ALLOC)");
      hipError_t e = hipMalloc(&ar->status, 256);
      if (e != hipSuccess) {
        ar->status = nullptr;
        (void)hipGetLastError();
        return fail(MS_ERR_NOMEM, "hipMalloc(256): %s", hipGetErrorString(e));
      }
      HIP_TRY(hipMemset(ar->status, 0, 256));
    }
  }
  *out = ar;
  return MS_OK;
}

unsigned long long* dummy_bits_of(const Arena& ar) {
  return reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(ar.status) + 64);
}

int ensure(void** p, size_t* have, size_t need, hipStream_t st) {
  if (need <= *have) return MS_OK;
  if (*p) {
    HIP_TRY(hipStreamSynchronize(st));
    HIP_TRY(hipFree(*p));
    *p = nullptr;
    *have = 0;
  }
  if (getenv("MS_FAIL_ALLOC")) return fail(MS_ERR_NOMEM, "scratch allocation of %zu bytes refused (MS_FAIL_ALLOC)", need);
  hipError_t e = hipMalloc(p, need);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(MS_ERR_NOMEM, "hipMalloc(%zu): %s", need, hipGetErrorString(e));
  }
  *have = need;
  return MS_OK;
}

struct ProfScope {
  int cls;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(int c, hipStream_t s) : cls(c), st(s) {
    if (!g_prof || c < 0) return;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) { a = b = nullptr; return; }
    (void)hipEventRecord(a, st);
  }
  ~ProfScope() {
    if (!a) return;
    (void)hipEventRecord(b, st);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_recs.push_back({cls, a, b});
  }
};

// Point the plan's device arrays into a plan area of hp.lay.bytes bytes.
void bind_plan(HostPlan& hp, void* area) {
  PlanArgs& pa = hp.pa;
  char* b = reinterpret_cast<char*>(area);
  const Layout& y = hp.lay;
  pa.zloc = reinterpret_cast<uint16_t*>(b + y.zloc);
  pa.ctot = reinterpret_cast<uint32_t*>(b + y.ctot);
  pa.zc = reinterpret_cast<uint32_t*>(b + y.zc);
  pa.zg = reinterpret_cast<uint32_t*>(b + y.zg);
  pa.P = reinterpret_cast<uint32_t*>(b + y.P);
  pa.side = reinterpret_cast<uint8_t*>(b + y.side);
  pa.kcnt = reinterpret_cast<uint32_t*>(b + y.kcnt);
  pa.toff = reinterpret_cast<uint32_t*>(b + y.toff);
  pa.tail_src = reinterpret_cast<uint32_t*>(b + y.tail_src);
  pa.bcnt = reinterpret_cast<uint32_t*>(b + y.bcnt);
  pa.bfill = reinterpret_cast<uint32_t*>(b + y.bfill);
  pa.boff = reinterpret_cast<uint32_t*>(b + y.boff);
  pa.part = reinterpret_cast<uint32_t*>(b + y.part);
  pa.pool_x = reinterpret_cast<uint32_t*>(b + y.pool_x);
  pa.pool_step = reinterpret_cast<uint32_t*>(b + y.pool_step);
  pa.pool_src = reinterpret_cast<uint32_t*>(b + y.pool_src);
  pa.tail_xsrc = hp.fused ? reinterpret_cast<uint32_t*>(b + y.tail_xsrc) : nullptr;
  pa.pool_xsrc = hp.fused ? reinterpret_cast<uint32_t*>(b + y.pool_xsrc) : nullptr;
  pa.bnd = hp.fused ? reinterpret_cast<uint32_t*>(b + y.bnd) : nullptr;
  pa.desc = hp.fused ? reinterpret_cast<uint32_t*>(b + y.desc) : nullptr;
  pa.bits_part = reinterpret_cast<unsigned long long*>(b + y.bits_part);
  pa.lab = pa.placement == 2 ? reinterpret_cast<uint32_t*>(b + y.lab) : nullptr;
}

// Arguments of fused pass g, reading cur and writing other.
GroupArgs group_args(const HostPlan& hp, uint32_t g, const void* cur, void* other) {
  const PlanArgs& pa = hp.pa;
  GroupArgs ga;
  memset(&ga, 0, sizeof ga);
  const GroupInfo& gi = pa.grp[g];
  ga.X = cur;
  ga.Z = other;
  ga.n = hp.n;
  ga.c = hp.c;
  ga.tpm = gi.tpm;
  ga.ntiles = (uint32_t)((uint64_t)pa.lev[gi.lf + gi.lam - 1].nmerge * gi.tpm);
  ga.key0 = pa.key0;
  ga.key1 = pa.key1;
  ga.vec_ok = ((uintptr_t)cur % 16 == 0 && (uintptr_t)other % 16 == 0) ? 1u : 0u;
  ga.P = pa.P;
  ga.side = pa.side;
  ga.bnd = pa.bnd + gi.bnd_first * kBndStride;
  ga.toff = pa.toff;
  ga.tail_xsrc = pa.tail_xsrc;
  ga.boff = pa.boff;
  ga.pool_x = pa.pool_x;
  ga.pool_xsrc = pa.pool_xsrc;
  ga.tail_cap = pa.tail_cap;
  ga.pool_cap = pa.pool_cap;
  ga.desc = pa.desc ? pa.desc + hp.gdesc_first[g] : nullptr;
  ga.desc_words = hp.gdesc_words[g];
  for (uint32_t k = 0; k < gi.lam; ++k) {
    const HbmLevel& lv = pa.lev[gi.lf + k];
    ga.L[k] = lv.L;
    ga.blog[k] = lv.blog;
    ga.bpm[k] = lv.bpm;
    ga.merge_base[k] = lv.merge_base;
    ga.bucket_base[k] = lv.bucket_base;
  }
  return ga;
}

// The launch sequence of one call: the plan (on plan_st, forked from and
// joined back into st by the two events, or on st itself when plan_st is
// null), the leaf kernel and the HBM passes, alternating between the
// caller's array X and the scratch copy Y so that the last pass lands in X.
// plan_area holds hp.lay.bytes bytes.  `prof` brackets the launches with
// timing events when profiling is on.
int enqueue_call(HostPlan& hp, void* X, void* Y, void* plan_area, uint64_t seed, hipStream_t st,
                 hipStream_t plan_st, hipEvent_t plan_fork, hipEvent_t plan_join, unsigned long long* bits,
                 uint32_t* status, bool ident, bool prof) {
  const uint64_t n = hp.n;
  const uint32_t eb = hp.eb;
  PlanArgs& pa = hp.pa;
  pa.key0 = (uint32_t)seed;
  pa.key1 = (uint32_t)(seed >> 32);
  pa.bits = bits;
  pa.status = status;
  const bool fork = hp.nlev && plan_st;
  if (hp.nlev) {
    bind_plan(hp, plan_area);
    // the plan depends only on (n, cutoff, seed), the leaf kernel only on
    // the data: with a plan stream the plan runs beside the leaf kernel and
    // the first HBM pass waits for it
    if (fork) {
      HIP_TRY(hipEventRecord(plan_fork, st));
      HIP_TRY(hipStreamWaitEvent(plan_st, plan_fork, 0));
    }
    {
      ProfScope ps(prof ? 0 : -1, fork ? plan_st : st);
      launch_plan(pa, fork ? plan_st : st);
      // the tile descriptors of every fused pass (each pass reads the
      // buffer the previous one wrote: the same alternation as below)
      if (hp.fused && !pass_tree()) {
        void* c = (hp.ngroup % 2 == 0) ? X : Y;
        for (uint32_t g = 0; g < hp.ngroup; ++g) {
          void* o = c == X ? Y : X;
          const GroupInfo& gi = pa.grp[g];
          const GroupArgs ga = group_args(hp, g, c, o);
          launch_pass_desc(ga, (int)gi.lam, eb, gi.T, (uint64_t)pa.lev[gi.lf + gi.lam - 1].nmerge * gi.tpm,
                           fork ? plan_st : st);
          c = o;
        }
      }
    }
    if (fork) HIP_TRY(hipEventRecord(plan_join, plan_st));
  }
  const uint32_t npass = hp.fused ? hp.ngroup : hp.nlev;
  void* cur = (npass % 2 == 0) ? X : Y;
  {
    LeafArgs la;
    la.in = X;
    la.out = cur;
    la.n = n;
    la.c = hp.c;
    la.lds_levels = hp.lam;
    la.key0 = pa.key0;
    la.key1 = pa.key1;
    la.bits = bits;
    la.status = status;
    ProfScope ps(prof ? 1 : -1, st);
    launch_leaf(la, eb, ident, hp.leaf_big, hp.q >> hp.lam, st);
  }
  if (fork) HIP_TRY(hipStreamWaitEvent(st, plan_join, 0));
  for (uint32_t g = 0; hp.fused && g < hp.ngroup; ++g) {
    void* other = cur == X ? Y : X;
    const GroupInfo& gi = pa.grp[g];
    const GroupArgs ga = group_args(hp, g, cur, other);
    const HbmLevel& top = pa.lev[gi.lf + gi.lam - 1];
    {
      ProfScope ps(prof ? 2 : -1, st);
      launch_fused(ga, (int)gi.lam, eb, gi.T, (uint64_t)top.nmerge * gi.tpm, st);
    }
    cur = other;
  }
  for (uint32_t l = 0; !hp.fused && l < hp.nlev; ++l) {
    void* other = cur == X ? Y : X;
    const HbmLevel& lv = pa.lev[l];
    PassArgs a;
    a.in = cur;
    a.out = other;
    a.n = n;
    a.c = hp.c;
    a.L = lv.L;
    a.tpm = lv.tpm;
    a.cpm = lv.cpm;
    a.chunk_base = lv.chunk_base;
    a.merge_base = lv.merge_base;
    a.zloc = pa.zloc;
    a.zc = pa.zc;
    a.P = pa.P;
    a.side = pa.side;
    a.key0 = pa.key0;
    a.key1 = pa.key1;
    a.vec_ok = ((uintptr_t)cur % 16 == 0) ? 1u : 0u;
    a.lab = pa.placement == 2 ? pa.lab : nullptr;
    {
      ProfScope ps(prof ? 2 : -1, st);
      if (pa.placement == 1) launch_merge_r1(pa, (int)l, cur, other, eb, st);
      else launch_merge_pass(a, eb, (uint64_t)lv.nmerge * lv.tpm, st);
    }
    if (pa.placement != 2) {
      // (BalancedShuffle's labels already hold the insertion loop)
      ProfScope ps(prof ? 3 : -1, st);
      launch_patch(pa, (int)l, cur, other, eb, st);
    }
    cur = other;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(MS_ERR_HIP, "kernel launch: %s", hipGetErrorString(e));
  return MS_OK;
}

int check_args(const HostPlan& hp, const void* ptr) {
  if (hp.n > 0 && ptr == nullptr) return fail(MS_ERR_INVALID, "null pointer with n = %llu", (unsigned long long)hp.n);
  if (((uintptr_t)ptr) % hp.eb != 0) return fail(MS_ERR_INVALID, "pointer not aligned to %u bytes", hp.eb);
  return MS_OK;
}

// status: the word the call's kernels flag (null: the stream's own).
int run_one(void* ptr, uint64_t n, uint32_t eb, uint64_t seed, hipStream_t st, const ms_config* cfg,
            unsigned long long* d_bits, bool ident, uint32_t* status = nullptr) {
  HostPlan hp;
  int rc = make_plan(n, eb, cfg, hp);
  if (rc) return rc;
  if ((rc = check_args(hp, ptr))) return rc;
  if (n <= 1) return MS_OK;
  Arena* arp;
  if ((rc = arena_of(st, &arp))) return rc;
  // the stream's scratch is this call's until its launches are queued
  std::lock_guard<std::mutex> alk(arp->mu);
  Arena& ar = *arp;
  if ((rc = ensure(&ar.data, &ar.data_bytes, hp.nlev ? n * eb : 0, st))) return rc;
  if ((rc = ensure(&ar.plan, &ar.plan_bytes, hp.lay.bytes, st))) return rc;
  if (hp.nlev && !ar.plan_st) {
    HIP_TRY(hipStreamCreateWithFlags(&ar.plan_st, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&ar.plan_fork, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&ar.plan_join, hipEventDisableTiming));
  }
  return enqueue_call(hp, ptr, ar.data, ar.plan, seed, st, ar.plan_st, ar.plan_fork, ar.plan_join,
                      d_bits ? d_bits : dummy_bits_of(ar), status ? status : ar.status, ident, true);
}

// ---------------------------------------------------------------------------
// calls that allocate nothing: scratch in a fixed device array
// ---------------------------------------------------------------------------
// Layout: the status word (byte 0) and a bit counter for calls without one
// (byte 64) in the first 256 bytes, then the array copy, then the plan.
constexpr size_t kNoAllocBytes = 64ull << 20;
constexpr size_t kNoAllocHead = 256;
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// Device address of `scratch` on each device (its host-side name is not a
// device address), resolved once per device with that device current.
void* g_noalloc_ptr[64] = {};

int noalloc_area(char** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(MS_ERR_HIP, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(MS_ERR_HIP, "hipGetSymbolAddress(scratch) gave a null address");
    g_noalloc_ptr[dev] = p;
  }
  *out = reinterpret_cast<char*>(g_noalloc_ptr[dev]);
  return MS_OK;
}

int run_noalloc(void* ptr, uint64_t n, uint32_t eb, uint64_t seed, hipStream_t st, const ms_config* cfg,
                unsigned long long* d_bits) {
  HostPlan hp;
  int rc = make_plan(n, eb, cfg, hp);
  if (rc) return rc;
  if ((rc = check_args(hp, ptr))) return rc;
  const size_t data = hp.nlev ? align256(n * eb) : 0;
  const size_t need = kNoAllocHead + data + hp.lay.bytes;
  if (need > kNoAllocBytes)
    return fail(MS_ERR_UNSUPPORTED, "n = %llu needs %zu bytes of scratch, above the %zu of the allocation-free entry point",
                (unsigned long long)n, need, kNoAllocBytes);
  if (n <= 1) return MS_OK;
  char* area;
  if ((rc = noalloc_area(&area))) return rc;
  unsigned long long* bits = d_bits ? d_bits : reinterpret_cast<unsigned long long*>(area + 64);
  uint32_t* status = reinterpret_cast<uint32_t*>(area);
  // every kernel on the caller's stream, in order; no events, no profiling
  return enqueue_call(hp, ptr, area + kNoAllocHead, area + kNoAllocHead + data, seed, st, nullptr, nullptr,
                      nullptr, bits, status, false, false);
}

// The arrays of a batched call with at most kWaveMaxN elements run in
// waves: per wave, one launch per plan stage for all of its arrays that need
// HBM passes, one leaf launch per element size and one launch per (fused
// pass, element size, levels in the pass), so that the launch count does not
// grow with the number of arrays.  Every array has its own plan tables and
// array copy inside the wave's scratch.
constexpr uint64_t kWaveMaxN = 1ull << 21;
constexpr size_t kWaveScratch = 4ull << 30;
constexpr uint32_t kWaveMaxArrays = 8192;

// Arrays per wave: kWaveMaxArrays, or fewer through MS_WAVE_ARRAYS (a tuning
// and testing knob; the permutations do not depend on it).
uint32_t wave_max_arrays() {
  const char* e = getenv("MS_WAVE_ARRAYS");
  const long v = e ? atol(e) : 0;
  return v > 0 && v < (long)kWaveMaxArrays ? (uint32_t)v : kWaveMaxArrays;
}

bool wave_eligible(const HostPlan& hp) { return hp.n <= kWaveMaxN && (hp.nlev == 0 || hp.fused); }

int stage_buffer(Arena& ar, size_t bytes, void** out, int* which) {
  const int i = ar.stage_next;
  ar.stage_next ^= 1;
  if (!ar.stage_done[i]) HIP_TRY(hipEventCreateWithFlags(&ar.stage_done[i], hipEventDisableTiming));
  // the copy that last read this buffer must have run before it is rewritten
  HIP_TRY(hipEventSynchronize(ar.stage_done[i]));
  if (ar.stage_bytes[i] < bytes) {
    if (ar.stage[i]) HIP_TRY(hipHostFree(ar.stage[i]));
    ar.stage[i] = nullptr;
    ar.stage_bytes[i] = 0;
    if (getenv("MS_FAIL_ALLOC")) return fail(MS_ERR_NOMEM, "staging allocation of %zu bytes refused (MS_FAIL_ALLOC)", bytes);
    hipError_t e = hipHostMalloc(&ar.stage[i], bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
      ar.stage[i] = nullptr;
      (void)hipGetLastError();
      return fail(MS_ERR_NOMEM, "hipHostMalloc(%zu): %s", bytes, hipGetErrorString(e));
    }
    ar.stage_bytes[i] = bytes;
  }
  *out = ar.stage[i];
  *which = i;
  return MS_OK;
}

// One wave of a batched call: arrays hps[i0 .. i1) with one device region
// holding, in order, the launch descriptors (plan arguments, unit prefixes,
// leaf and fused-pass arguments with their workgroup prefixes), then each
// array's plan tables, then each array's copy.
constexpr int kUnits = 5;    // plan stages launched per array
constexpr int kLeafCls = 6;  // leaf launch classes: element size x super-block size
struct GSec {
  size_t off = 0, tpre_off = 0;
  uint32_t n = 0, fill = 0, tiles = 0;
};
struct WaveLayout {
  size_t i0 = 0, i1 = 0;
  uint32_t np = 0;
  uint32_t nleaf[kLeafCls] = {0, 0, 0, 0, 0, 0};
  size_t pa_off = 0, pre_off[kUnits] = {}, leaf_off[kLeafCls] = {}, wpre_off[kLeafCls] = {};
  std::map<uint32_t, GSec> gsec;  // key (g * 3 + cls) * 4 + lam - 1, ordered by pass
  std::vector<size_t> plan_off, data_off;
  size_t desc_bytes = 0, bytes = 0;
  // set by wave_fill
  uint32_t units[kUnits] = {0, 0, 0, 0, 0};
  uint32_t lwg[kLeafCls] = {0, 0, 0, 0, 0, 0};
};

uint32_t cls_of(uint32_t eb) { return eb == 4 ? 0u : eb == 8 ? 1u : 2u; }
uint32_t leaf_cls(const HostPlan& hp) { return cls_of(hp.eb) * 2 + (hp.leaf_big ? 1u : 0u); }
uint32_t eb_of_cls(uint32_t cls) { return cls == 0 ? 4u : cls == 1 ? 8u : 16u; }

// The arrays of the wave that starts at i0 (at most wmax arrays and
// kWaveScratch bytes of plans and copies, at least one array).
size_t wave_end(const std::vector<HostPlan>& hps, size_t i0, uint32_t wmax) {
  size_t i1 = i0, scratch = 0;
  while (i1 < hps.size() && i1 - i0 < wmax) {
    const HostPlan& hp = hps[i1];
    const size_t need = hp.nlev ? align256(hp.lay.bytes) + align256(hp.n * hp.eb) : 0;
    if (i1 > i0 && scratch + need > kWaveScratch) break;
    scratch += need;
    ++i1;
  }
  return i1;
}

void wave_layout(const std::vector<HostPlan>& hps, size_t i0, size_t i1, WaveLayout& w) {
  w.i0 = i0;
  w.i1 = i1;
  std::map<uint32_t, uint32_t> gcount;
  for (size_t i = i0; i < i1; ++i) {
    const HostPlan& hp = hps[i];
    ++w.nleaf[leaf_cls(hp)];
    if (hp.nlev) ++w.np;
    for (uint32_t g = 0; g < hp.ngroup; ++g) ++gcount[(g * 3 + cls_of(hp.eb)) * 4 + hp.glam[g] - 1];
  }
  size_t o = 0;
  w.pa_off = o;
  o += align256((size_t)w.np * sizeof(PlanArgs));
  for (int k = 0; k < kUnits; ++k) {
    w.pre_off[k] = o;
    o += align256(((size_t)w.np + 1) * 4);
  }
  for (int c = 0; c < kLeafCls; ++c) {
    w.leaf_off[c] = o;
    o += align256((size_t)w.nleaf[c] * sizeof(LeafArgs));
    w.wpre_off[c] = o;
    o += align256(((size_t)w.nleaf[c] + 1) * 4);
  }
  for (const auto& kv : gcount) {
    GSec sc;
    sc.off = o;
    o += align256((size_t)kv.second * sizeof(GroupArgs));
    sc.tpre_off = o;
    o += align256(((size_t)kv.second + 1) * 4);
    sc.n = kv.second;
    w.gsec[kv.first] = sc;
  }
  w.desc_bytes = o;
  const size_t nw = i1 - i0;
  w.plan_off.assign(nw, 0);
  w.data_off.assign(nw, 0);
  for (size_t j = 0; j < nw; ++j) {
    if (!hps[i0 + j].nlev) continue;
    w.plan_off[j] = o;
    o += align256(hps[i0 + j].lay.bytes);
  }
  for (size_t j = 0; j < nw; ++j) {
    if (!hps[i0 + j].nlev) continue;
    w.data_off[j] = o;
    o += align256(hps[i0 + j].n * hps[i0 + j].eb);
  }
  w.bytes = o;
}

// Write the wave's descriptors to h (desc_bytes bytes, to be copied to the
// start of the device region d).  Array a = idx[i] uses seeds[a] (or seed +
// a), counts its bits in d_bits[a] (or `spare`) and flags `status`.
void wave_fill(std::vector<HostPlan>& hps, const std::vector<uint32_t>& idx, WaveLayout& w, char* h, char* d,
               void* const* ptrs, uint64_t seed, const uint64_t* seeds, unsigned long long* d_bits,
               unsigned long long* spare, uint32_t* status) {
  const size_t head = offsetof(PlanArgs, lev);
  uint32_t pfill = 0, lfill[kLeafCls] = {0, 0, 0, 0, 0, 0};
  for (auto& kv : w.gsec) kv.second.fill = kv.second.tiles = 0;
  for (int k = 0; k < kUnits; ++k) w.units[k] = 0;
  for (int c = 0; c < kLeafCls; ++c) w.lwg[c] = 0;
  for (size_t j = 0; j < w.i1 - w.i0; ++j) {
    HostPlan& hp = hps[w.i0 + j];
    const uint32_t a = idx[w.i0 + j];
    const uint64_t sa = seeds ? seeds[a] : seed + a;
    unsigned long long* bits = d_bits ? d_bits + a : spare;
    void* X = ptrs[a];
    void* Y = hp.nlev ? d + w.data_off[j] : X;
    void* cur = (hp.ngroup % 2 == 0) ? X : Y;
    PlanArgs& pa = hp.pa;
    pa.key0 = (uint32_t)sa;
    pa.key1 = (uint32_t)(sa >> 32);
    pa.bits = bits;
    pa.status = status;
    if (hp.nlev) {
      bind_plan(hp, d + w.plan_off[j]);
      // only the levels and passes in use are read on the device
      char* dst = h + w.pa_off + (size_t)pfill * sizeof(PlanArgs);
      memcpy(dst, &pa, head);
      memcpy(dst + head, pa.lev, hp.nlev * sizeof(HbmLevel));
      memcpy(dst + offsetof(PlanArgs, grp), pa.grp, hp.ngroup * sizeof(GroupInfo));
      const uint64_t per[kUnits] = {pa.total_chunks, (std::max(pa.total_chunks, pa.total_buckets) + 255) / 256,
                                    (pa.total_merges + 255) / 256, pa.total_tail_wgs,
                                    pa.total_tail_wgs + (pa.total_bnd + 255) / 256};
      for (int k = 0; k < kUnits; ++k) {
        reinterpret_cast<uint32_t*>(h + w.pre_off[k])[pfill] = w.units[k];
        w.units[k] += (uint32_t)per[k];
      }
      ++pfill;
    }
    LeafArgs la;
    la.in = X;
    la.out = cur;
    la.n = hp.n;
    la.c = hp.c;
    la.lds_levels = hp.lam;
    la.key0 = pa.key0;
    la.key1 = pa.key1;
    la.bits = bits;
    la.status = status;
    const uint32_t lc = leaf_cls(hp);
    memcpy(h + w.leaf_off[lc] + (size_t)lfill[lc] * sizeof(LeafArgs), &la, sizeof la);
    reinterpret_cast<uint32_t*>(h + w.wpre_off[lc])[lfill[lc]] = w.lwg[lc];
    ++lfill[lc];
    w.lwg[lc] += (uint32_t)(hp.q >> hp.lam);
    for (uint32_t g = 0; g < hp.ngroup; ++g) {
      void* other = cur == X ? Y : X;
      const GroupArgs ga = group_args(hp, g, cur, other);
      GSec& sc = w.gsec[(g * 3 + cls_of(hp.eb)) * 4 + hp.glam[g] - 1];
      memcpy(h + sc.off + (size_t)sc.fill * sizeof(GroupArgs), &ga, sizeof ga);
      reinterpret_cast<uint32_t*>(h + sc.tpre_off)[sc.fill] = sc.tiles;
      sc.tiles += ga.ntiles;
      ++sc.fill;
      cur = other;
    }
  }
  for (int k = 0; k < kUnits; ++k) reinterpret_cast<uint32_t*>(h + w.pre_off[k])[w.np] = w.units[k];
  for (int c = 0; c < kLeafCls; ++c) reinterpret_cast<uint32_t*>(h + w.wpre_off[c])[w.nleaf[c]] = w.lwg[c];
  for (auto& kv : w.gsec) reinterpret_cast<uint32_t*>(h + kv.second.tpre_off)[kv.second.n] = kv.second.tiles;
}

// The wave's launches on st, reading the descriptors at d: the plan stages
// and the pass descriptors of every array, the leaf kernels, the passes.
int wave_launch(const WaveLayout& w, char* d, hipStream_t st, bool prof) {
  if (w.np) {
    const uint32_t* pre[kUnits];
    for (int k = 0; k < kUnits; ++k) pre[k] = reinterpret_cast<const uint32_t*>(d + w.pre_off[k]);
    ProfScope ps(prof ? 0 : -1, st);
    launch_plan_multi(reinterpret_cast<const PlanArgs*>(d + w.pa_off), w.np, pre, w.units, st);
    if (!pass_tree()) {
      for (const auto& kv : w.gsec) {
        const uint32_t key = kv.first;
        const uint32_t lam = key % 4 + 1, cls = (key / 4) % 3;
        launch_pass_desc_multi(reinterpret_cast<const GroupArgs*>(d + kv.second.off),
                               reinterpret_cast<const uint32_t*>(d + kv.second.tpre_off), kv.second.n,
                               kv.second.tiles, (int)lam, eb_of_cls(cls), st);
      }
    }
  }
  for (int c = 0; c < kLeafCls; ++c) {
    if (!w.nleaf[c]) continue;
    ProfScope ps(prof ? 1 : -1, st);
    launch_leaf_multi(reinterpret_cast<const LeafArgs*>(d + w.leaf_off[c]),
                      reinterpret_cast<const uint32_t*>(d + w.wpre_off[c]), w.nleaf[c], w.lwg[c],
                      eb_of_cls((uint32_t)c / 2), (c & 1) != 0, st);
  }
  for (const auto& kv : w.gsec) {
    const uint32_t key = kv.first;
    const uint32_t lam = key % 4 + 1, cls = (key / 4) % 3;
    ProfScope ps(prof ? 2 : -1, st);
    launch_fused_multi(reinterpret_cast<const GroupArgs*>(d + kv.second.off),
                       reinterpret_cast<const uint32_t*>(d + kv.second.tpre_off), kv.second.n, kv.second.tiles,
                       (int)lam, eb_of_cls(cls), st);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(MS_ERR_HIP, "kernel launch: %s", hipGetErrorString(e));
  return MS_OK;
}

// The waves of a batched call on st: each wave's descriptors go through a
// pinned staging buffer into the stream's wave region, then its launches.
// seeds: per-array seeds, or null for seed + array index.
int run_waves(void* const* ptrs, std::vector<HostPlan>& hps, const std::vector<uint32_t>& idx, uint64_t seed,
              const uint64_t* seeds, hipStream_t st, unsigned long long* d_bits) {
  Arena* arp;
  int rc0;
  if ((rc0 = arena_of(st, &arp))) return rc0;
  std::lock_guard<std::mutex> alk(arp->mu);
  Arena& ar = *arp;
  const uint32_t wmax = wave_max_arrays();
  size_t i0 = 0;
  while (i0 < idx.size()) {
    WaveLayout w;
    wave_layout(hps, i0, wave_end(hps, i0, wmax), w);
    int rc;
    if ((rc = ensure(&ar.wave, &ar.wave_bytes, w.bytes, st))) return rc;
    void* stg = nullptr;
    int si = 0;
    if ((rc = stage_buffer(ar, w.desc_bytes, &stg, &si))) return rc;
    char* h = reinterpret_cast<char*>(stg);
    char* d = reinterpret_cast<char*>(ar.wave);
    wave_fill(hps, idx, w, h, d, ptrs, seed, seeds, d_bits, dummy_bits_of(ar), ar.status);
    HIP_TRY(hipMemcpyAsync(d, h, w.desc_bytes, hipMemcpyHostToDevice, st));
    HIP_TRY(hipEventRecord(ar.stage_done[si], st));
    if ((rc = wave_launch(w, d, st, true))) return rc;
    i0 = w.i1;
  }
  return MS_OK;
}

// ---------------------------------------------------------------------------
// batched calls captured once in a HIP graph and replayed
// ---------------------------------------------------------------------------
// The graph owns every buffer its kernels touch besides the arrays: each
// wave's region (descriptors written once, at creation), each full-path
// array's plan tables and copy, and a status word.  Its nodes are kernel
// launches only (every clear is done by a kernel) and the event edges of
// the side streams the full-path arrays run on.
struct BatchGraph {
  int device = 0;
  std::vector<void*> bufs;
  uint32_t* status = nullptr;  // status word (byte 0), spare bit counter (byte 64)
  hipStream_t cap = nullptr;
  hipStream_t side[kSideStreams] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kSideStreams] = {};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint64_t bytes = 0;
};

void graph_free(BatchGraph* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  for (void* b : g->bufs) (void)hipFree(b);
  if (g->status) (void)hipFree(g->status);
  for (int i = 0; i < kSideStreams; ++i) {
    if (g->side[i]) (void)hipStreamDestroy(g->side[i]);
    if (g->join[i]) (void)hipEventDestroy(g->join[i]);
  }
  if (g->fork) (void)hipEventDestroy(g->fork);
  if (g->cap) (void)hipStreamDestroy(g->cap);
  delete g;
}

int graph_alloc(BatchGraph* g, size_t bytes, void** out) {
  *out = nullptr;
  if (!bytes) return MS_OK;
  if (getenv("MS_FAIL_ALLOC")) return fail(MS_ERR_NOMEM, "graph scratch of %zu bytes refused (MS_FAIL_ALLOC)", bytes);
  hipError_t e = hipMalloc(out, bytes);
  if (e != hipSuccess) {
    *out = nullptr;
    (void)hipGetLastError();
    return fail(MS_ERR_NOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
  }
  g->bufs.push_back(*out);
  g->bytes += bytes;
  return MS_OK;
}

int graph_build(BatchGraph* g, void* const* ptrs, const uint64_t* sizes, const uint32_t* elem_bytes,
                const uint64_t* seeds, uint32_t count, const ms_config* cfgs, unsigned long long* d_bits) {
  std::vector<uint32_t> wave_idx, large;
  std::vector<HostPlan> wave_hp, large_hp;
  for (uint32_t a = 0; a < count; ++a) {
    HostPlan hp;
    const uint32_t eb = elem_bytes ? elem_bytes[a] : 4u;
    int rc = make_plan(sizes[a], eb, cfgs ? &cfgs[a] : nullptr, hp);
    if (rc) return fail(rc, "array %u: %s", a, g_err.c_str());
    if (sizes[a] > 0 && !ptrs[a]) return fail(MS_ERR_INVALID, "array %u: null pointer", a);
    if (((uintptr_t)ptrs[a]) % eb != 0) return fail(MS_ERR_INVALID, "array %u: pointer not aligned to %u bytes", a, eb);
    if (sizes[a] <= 1) continue;
    if (wave_eligible(hp)) {
      wave_idx.push_back(a);
      wave_hp.push_back(hp);
    } else {
      large.push_back(a);
      large_hp.push_back(hp);
    }
  }
  HIP_TRY(hipGetDevice(&g->device));
  {
    void* st = nullptr;
    int rc = graph_alloc(g, 256, &st);
    if (rc) return rc;
    g->bufs.pop_back();
    g->status = reinterpret_cast<uint32_t*>(st);
    HIP_TRY(hipMemset(g->status, 0, 256));
  }
  unsigned long long* spare = reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(g->status) + 64);
  HIP_TRY(hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking));
  HIP_TRY(hipEventCreateWithFlags(&g->fork, hipEventDisableTiming));
  for (int i = 0; i < kSideStreams; ++i) {
    HIP_TRY(hipStreamCreateWithFlags(&g->side[i], hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&g->join[i], hipEventDisableTiming));
  }
  // the waves' regions, descriptors written now
  std::vector<WaveLayout> waves;
  std::vector<char*> wave_d;
  const uint32_t wmax = wave_max_arrays();
  for (size_t i0 = 0; i0 < wave_idx.size();) {
    WaveLayout w;
    wave_layout(wave_hp, i0, wave_end(wave_hp, i0, wmax), w);
    void* d = nullptr;
    int rc = graph_alloc(g, w.bytes, &d);
    if (rc) return rc;
    std::vector<char> h(w.desc_bytes);
    wave_fill(wave_hp, wave_idx, w, h.data(), reinterpret_cast<char*>(d), ptrs, 0, seeds, d_bits, spare,
              g->status);
    HIP_TRY(hipMemcpy(d, h.data(), w.desc_bytes, hipMemcpyHostToDevice));
    i0 = w.i1;
    waves.push_back(std::move(w));
    wave_d.push_back(reinterpret_cast<char*>(d));
  }
  // the full-path arrays' plan tables and copies
  std::vector<void*> ldata(large.size()), lplan(large.size());
  for (size_t i = 0; i < large.size(); ++i) {
    const HostPlan& hp = large_hp[i];
    int rc;
    if ((rc = graph_alloc(g, hp.nlev ? hp.n * hp.eb : 0, &ldata[i]))) return rc;
    if ((rc = graph_alloc(g, hp.lay.bytes, &lplan[i]))) return rc;
  }
  // capture: full-path arrays on the side streams, waves on the capture stream
  HIP_TRY(hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal));
  const bool side = !large.empty();
  int err = MS_OK;
  if (side) {
    if (hipEventRecord(g->fork, g->cap) != hipSuccess) err = fail(MS_ERR_HIP, "event record in capture");
    for (int i = 0; i < kSideStreams && err == MS_OK; ++i)
      if (hipStreamWaitEvent(g->side[i], g->fork, 0) != hipSuccess) err = fail(MS_ERR_HIP, "stream wait in capture");
  }
  for (size_t i = 0; i < large.size() && err == MS_OK; ++i) {
    const uint32_t a = large[i];
    err = enqueue_call(large_hp[i], ptrs[a], ldata[i], lplan[i], seeds[a], g->side[i % kSideStreams], nullptr,
                       nullptr, nullptr, d_bits ? d_bits + a : spare, g->status, false, false);
  }
  for (size_t k = 0; k < waves.size() && err == MS_OK; ++k) err = wave_launch(waves[k], wave_d[k], g->cap, false);
  if (side) {
    for (int i = 0; i < kSideStreams; ++i) {
      if (hipEventRecord(g->join[i], g->side[i]) != hipSuccess ||
          hipStreamWaitEvent(g->cap, g->join[i], 0) != hipSuccess) {
        if (err == MS_OK) err = fail(MS_ERR_HIP, "join in capture");
      }
    }
  }
  const hipError_t ec = hipStreamEndCapture(g->cap, &g->graph);
  if (err != MS_OK) return err;
  if (ec != hipSuccess) return fail(MS_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(ec));
  HIP_TRY(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
  return MS_OK;
}

}  // namespace

extern "C" {

int ms_shuffle_ex(void* dev_ptr, uint64_t n, uint32_t elem_bytes, uint64_t seed, void* stream,
                  const ms_config* cfg, unsigned long long* d_bits) {
  g_err.clear();
  return run_one(dev_ptr, n, elem_bytes, seed, reinterpret_cast<hipStream_t>(stream), cfg, d_bits, false);
}

int ms_shuffle_noalloc(void* dev_ptr, uint64_t n, uint32_t elem_bytes, uint64_t seed, void* stream,
                       const ms_config* cfg, unsigned long long* d_bits) {
  g_err.clear();
  return run_noalloc(dev_ptr, n, elem_bytes, seed, reinterpret_cast<hipStream_t>(stream), cfg, d_bits);
}

int ms_shuffle(void* dev_ptr, uint64_t n, uint32_t elem_bytes, uint64_t seed, void* stream) {
  return ms_shuffle_ex(dev_ptr, n, elem_bytes, seed, stream, nullptr, nullptr);
}

int ms_permutation_ex(uint32_t* out, uint64_t n, uint64_t seed, void* stream, const ms_config* cfg,
                      unsigned long long* d_bits) {
  g_err.clear();
  return run_one(out, n, 4, seed, reinterpret_cast<hipStream_t>(stream), cfg, d_bits, true);
}

int ms_permutation(uint32_t* out, uint64_t n, uint64_t seed) {
  return ms_permutation_ex(out, n, seed, nullptr, nullptr, nullptr);
}

static int run_batched(void* const* ptrs, const uint64_t* sizes, const uint32_t* elem_bytes, uint32_t count,
                       uint64_t seed, const uint64_t* seeds, void* stream, const ms_config* cfg,
                       unsigned long long* d_bits_per_array);

int ms_shuffle_batched_ex(void* const* ptrs, const uint64_t* sizes, const uint32_t* elem_bytes, uint32_t count,
                          uint64_t seed, void* stream, const ms_config* cfg, unsigned long long* d_bits_per_array) {
  g_err.clear();
  return run_batched(ptrs, sizes, elem_bytes, count, seed, nullptr, stream, cfg, d_bits_per_array);
}

int ms_shuffle_batched_seeds(void* const* ptrs, const uint64_t* sizes, const uint32_t* elem_bytes,
                             const uint64_t* seeds, uint32_t count, void* stream, const ms_config* cfg,
                             unsigned long long* d_bits_per_array) {
  g_err.clear();
  if (count && !seeds) return fail(MS_ERR_INVALID, "null seed array");
  return run_batched(ptrs, sizes, elem_bytes, count, 0, seeds, stream, cfg, d_bits_per_array);
}

static int run_batched(void* const* ptrs, const uint64_t* sizes, const uint32_t* elem_bytes, uint32_t count,
                       uint64_t seed, const uint64_t* seeds, void* stream, const ms_config* cfg,
                       unsigned long long* d_bits_per_array) {
  if (count == 0) return MS_OK;
  if (!ptrs || !sizes) return fail(MS_ERR_INVALID, "null pointer or size array");
  const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  // every argument is checked before anything is launched
  std::vector<uint32_t> wave_idx, large;
  std::vector<HostPlan> wave_hp;
  wave_hp.reserve(count);
  {
    HostPlan hp;
    for (uint32_t a = 0; a < count; ++a) {
      const uint64_t n = sizes[a];
      const uint32_t eb = elem_bytes ? elem_bytes[a] : 4u;
      int rc = make_plan(n, eb, cfg, hp);
      if (rc) return fail(rc, "array %u: %s", a, g_err.c_str());
      if (n > 0 && !ptrs[a]) return fail(MS_ERR_INVALID, "array %u: null pointer", a);
      if (((uintptr_t)ptrs[a]) % eb != 0) return fail(MS_ERR_INVALID, "array %u: pointer not aligned to %u bytes", a, eb);
      if (n <= 1) continue;
      if (wave_eligible(hp)) {
        wave_idx.push_back(a);
        wave_hp.push_back(hp);
      } else {
        large.push_back(a);
      }
    }
  }
  Arena* car;  // the caller stream's arena: its side streams and status word
  {
    int rc;
    if ((rc = arena_of(st, &car))) return rc;
  }
  // the largest arrays take the full path each, spread over the caller
  // stream's side streams (forked from and joined back into it) so that
  // they overlap one another and the waves; the side streams and their
  // events belong to this stream, and side_mu keeps another call on it from
  // recording them in between
  const bool side = large.size() > 1 || (!large.empty() && !wave_idx.empty());
  std::unique_lock<std::mutex> slk(car->side_mu, std::defer_lock);
  if (side) {
    slk.lock();
    if (!car->side_init) {
      for (int i = 0; i < kSideStreams; ++i) {
        HIP_TRY(hipStreamCreateWithFlags(&car->side[i], hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&car->join[i], hipEventDisableTiming));
      }
      HIP_TRY(hipEventCreateWithFlags(&car->fork, hipEventDisableTiming));
      car->side_init = true;
    }
    HIP_TRY(hipEventRecord(car->fork, st));
    for (int i = 0; i < kSideStreams; ++i) HIP_TRY(hipStreamWaitEvent(car->side[i], car->fork, 0));
  }
  int err = MS_OK;
  for (size_t i = 0; i < large.size() && err == MS_OK; ++i) {
    const uint32_t a = large[i];
    const uint32_t eb = elem_bytes ? elem_bytes[a] : 4u;
    const hipStream_t s2 = side ? car->side[i % kSideStreams] : st;
    err = run_one(ptrs[a], sizes[a], eb, seeds ? seeds[a] : seed + a, s2, cfg,
                  d_bits_per_array ? d_bits_per_array + a : nullptr, false, car->status);
  }
  if (err == MS_OK && !wave_idx.empty())
    err = run_waves(ptrs, wave_hp, wave_idx, seed, seeds, st, d_bits_per_array);
  if (side) {
    // joined even after an error, so that the caller's stream still orders
    // after whatever was launched
    const std::string msg = g_err;
    for (int i = 0; i < kSideStreams; ++i) {
      HIP_TRY(hipEventRecord(car->join[i], car->side[i]));
      HIP_TRY(hipStreamWaitEvent(st, car->join[i], 0));
    }
    g_err = msg;
  }
  return err;
}

int ms_shuffle_batched(void* const* ptrs, const uint64_t* sizes, uint32_t count, uint64_t seed, void* stream) {
  return ms_shuffle_batched_ex(ptrs, sizes, nullptr, count, seed, stream, nullptr, nullptr);
}

int ms_batch_graph_create(void* const* ptrs, const uint64_t* sizes, const uint32_t* elem_bytes,
                          const uint64_t* seeds, uint32_t count, const ms_config* cfgs,
                          unsigned long long* d_bits_per_array, ms_batch_graph** out) {
  g_err.clear();
  if (!out) return fail(MS_ERR_INVALID, "null output handle");
  *out = nullptr;
  if (count && (!ptrs || !sizes || !seeds)) return fail(MS_ERR_INVALID, "null pointer, size or seed array");
  BatchGraph* g = new BatchGraph;
  const int rc = graph_build(g, ptrs, sizes, elem_bytes, seeds, count, cfgs, d_bits_per_array);
  if (rc != MS_OK) {
    const std::string msg = g_err;
    graph_free(g);
    g_err = msg;
    return rc;
  }
  *out = reinterpret_cast<ms_batch_graph*>(g);
  return MS_OK;
}

int ms_batch_graph_launch(ms_batch_graph* h, void* stream) {
  g_err.clear();
  BatchGraph* g = reinterpret_cast<BatchGraph*>(h);
  if (!g) return fail(MS_ERR_INVALID, "null graph");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != g->device) return fail(MS_ERR_INVALID, "graph built on device %d, launched on device %d", g->device, dev);
  HIP_TRY(hipGraphLaunch(g->exec, reinterpret_cast<hipStream_t>(stream)));
  return MS_OK;
}

int ms_batch_graph_status(ms_batch_graph* h, void* stream, uint32_t* flags) {
  g_err.clear();
  BatchGraph* g = reinterpret_cast<BatchGraph*>(h);
  if (!g || !flags) return fail(MS_ERR_INVALID, "null graph or output");
  HIP_TRY(hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)));
  uint32_t v = 0;
  HIP_TRY(hipMemcpy(&v, g->status, 4, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemset(g->status, 0, 4));
  *flags = v;
  return v ? MS_ERR_CAPACITY : MS_OK;
}

uint64_t ms_batch_graph_bytes(const ms_batch_graph* h) {
  const BatchGraph* g = reinterpret_cast<const BatchGraph*>(h);
  return g ? g->bytes : 0;
}

int ms_batch_graph_destroy(ms_batch_graph* h) {
  g_err.clear();
  BatchGraph* g = reinterpret_cast<BatchGraph*>(h);
  if (!g) return MS_OK;
  HIP_TRY(hipDeviceSynchronize());
  graph_free(g);
  return MS_OK;
}

int ms_plan(uint64_t n, uint32_t elem_bytes, const ms_config* cfg, ms_plan_info* out) {
  g_err.clear();
  if (!out) return fail(MS_ERR_INVALID, "null output");
  HostPlan hp;
  int rc = make_plan(n, elem_bytes, cfg, hp);
  if (rc) return rc;
  out->levels = hp.c;
  out->lds_levels = hp.lam;
  out->hbm_levels = hp.nlev;
  out->leaf_B = hp.B;
  out->leaves = hp.q;
  out->scratch_bytes = scratch_of(hp);
  out->pass_tiles = hp.pass_tiles;
  out->hbm_passes = hp.fused ? hp.ngroup : hp.nlev;
  out->max_levels_per_pass = hp.nlev ? 1u : 0u;
  for (uint32_t g = 0; hp.fused && g < hp.ngroup; ++g)
    out->max_levels_per_pass = std::max(out->max_levels_per_pass, hp.glam[g]);
  return MS_OK;
}

uint64_t ms_scratch_bytes(uint64_t n, uint32_t elem_bytes) {
  HostPlan hp;
  if (make_plan(n, elem_bytes, nullptr, hp)) return 0;
  return scratch_of(hp);
}

uint32_t ms_leaf_B_for(uint64_t n, uint32_t elem_bytes) {
  ms_tune_entry e;
  if (tune_lookup(n, elem_bytes, &e) && e.leaf_B) return e.leaf_B;
  return kDefaultB;
}

int ms_tune_set(const ms_tune_entry* entries, uint32_t count) {
  g_err.clear();
  if (count && !entries) return fail(MS_ERR_INVALID, "null entry array");
  std::map<uint64_t, ms_tune_entry> t;
  for (uint32_t i = 0; i < count; ++i) {
    const ms_tune_entry& e = entries[i];
    if (e.elem_bytes != 4 && e.elem_bytes != 8 && e.elem_bytes != 16)
      return fail(MS_ERR_INVALID, "entry %u: element size %u", i, e.elem_bytes);
    if (e.log2_n > 32) return fail(MS_ERR_INVALID, "entry %u: log2_n %u", i, e.log2_n);
    if (e.leaf_B == 0 || e.leaf_B + 1 > (uint32_t)leaf_max_block())
      return fail(MS_ERR_INVALID, "entry %u: cutoff %u", i, e.leaf_B);
    if (e.levels_per_pass > (uint32_t)kGroupMax) return fail(MS_ERR_INVALID, "entry %u: levels per pass %u", i, e.levels_per_pass);
    if (e.flags & ~MS_CFG_LEAF_BIG) return fail(MS_ERR_INVALID, "entry %u: flags %u", i, e.flags);
    t[((uint64_t)e.elem_bytes << 32) | e.log2_n] = e;
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.swap(t);
  return MS_OK;
}

int ms_device_status(void* stream, uint32_t* flags) {
  g_err.clear();
  const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  int rc;
  Arena* ar;
  if ((rc = arena_of(st, &ar))) return rc;
  HIP_TRY(hipStreamSynchronize(st));
  uint32_t v = 0, w = 0;
  HIP_TRY(hipMemcpy(&v, ar->status, 4, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemset(ar->status, 0, 4));
  // the allocation-free calls' flags, if that entry point has run on this device
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  void* na = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    na = g_noalloc_ptr[dev];
  }
  if (na) {
    HIP_TRY(hipMemcpy(&w, na, 4, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemset(na, 0, 4));
  }
  v |= w;
  if (flags) *flags = v;
  return v ? MS_ERR_CAPACITY : MS_OK;
}

int ms_release(void) {
  g_err.clear();
  std::lock_guard<std::mutex> lk(g_mu);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceSynchronize());
  DeviceCtx& d = g_dev[dev];
  for (auto& kv : d.arenas) {
    Arena& ar = kv.second;
    if (ar.data) HIP_TRY(hipFree(ar.data));
    if (ar.plan) HIP_TRY(hipFree(ar.plan));
    if (ar.wave) HIP_TRY(hipFree(ar.wave));
    for (int i = 0; i < 2; ++i) {
      if (ar.stage[i]) HIP_TRY(hipHostFree(ar.stage[i]));
      if (ar.stage_done[i]) HIP_TRY(hipEventDestroy(ar.stage_done[i]));
    }
    if (ar.plan_fork) HIP_TRY(hipEventDestroy(ar.plan_fork));
    if (ar.plan_join) HIP_TRY(hipEventDestroy(ar.plan_join));
    if (ar.plan_st) HIP_TRY(hipStreamDestroy(ar.plan_st));
    if (ar.status) HIP_TRY(hipFree(ar.status));
    if (ar.side_init) {
      for (int i = 0; i < kSideStreams; ++i) {
        HIP_TRY(hipStreamDestroy(ar.side[i]));
        HIP_TRY(hipEventDestroy(ar.join[i]));
      }
      HIP_TRY(hipEventDestroy(ar.fork));
    }
  }
  d.arenas.clear();
  return MS_OK;
}

const char* ms_last_error(void) { return g_err.c_str(); }

int ms_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_prof = on != 0;
  return MS_OK;
}

int ms_profile_read(double ms_per_class[4], uint64_t launches_per_class[4]) {
  g_err.clear();
  std::lock_guard<std::mutex> lk(g_mu);
  for (int i = 0; i < 4; ++i) {
    if (ms_per_class) ms_per_class[i] = 0.0;
    if (launches_per_class) launches_per_class[i] = 0;
  }
  int rc = MS_OK;
  for (auto& r : g_prof_recs) {
    float t = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) {
      rc = fail(MS_ERR_HIP, "profile event read failed");
    } else if (r.cls >= 0 && r.cls < 4) {
      if (ms_per_class) ms_per_class[r.cls] += t;
      if (launches_per_class) launches_per_class[r.cls] += 1;
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_prof_recs.clear();
  return rc;
}

}  // extern "C"
