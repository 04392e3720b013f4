// Drives the library's host runtime under AddressSanitizer and
// UndefinedBehaviorSanitizer without a GPU: the planner over the whole
// accepted size range, every element size and knob, the tuning table, and
// the argument checks of every entry point (each must fail before touching a
// device).
#include <cstdint>
#include <cstdio>
#include <vector>

#include "mergeshuffle.h"

static int bad = 0;
#define EXPECT(c)                                                  \
  do {                                                             \
    if (!(c)) {                                                    \
      std::printf("failed: %s (line %d)\n", #c, __LINE__);        \
      ++bad;                                                       \
    }                                                              \
  } while (0)

int main() {
  const uint32_t ebs[] = {4, 8, 16};
  const uint32_t flags[] = {0u, MS_CFG_HBM_ONLY, MS_CFG_ONE_LEVEL_PASSES, MS_CFG_PLACEMENT_R1,
                            MS_CFG_PLACEMENT_BALANCED, MS_CFG_LEAF_BIG, MS_CFG_TUNED};
  std::vector<uint64_t> sizes = {0, 1, 2, 3, 4096, 4097, 8193, 12289, 65537, 1000003, (1ull << 27) + 5,
                                 (1ull << 30), (1ull << 31) + 3, (1ull << 32) - (1ull << 16)};
  for (uint64_t n = 5; n < (1ull << 32); n = n * 3 + 1) sizes.push_back(n);
  for (uint64_t n : sizes)
    for (uint32_t eb : ebs)
      for (uint32_t f : flags)
        for (uint32_t B : {0u, 1u, 100u, 4096u})
          for (uint32_t lpp : {0u, 1u, 4u}) {
            ms_config c{B, lpp, 0, f};
            ms_plan_info info;
            const int rc = ms_plan(n, eb, &c, &info);
            EXPECT(rc == MS_OK);
            if (rc == MS_OK) EXPECT(info.lds_levels + info.hbm_levels == info.levels);
          }
  ms_plan_info info;
  EXPECT(ms_plan((1ull << 32) - (1ull << 16) + 1, 4, nullptr, &info) == MS_ERR_UNSUPPORTED);
  EXPECT(ms_plan(100, 3, nullptr, &info) == MS_ERR_UNSUPPORTED);
  {
    ms_config c{5000, 0, 0, 0};
    EXPECT(ms_plan(100, 4, &c, &info) == MS_ERR_UNSUPPORTED);
    ms_config both{0, 0, 0, MS_CFG_PLACEMENT_R1 | MS_CFG_PLACEMENT_BALANCED};
    EXPECT(ms_plan(100000, 4, &both, &info) == MS_ERR_INVALID);
  }
  EXPECT(ms_scratch_bytes(1ull << 30, 4) >= (4ull << 30));
  // tuning table
  ms_tune_entry good[2] = {{4, 12, 1000, 2, MS_CFG_LEAF_BIG}, {8, 20, 2048, 0, 0}};
  EXPECT(ms_tune_set(good, 2) == MS_OK);
  EXPECT(ms_leaf_B_for(5000, 4) == 1000 && ms_leaf_B_for(9000, 4) == 4096);
  ms_tune_entry badent = {4, 40, 10, 0, 0};
  EXPECT(ms_tune_set(&badent, 1) == MS_ERR_INVALID);
  EXPECT(ms_leaf_B_for(5000, 4) == 1000);
  EXPECT(ms_tune_set(nullptr, 0) == MS_OK);
  EXPECT(ms_leaf_B_for(5000, 4) == 4096);
  // argument checks that fail before any device work
  alignas(16) static uint32_t host[64];
  EXPECT(ms_shuffle(nullptr, 10, 4, 1, nullptr) == MS_ERR_INVALID);
  EXPECT(ms_shuffle(reinterpret_cast<char*>(host) + 2, 10, 4, 1, nullptr) == MS_ERR_INVALID);
  EXPECT(ms_shuffle(host, 10, 12, 1, nullptr) == MS_ERR_UNSUPPORTED);
  EXPECT(ms_shuffle(host, 1ull << 33, 4, 1, nullptr) == MS_ERR_UNSUPPORTED);
  EXPECT(ms_shuffle(host, 1, 4, 1, nullptr) == MS_OK);  // nothing to do
  EXPECT(ms_shuffle_noalloc(host, 1ull << 30, 4, 1, nullptr, nullptr, nullptr) == MS_ERR_UNSUPPORTED);
  {
    void* ptrs[3] = {host, nullptr, host};
    uint64_t sz[3] = {5, 7, 9};
    uint32_t eb[3] = {4, 4, 4};
    EXPECT(ms_shuffle_batched_ex(ptrs, sz, eb, 3, 1, nullptr, nullptr, nullptr) == MS_ERR_INVALID);
    uint64_t seeds[3] = {1, 2, 3};
    EXPECT(ms_shuffle_batched_seeds(ptrs, sz, eb, nullptr, 3, nullptr, nullptr, nullptr) == MS_ERR_INVALID);
    ms_batch_graph* g = nullptr;
    EXPECT(ms_batch_graph_create(ptrs, sz, eb, seeds, 3, nullptr, nullptr, &g) == MS_ERR_INVALID && !g);
    EXPECT(ms_batch_graph_create(ptrs, sz, eb, seeds, 3, nullptr, nullptr, nullptr) == MS_ERR_INVALID);
    EXPECT(ms_batch_graph_destroy(nullptr) == MS_OK);
  }
  EXPECT(ms_last_error() != nullptr);
  std::printf("host driver: %d bad\n", bad);
  return bad != 0;
}
