/* Drives the oracle under AddressSanitizer and UndefinedBehaviorSanitizer:
 * every placement over small and ragged sizes and many cutoffs, the merges
 * alone and the bounded draws; each permutation is checked to be one. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

uint64_t oracle_shuffle_u32(uint32_t *t, uint64_t n, uint64_t cutoff, uint64_t seed, int placement, int threads);
uint64_t oracle_merge_seeded(uint32_t *t, uint64_t n1, uint64_t n2, int placement, uint64_t seed, uint32_t L,
                             uint32_t m, uint64_t *bits);
uint64_t oracle_fisher_yates_seeded(uint32_t *t, uint64_t n, uint64_t seed, uint32_t unit);
uint64_t oracle_random_int(uint64_t seed, uint32_t L, uint32_t u, uint64_t d, uint64_t k, uint64_t *bits);

static int is_perm(const uint32_t *t, uint64_t n) {
  uint8_t *seen = calloc(n + 1, 1);
  int ok = 1;
  for (uint64_t i = 0; i < n && ok; i++) {
    if (t[i] >= n || seen[t[i]]) ok = 0;
    else seen[t[i]] = 1;
  }
  free(seen);
  return ok;
}

int main(void) {
  static const uint64_t sizes[] = {0, 1, 2, 3, 5, 17, 64, 100, 1000, 4095, 4096, 4097, 8193, 70001, 300007};
  static const uint64_t cutoffs[] = {1, 2, 3, 7, 100, 4096};
  int bad = 0;
  for (size_t a = 0; a < sizeof sizes / sizeof sizes[0]; a++) {
    for (size_t b = 0; b < sizeof cutoffs / sizeof cutoffs[0]; b++) {
      for (int placement = 0; placement < 3; placement++) {
        const uint64_t n = sizes[a];
        uint32_t *t = malloc((n + 1) * sizeof(uint32_t));
        for (uint64_t i = 0; i < n; i++) t[i] = (uint32_t)i;
        oracle_shuffle_u32(t, n, cutoffs[b], 7 + a * 31 + b, placement, 2);
        if (!is_perm(t, n)) {
          printf("not a permutation: n=%llu cutoff=%llu placement=%d\n", (unsigned long long)n,
                 (unsigned long long)cutoffs[b], placement);
          bad++;
        }
        free(t);
      }
    }
  }
  for (uint64_t n1 = 0; n1 < 40; n1 += 3) {
    for (uint64_t n2 = 0; n2 < 40; n2 += 5) {
      for (int placement = 0; placement < 3; placement++) {
        uint32_t *t = malloc((n1 + n2 + 1) * sizeof(uint32_t));
        uint64_t bits = 0;
        for (uint64_t i = 0; i < n1 + n2; i++) t[i] = (uint32_t)i;
        oracle_merge_seeded(t, n1, n2, placement, 99, 3, 5, &bits);
        if (!is_perm(t, n1 + n2)) bad++;
        free(t);
      }
    }
  }
  {
    uint32_t t[4097];
    for (int i = 0; i < 4097; i++) t[i] = (uint32_t)i;
    oracle_fisher_yates_seeded(t, 4097, 5, 3);
    if (!is_perm(t, 4097)) bad++;
    uint64_t bits = 0;
    for (uint64_t k = 1; k < 5000; k += 7)
      if (oracle_random_int(11, 0, 2, k, k, &bits) >= k) bad++;
    if (oracle_random_int(11, 0, 2, 1, 1ull << 32, &bits) >> 32) bad++;
  }
  printf("oracle driver: %d bad\n", bad);
  return bad != 0;
}
