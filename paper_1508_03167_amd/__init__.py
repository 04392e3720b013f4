"""MergeShuffle (arXiv 1508.03167) for MI355X: HIP kernels behind a C ABI.

The array is cut into leaves shuffled by Fisher-Yates in LDS, then merged
level by level by random interleaving (Algorithm MergeShuffle, Algorithm 2).
See include/mergeshuffle.h for the C entry points; this package holds the
kernels (csrc/), their build (build.py) and a thin ctypes binding (_lib.py).
"""
from ._lib import (BatchGraph, MSConfig, MSError, config, device_status, leaf_B_for, lib, permutation, plan,
                   profile_enable, profile_read, release, scratch_bytes, shuffle_, shuffle_batched_,
                   shuffle_batched_seeds_, shuffle_noalloc_, tune_set)

__all__ = ["BatchGraph", "MSConfig", "MSError", "config", "device_status", "leaf_B_for", "lib", "permutation",
           "plan", "profile_enable", "profile_read", "release", "scratch_bytes", "shuffle_", "shuffle_batched_",
           "shuffle_batched_seeds_", "shuffle_noalloc_", "tune_set"]
