"""ctypes access to the CPU oracle (ms_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the package's smoke() check
and by the cpu_baseline leg of bench.py; never by the product library.
The oracle replays MergeShuffle step by step (Algorithm 1, Algorithm 2 and
the listings of Appendix A) with the Philox stream rule described in
ms_oracle.c, and counts the fair bits it consumes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ms_oracle.c")
_LIB = os.path.join(_HERE, "libms_oracle.so")

R2 = 0  # stable interleave placement (the contract)
R1 = 1  # in-place swap placement of the printed listing
BALANCED = 2  # BalancedShuffle (Section 2): interleave by a uniform word of C(n1+n2, n1)

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP on, as in the paper's listing)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC]
        )
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        L.oracle_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.oracle_philox4x32_10.restype = None
        L.oracle_levels.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.oracle_levels.restype = ctypes.c_uint32
        L.oracle_shuffle_u32.argtypes = [u32p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                         ctypes.c_int, ctypes.c_int]
        L.oracle_shuffle_u32.restype = ctypes.c_uint64
        L.oracle_permutation.argtypes = [u32p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                         ctypes.c_int]
        L.oracle_permutation.restype = ctypes.c_uint64
        L.oracle_shuffle_scripted.argtypes = [u32p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                                              u32p, ctypes.c_uint32, u32p, u64p]
        L.oracle_shuffle_scripted.restype = ctypes.c_int
        L.oracle_merge_scripted.argtypes = [u32p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                                            u32p, ctypes.c_uint32, u64p]
        L.oracle_merge_scripted.restype = ctypes.c_uint64
        L.oracle_merge_seeded.argtypes = [u32p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                                          ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, u64p]
        L.oracle_merge_seeded.restype = ctypes.c_uint64
        L.oracle_fisher_yates_seeded.argtypes = [u32p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32]
        L.oracle_fisher_yates_seeded.restype = ctypes.c_uint64
        L.oracle_random_int.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                        ctypes.c_uint64, ctypes.c_uint64, u64p]
        L.oracle_random_int.restype = ctypes.c_uint64
        L.oracle_random_bit.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64]
        L.oracle_random_bit.restype = ctypes.c_int
        L.oracle_fdr_on_bits.argtypes = [ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint8), ctypes.c_uint32,
                                         u32p]
        L.oracle_fdr_on_bits.restype = ctypes.c_int64
        L.oracle_sample_permutations.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                                 ctypes.c_uint64, u32p, u64p]
        L.oracle_sample_permutations.restype = None
        L.oracle_max_threads.argtypes = []
        L.oracle_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _u32(a: np.ndarray):
    assert a.dtype == np.uint32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def philox4x32_10(ctr, key) -> tuple:
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    lib().oracle_philox4x32_10(c, k, o)
    return tuple(int(x) for x in o)


def levels(n: int, cutoff: int) -> int:
    return int(lib().oracle_levels(n, cutoff))


def shuffle_u32(a: np.ndarray, cutoff: int, seed: int, placement: int = R2, threads: int = 1) -> int:
    """Shuffle a (uint32, contiguous) in place; return the fair bits used."""
    return int(lib().oracle_shuffle_u32(_u32(a), a.size, cutoff, seed & (2**64 - 1), placement, threads))


def permutation(n: int, cutoff: int, seed: int, threads: int = 1):
    """(pi, bits): pi = the permutation MergeShuffle makes of 0..n-1."""
    out = np.empty(n, dtype=np.uint32)
    bits = int(lib().oracle_permutation(_u32(out), n, cutoff, seed & (2**64 - 1), threads))
    return out, bits


def shuffle_scripted(n: int, cutoff: int, script, placement: int = R2):
    """Run on 0..n-1 with scripted choices.  Returns (perm or None, consumed, need)."""
    arr = np.arange(n, dtype=np.uint32)
    sc = np.asarray(script, dtype=np.uint32)
    if sc.size == 0:
        sc = np.zeros(1, dtype=np.uint32)
        ln = 0
    else:
        ln = sc.size
    consumed = ctypes.c_uint32(0)
    need = ctypes.c_uint64(0)
    starved = lib().oracle_shuffle_scripted(_u32(arr), n, cutoff, placement, _u32(sc), ln,
                                            ctypes.byref(consumed), ctypes.byref(need))
    if starved:
        return None, int(consumed.value), int(need.value)
    return arr, int(consumed.value), 0


def merge_scripted(values, n1: int, script, placement: int = R2):
    """One Merge of values[:n1] and values[n1:] under a script.  (out, P) or (None, need)."""
    arr = np.ascontiguousarray(values, dtype=np.uint32).copy()
    sc = np.asarray(script, dtype=np.uint32)
    ln = sc.size
    if sc.size == 0:
        sc = np.zeros(1, dtype=np.uint32)
    need = ctypes.c_uint64(0)
    P = lib().oracle_merge_scripted(_u32(arr), n1, arr.size - n1, placement, _u32(sc), ln, ctypes.byref(need))
    if P == 2**64 - 1:
        return None, int(need.value)
    return arr, int(P)


def merge_seeded(values, n1: int, seed: int, L: int, m: int, placement: int = R2):
    """One Merge from the Philox streams of (seed, L, m).  Returns (out, P, bits)."""
    arr = np.ascontiguousarray(values, dtype=np.uint32).copy()
    bits = ctypes.c_uint64(0)
    P = lib().oracle_merge_seeded(_u32(arr), n1, arr.size - n1, placement, seed & (2**64 - 1), L, m,
                                  ctypes.byref(bits))
    return arr, int(P), int(bits.value)


def fisher_yates_seeded(values, seed: int, unit: int):
    arr = np.ascontiguousarray(values, dtype=np.uint32).copy()
    bits = int(lib().oracle_fisher_yates_seeded(_u32(arr), arr.size, seed & (2**64 - 1), unit))
    return arr, bits


def random_int(seed: int, L: int, unit: int, d: int, k: int):
    bits = ctypes.c_uint64(0)
    v = lib().oracle_random_int(seed & (2**64 - 1), L, unit, d, k, ctypes.byref(bits))
    return int(v), int(bits.value)


def random_bit(seed: int, L: int, m: int, t: int) -> int:
    return int(lib().oracle_random_bit(seed & (2**64 - 1), L, m, t))


def fdr_on_bits(k: int, bits):
    """Fast Dice Roller on an explicit bit list: (value or -1, bits read)."""
    b = (ctypes.c_uint8 * max(len(bits), 1))(*[int(x) for x in bits])
    used = ctypes.c_uint32(0)
    v = lib().oracle_fdr_on_bits(k, b, len(bits), ctypes.byref(used))
    return int(v), int(used.value)


def sample_permutations(n: int, cutoff: int, seed0: int, count: int):
    """(perms [count, n] uint32, bits [count]) for seeds seed0 .. seed0+count-1."""
    out = np.empty((count, n), dtype=np.uint32)
    bits = np.empty(count, dtype=np.uint64)
    lib().oracle_sample_permutations(n, cutoff, seed0, count, _u32(out),
                                     bits.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    return out, bits


def max_threads() -> int:
    return int(lib().oracle_max_threads())
