"""ctypes binding of libmergeshuffle.so (argument marshalling only).

Every step of the shuffle runs in the library's HIP kernels; this module only
turns torch tensors into device pointers and streams.  It raises if the
library is missing: there is no other implementation to fall back on.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmergeshuffle.so")

MS_OK = 0
MS_ERR_INVALID = -1
MS_ERR_UNSUPPORTED = -2
MS_ERR_NOMEM = -3
MS_ERR_HIP = -4
MS_ERR_CAPACITY = -5
MS_CFG_HBM_ONLY = 1
MS_CFG_ONE_LEVEL_PASSES = 2
MS_CFG_PLACEMENT_R1 = 4
MS_CFG_LEAF_BIG = 8
MS_CFG_TUNED = 16
MS_CFG_PLACEMENT_BALANCED = 32

SYMBOLS = [
    "ms_shuffle", "ms_permutation", "ms_shuffle_batched", "ms_shuffle_ex", "ms_permutation_ex",
    "ms_shuffle_batched_ex", "ms_plan", "ms_scratch_bytes", "ms_leaf_B_for", "ms_device_status",
    "ms_release", "ms_last_error", "ms_profile_enable", "ms_profile_read", "ms_shuffle_noalloc",
    "ms_shuffle_batched_seeds", "ms_batch_graph_create", "ms_batch_graph_launch", "ms_batch_graph_status",
    "ms_batch_graph_bytes", "ms_batch_graph_destroy", "ms_tune_set",
]
NOALLOC_SCRATCH_BYTES = 64 << 20


class MSConfig(ctypes.Structure):
    _fields_ = [("leaf_B", ctypes.c_uint32), ("levels_per_pass", ctypes.c_uint32),
                ("lds_levels_max", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


class MSTuneEntry(ctypes.Structure):
    _fields_ = [("elem_bytes", ctypes.c_uint32), ("log2_n", ctypes.c_uint32), ("leaf_B", ctypes.c_uint32),
                ("levels_per_pass", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


class MSPlanInfo(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_uint32), ("lds_levels", ctypes.c_uint32), ("hbm_levels", ctypes.c_uint32),
                ("leaf_B", ctypes.c_uint32), ("leaves", ctypes.c_uint64), ("scratch_bytes", ctypes.c_uint64),
                ("pass_tiles", ctypes.c_uint64), ("hbm_passes", ctypes.c_uint32),
                ("max_levels_per_pass", ctypes.c_uint32)]


class MSError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mergeshuffle error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1508_03167_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
        cfgp = ctypes.POINTER(MSConfig)
        L.ms_shuffle.argtypes = [vp, u64, u32, u64, vp]
        L.ms_permutation.argtypes = [vp, u64, u64]
        L.ms_shuffle_batched.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(u64), u32, u64, vp]
        L.ms_shuffle_ex.argtypes = [vp, u64, u32, u64, vp, cfgp, vp]
        L.ms_permutation_ex.argtypes = [vp, u64, u64, vp, cfgp, vp]
        L.ms_shuffle_batched_ex.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(u64), ctypes.POINTER(u32), u32,
                                            u64, vp, cfgp, vp]
        L.ms_shuffle_noalloc.argtypes = [vp, u64, u32, u64, vp, cfgp, vp]
        L.ms_shuffle_batched_seeds.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(u64), ctypes.POINTER(u32),
                                               ctypes.POINTER(u64), u32, vp, cfgp, vp]
        L.ms_batch_graph_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(u64), ctypes.POINTER(u32),
                                            ctypes.POINTER(u64), u32, cfgp, vp, ctypes.POINTER(vp)]
        L.ms_batch_graph_launch.argtypes = [vp, vp]
        L.ms_batch_graph_status.argtypes = [vp, vp, ctypes.POINTER(u32)]
        L.ms_batch_graph_bytes.argtypes = [vp]
        L.ms_batch_graph_bytes.restype = u64
        L.ms_batch_graph_destroy.argtypes = [vp]
        L.ms_tune_set.argtypes = [ctypes.POINTER(MSTuneEntry), u32]
        L.ms_plan.argtypes = [u64, u32, cfgp, ctypes.POINTER(MSPlanInfo)]
        L.ms_scratch_bytes.argtypes = [u64, u32]
        L.ms_scratch_bytes.restype = u64
        L.ms_leaf_B_for.argtypes = [u64, u32]
        L.ms_leaf_B_for.restype = u32
        L.ms_device_status.argtypes = [vp, ctypes.POINTER(u32)]
        L.ms_release.argtypes = []
        L.ms_last_error.argtypes = []
        L.ms_last_error.restype = ctypes.c_char_p
        L.ms_profile_enable.argtypes = [i32]
        L.ms_profile_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(u64)]
        for name in ("ms_shuffle", "ms_permutation", "ms_shuffle_batched", "ms_shuffle_ex", "ms_permutation_ex",
                     "ms_shuffle_noalloc", "ms_shuffle_batched_seeds", "ms_batch_graph_create",
                     "ms_batch_graph_launch", "ms_batch_graph_status", "ms_batch_graph_destroy", "ms_tune_set",
                     "ms_shuffle_batched_ex", "ms_plan", "ms_device_status", "ms_release", "ms_profile_enable",
                     "ms_profile_read"):
            getattr(L, name).restype = i32
        _lib = L
    return _lib


def _check(rc: int):
    if rc != MS_OK:
        raise MSError(rc, lib().ms_last_error().decode())


def _cfg(leaf_B=0, lds_levels_max=0, hbm_only=False, levels_per_pass=0, one_level_passes=False, placement="R2",
         leaf_big=False, tuned=False):
    if placement not in ("R1", "R2", "BAL"):
        raise ValueError(f"placement {placement!r} is none of 'R1', 'R2', 'BAL'")
    r1 = placement == "R1"
    bal = placement == "BAL"
    if not (leaf_B or lds_levels_max or hbm_only or levels_per_pass or one_level_passes or r1 or bal or leaf_big
            or tuned):
        return None
    flags = ((MS_CFG_HBM_ONLY if hbm_only else 0) | (MS_CFG_ONE_LEVEL_PASSES if one_level_passes else 0)
             | (MS_CFG_PLACEMENT_R1 if r1 else 0) | (MS_CFG_PLACEMENT_BALANCED if bal else 0)
             | (MS_CFG_LEAF_BIG if leaf_big else 0) | (MS_CFG_TUNED if tuned else 0))
    return ctypes.byref(MSConfig(leaf_B, levels_per_pass, lds_levels_max, flags))


def _stream(stream):
    import torch

    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def shuffle_(t, seed: int, *, stream=None, bits=None, leaf_B=0, lds_levels_max=0, hbm_only=False,
             levels_per_pass=0, one_level_passes=False, placement="R2", leaf_big=False, tuned=False):
    """Shuffle the contiguous device tensor t in place along its first dimension
    (row size 4, 8 or 16 bytes).  bits: optional int64 device tensor, += bits used.
    placement "R1" places each merge's elements as the printed listing's swaps do;
    "BAL" merges by BalancedShuffle's uniform word (Section 2)."""
    assert t.is_cuda and t.is_contiguous()
    eb = t.element_size() * (t[0].numel() if t.dim() > 1 else 1)
    n = t.shape[0]
    rc = lib().ms_shuffle_ex(_ptr(t), n, eb, seed & (2**64 - 1), _stream(stream),
                             _cfg(leaf_B, lds_levels_max, hbm_only, levels_per_pass, one_level_passes, placement,
                                  leaf_big, tuned),
                             ctypes.c_void_p(bits.data_ptr()) if bits is not None else None)
    _check(rc)
    return t


def shuffle_noalloc_(t, seed: int, *, stream=None, bits=None, leaf_B=0, lds_levels_max=0, hbm_only=False,
                     levels_per_pass=0, one_level_passes=False, placement="R2"):
    """As shuffle_, through the entry point that allocates nothing (scratch in a
    fixed 64 MiB device array shared by every such call on the device)."""
    assert t.is_cuda and t.is_contiguous()
    eb = t.element_size() * (t[0].numel() if t.dim() > 1 else 1)
    rc = lib().ms_shuffle_noalloc(_ptr(t), t.shape[0], eb, seed & (2**64 - 1), _stream(stream),
                                  _cfg(leaf_B, lds_levels_max, hbm_only, levels_per_pass, one_level_passes,
                                       placement),
                                  ctypes.c_void_p(bits.data_ptr()) if bits is not None else None)
    _check(rc)
    return t


def permutation(out, seed: int, *, stream=None, bits=None, leaf_B=0, lds_levels_max=0, hbm_only=False,
                levels_per_pass=0, one_level_passes=False, placement="R2", leaf_big=False, tuned=False):
    """Write MergeShuffle's permutation of 0..n-1 into the int32/uint32 device tensor out."""
    assert out.is_cuda and out.is_contiguous() and out.element_size() == 4
    rc = lib().ms_permutation_ex(_ptr(out), out.numel(), seed & (2**64 - 1), _stream(stream),
                                 _cfg(leaf_B, lds_levels_max, hbm_only, levels_per_pass, one_level_passes, placement,
                                      leaf_big, tuned),
                                 ctypes.c_void_p(bits.data_ptr()) if bits is not None else None)
    _check(rc)
    return out


def shuffle_batched_(tensors, seed: int, *, stream=None, bits=None, leaf_B=0, placement="R2", tuned=False):
    """Shuffle each device tensor of the list in place; tensor a uses seed + a
    (tuned=True: each array takes the tuning table's knobs for its size)."""
    cnt = len(tensors)
    ptrs = (ctypes.c_void_p * max(cnt, 1))(*[t.data_ptr() for t in tensors])
    sizes = (ctypes.c_uint64 * max(cnt, 1))(*[t.shape[0] for t in tensors])
    ebs = (ctypes.c_uint32 * max(cnt, 1))(
        *[t.element_size() * (t[0].numel() if t.dim() > 1 else 1) for t in tensors])
    rc = lib().ms_shuffle_batched_ex(ptrs, sizes, ebs, cnt, seed & (2**64 - 1), _stream(stream),
                                     _cfg(leaf_B, placement=placement, tuned=tuned),
                                     ctypes.c_void_p(bits.data_ptr()) if bits is not None else None)
    _check(rc)
    return tensors


def shuffle_batched_seeds_(tensors, seeds, *, stream=None, bits=None, leaf_B=0):
    """Shuffle each device tensor of the list in place; tensor a uses seeds[a]."""
    cnt = len(tensors)
    if len(seeds) != cnt:
        raise ValueError("one seed per tensor")
    ptrs = (ctypes.c_void_p * max(cnt, 1))(*[t.data_ptr() for t in tensors])
    sizes = (ctypes.c_uint64 * max(cnt, 1))(*[t.shape[0] for t in tensors])
    ebs = (ctypes.c_uint32 * max(cnt, 1))(
        *[t.element_size() * (t[0].numel() if t.dim() > 1 else 1) for t in tensors])
    sds = (ctypes.c_uint64 * max(cnt, 1))(*[int(s) & (2**64 - 1) for s in seeds])
    rc = lib().ms_shuffle_batched_seeds(ptrs, sizes, ebs, sds, cnt, _stream(stream), _cfg(leaf_B),
                                        ctypes.c_void_p(bits.data_ptr()) if bits is not None else None)
    _check(rc)
    return tensors


def _elem_bytes(t) -> int:
    return t.element_size() * (t[0].numel() if t.dim() > 1 else 1)


def config(leaf_B=0, levels_per_pass=0, lds_levels_max=0, flags=0, leaf_big=False, tuned=False) -> MSConfig:
    """An ms_config value (for per-array knobs)."""
    flags |= (MS_CFG_LEAF_BIG if leaf_big else 0) | (MS_CFG_TUNED if tuned else 0)
    return MSConfig(leaf_B, levels_per_pass, lds_levels_max, flags)


def tune_set(entries):
    """Replace the library's tuning table: entries are dicts with elem_bytes,
    log2_n, leaf_B, levels_per_pass and leaf_big."""
    arr = (MSTuneEntry * max(len(entries), 1))(
        *[MSTuneEntry(e["elem_bytes"], e["log2_n"], e["leaf_B"], e["levels_per_pass"],
                      MS_CFG_LEAF_BIG if e.get("leaf_big") else 0) for e in entries])
    _check(lib().ms_tune_set(arr, len(entries)))


def leaf_B_for(n: int, elem_bytes: int = 4) -> int:
    """The cutoff a call of this size with tuned knobs uses."""
    return int(lib().ms_leaf_B_for(n, elem_bytes))


class BatchGraph:
    """A batched call captured once in a HIP graph (ms_batch_graph_*): every
    launch() shuffles the same tensors in place again with the same seeds
    and knobs.  The tensors must outlive the graph; call destroy() (or use it
    as a context manager) to free its scratch."""

    def __init__(self, tensors, seeds, cfgs=None, bits=None):
        cnt = len(tensors)
        if len(seeds) != cnt or (cfgs is not None and len(cfgs) != cnt):
            raise ValueError("one seed (and one config, if given) per tensor")
        self.tensors = list(tensors)
        ptrs = (ctypes.c_void_p * max(cnt, 1))(*[t.data_ptr() for t in tensors])
        sizes = (ctypes.c_uint64 * max(cnt, 1))(*[t.shape[0] for t in tensors])
        ebs = (ctypes.c_uint32 * max(cnt, 1))(*[_elem_bytes(t) for t in tensors])
        sds = (ctypes.c_uint64 * max(cnt, 1))(*[int(s) & (2**64 - 1) for s in seeds])
        cf = None
        if cfgs is not None:
            arr = (MSConfig * max(cnt, 1))(*cfgs)
            cf = ctypes.cast(arr, ctypes.POINTER(MSConfig))
        h = ctypes.c_void_p()
        rc = lib().ms_batch_graph_create(ptrs, sizes, ebs, sds, cnt, cf,
                                         ctypes.c_void_p(bits.data_ptr()) if bits is not None else None,
                                         ctypes.byref(h))
        _check(rc)
        self.handle = h

    def launch(self, stream=None):
        _check(lib().ms_batch_graph_launch(self.handle, _stream(stream)))

    def status(self, stream=None) -> int:
        flags = ctypes.c_uint32(0)
        rc = lib().ms_batch_graph_status(self.handle, _stream(stream), ctypes.byref(flags))
        if rc not in (MS_OK, MS_ERR_CAPACITY):
            _check(rc)
        return int(flags.value)

    @property
    def scratch_bytes(self) -> int:
        return int(lib().ms_batch_graph_bytes(self.handle))

    def destroy(self):
        if self.handle:
            _check(lib().ms_batch_graph_destroy(self.handle))
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()


def scratch_bytes(n: int, elem_bytes: int = 4) -> int:
    """Library scratch a call of this size needs (0 if unsupported)."""
    return int(lib().ms_scratch_bytes(n, elem_bytes))


def plan(n: int, elem_bytes: int = 4, leaf_B=0, lds_levels_max=0, hbm_only=False, levels_per_pass=0,
         one_level_passes=False, placement="R2") -> dict:
    info = MSPlanInfo()
    _check(lib().ms_plan(n, elem_bytes, _cfg(leaf_B, lds_levels_max, hbm_only, levels_per_pass, one_level_passes,
                                             placement),
                         ctypes.byref(info)))
    return {f: getattr(info, f) for f, _ in MSPlanInfo._fields_}


def device_status(stream=None) -> int:
    """Synchronize the stream, then read and clear the status flags of the
    calls made on it and of the allocation-free entry point (0 = clean).
    Raises MSError if the synchronization or the read fails."""
    flags = ctypes.c_uint32(0)
    rc = lib().ms_device_status(_stream(stream), ctypes.byref(flags))
    if rc not in (MS_OK, MS_ERR_CAPACITY):
        _check(rc)
    return int(flags.value)


def profile_enable(on: bool = True):
    _check(lib().ms_profile_enable(1 if on else 0))


def profile_read():
    """({class: total ms}, {class: launches}) for classes plan, leaf, merge_pass, patch."""
    ms = (ctypes.c_double * 4)()
    cnt = (ctypes.c_uint64 * 4)()
    _check(lib().ms_profile_read(ms, cnt))
    names = ["plan", "leaf", "merge_pass", "patch"]
    return {k: ms[i] for i, k in enumerate(names)}, {k: int(cnt[i]) for i, k in enumerate(names)}


def release():
    _check(lib().ms_release())
