"""Order-sensitive fingerprints of a permutation, computed the same way on the
CPU (numpy) and on the GPU (torch int64 ops), in chunks.

H(perm) = sum_t ((perm[t] * w(t)) mod p) mod p with p = 2^31 - 1 and
w(t) = (t * A + 11) mod p, for two multipliers A.  Any single transposition
changes both sums unless an unlikely coincidence hits both.
"""
P31 = 2**31 - 1
MULTS = (48271, 69621)
CHUNK = 1 << 24


def fingerprint_np(perm):
    import numpy as np

    n = perm.size
    out = []
    for A in MULTS:
        h = 0
        for s in range(0, n, CHUNK):
            t = np.arange(s, min(n, s + CHUNK), dtype=np.int64)
            w = (t * A + 11) % P31
            v = perm[s:s + CHUNK].astype(np.int64) % P31
            h = (h + int(((v * w) % P31).sum() % P31)) % P31
        out.append(h)
    return tuple(out)


def fingerprint_torch(perm):
    import torch

    n = perm.numel()
    out = []
    for A in MULTS:
        h = 0
        for s in range(0, n, CHUNK):
            e = min(n, s + CHUNK)
            t = torch.arange(s, e, dtype=torch.int64, device=perm.device)
            w = (t * A + 11) % P31
            v = (perm[s:e].to(torch.int64) & 0xFFFFFFFF) % P31
            h = (h + int(((v * w) % P31).sum().item() % P31)) % P31
        out.append(h)
    return tuple(out)
