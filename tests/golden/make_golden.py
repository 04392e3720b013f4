"""Write tests/golden/configs.json from the CPU oracle alone.

For each plain-permutation configuration it stores the random-bit count,
two order-sensitive fingerprints of the whole permutation (tests/hashing.py)
and a few hundred sampled (position, value) pairs.  Run from the repository
root:  python tests/golden/make_golden.py   (the 2^30 case takes minutes and
about 9 GiB of host memory).
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

from oracle import oracle as O  # noqa: E402
from paper_1508_03167_amd.inputs import sample_positions  # noqa: E402
import hashing  # noqa: E402

CONFIGS = [
    ("perm_n2^20_seed1", 1 << 20, 1),
    ("perm_n2^27_seed11", 1 << 27, 11),
    ("perm_n2^30_seed7", 1 << 30, 7),
    # the largest size the library accepts, 2^32 - 2^16 (about 33 GiB of host memory, several minutes)
    ("perm_n2^32-2^16_seed5", (1 << 32) - (1 << 16), 5),
]


def main(which=None):
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "configs.json")
    data = json.load(open(path)) if os.path.exists(path) else {}
    threads = max(1, min(16, os.cpu_count() or 1))
    for name, n, seed in CONFIGS:
        if which and name not in which:
            continue
        t = time.time()
        pi, bits = O.permutation(n, 4096, seed, threads=threads)
        pos = sample_positions(n, 512, seed + 1000)
        data[name] = {
            "n": n, "seed": seed, "cutoff": 4096, "bits": bits,
            "fingerprint": list(hashing.fingerprint_np(pi)),
            "samples": [[int(p), int(pi[p])] for p in pos],
        }
        print(name, "bits", bits, "oracle seconds", round(time.time() - t, 1), flush=True)
        del pi
        json.dump(data, open(path, "w"), indent=1)


if __name__ == "__main__":
    main(sys.argv[1:] or None)
