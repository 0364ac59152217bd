"""Writes nonsquare_maxabs_digests.json: the CPU oracle's per-mask maxima of
the two non-square workloads (20x16 and 16x20 uniform random functions), as
SHA-256 digests of consecutive blocks of masks, with the NL.

The full oracle passes take minutes on a few host cores, so the GPU tests
compare the library's maxabs array block by block against these digests
(bit-exact) and recompute the oracle only for a block that differs, to name
the first differing mask.  Only the oracle and the seeded input generators
are called here.

    python tests/golden/make_nonsquare_digests.py [nthreads]
"""
import hashlib
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1912_03732_amd import inputs  # noqa: E402

OUT = os.path.join(HERE, "nonsquare_maxabs_digests.json")
BLOCK = 4096  # masks per digest


def block_digests(maxabs: np.ndarray, block: int = BLOCK):
    a = np.ascontiguousarray(maxabs.astype("<i4"))
    return [hashlib.sha256(a[i:i + block].tobytes()).hexdigest()[:32] for i in range(0, a.size, block)]


def main():
    nthreads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    w = inputs.workload_nonsquare()
    rec = {"source": "oracle.walsh_nl over every mask of the seeded non-square workloads "
                     "(inputs.workload_nonsquare, seed %d)" % (inputs.SEED_BASE + 3),
           "block_masks": BLOCK, "boxes": {}}
    for key, n, m in (("s20x16", 20, 16), ("s16x20", 16, 20)):
        S = w[key]
        nl, mx = oracle.walsh_nl(S, n, m, nthreads=nthreads)
        rec["boxes"][key] = {"n": n, "m": m, "table_sha256": inputs.sha256(S), "nl": nl,
                             "maxabs_max": int(mx[1:].max()), "maxabs_min": int(mx[1:].min()),
                             "block_sha256_32": block_digests(mx)}
        print(key, "nl", nl, flush=True)
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
