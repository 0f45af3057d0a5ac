"""Write uniform32768_digest.json: SHA-256 digests of the CPU oracle's full output
for the n = 32768 uniform workload, one per 4096-row slab of M and of idx.

The n x n output (8 GiB of M and idx) is too large to keep as a fixture, and
the oracle takes minutes at this size, so the GPU tests compare the SHA-256 of
each row slab of their output with the digests stored here.  This script calls
only the oracle (Algorithm 4 as Section 3 describes it) and the seeded input
generator; nothing here comes from the HIP library.  A digest of W itself is
stored too, so that a change of the generator is reported as such.

    python tests/golden/make_uniform32768_digest.py
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

N = 32768
SLAB = 4096
OUT = os.path.join(HERE, "uniform32768_digest.json")


def slab_digests(A: np.ndarray, slab: int = SLAB):
    """SHA-256 (hex) of the raw little-endian bytes of each row slab."""
    return [hashlib.sha256(memoryview(np.ascontiguousarray(A[r0:r0 + slab])).cast("B")).hexdigest()
            for r0 in range(0, A.shape[0], slab)]


def main():
    t0 = time.time()
    W = workloads.config_uniform(N)
    w_digest = hashlib.sha256(memoryview(W).cast("B")).hexdigest()
    print("W generated (%.1f s), sha256 %s" % (time.time() - t0, w_digest), flush=True)
    t1 = time.time()
    M, idx = oracle.appd(W)
    print("oracle done (%.1f s)" % (time.time() - t1), flush=True)
    doc = {
        "source": "Oracle (oracle_appd_alg4: Algorithm 4 of Section 3, Prim's tree, descending "
                  "removals, traversal of both halves) on the seeded n = 32768 uniform workload "
                  "(workloads.config_uniform, seed %d); written by %s." %
                  (workloads.SEEDS["uniform"], os.path.basename(__file__)),
        "n": N,
        "slab_rows": SLAB,
        "W_sha256": w_digest,
        "M_sha256": slab_digests(M),
        "idx_sha256": slab_digests(idx),
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
        f.write("\n")
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
