"""Write the SHA-256 digests of the CPU oracle's PLE of the full-size
benchmark matrices, and of the reduced echelon form of the square one
(tests/golden/digests.json).  Calls only the oracle and the seeded input
generator; takes minutes of CPU per matrix (the reduced form of 65536^2 by the
oracle's back-substitution about half an hour).

    python tests/golden/make_digests.py            # all cases
    python tests/golden/make_digests.py 65536x65536_seed5
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1111_6549_amd import inputs  # noqa: E402

CASES = {
    "65536x65536_seed5": (65536, 65536, 5),
    "32768x131072_seed6": (32768, 131072, 6),
}
# reduced row echelon form (PLE, then the oracle's back-substitution)
RREF_CASES = {
    "65536x65536_seed5_rref": (65536, 65536, 5),
}
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "digests.json")


def ple_digest(r, P, Q, A):
    """Digest of a PLE result: rank (int64 LE), P, Q (int64 LE), L\\E words."""
    h = hashlib.sha256()
    h.update(np.int64(r).tobytes())
    h.update(np.ascontiguousarray(P, dtype="<i8").tobytes())
    h.update(np.ascontiguousarray(Q, dtype="<i8").tobytes())
    h.update(np.ascontiguousarray(A, dtype="<u8").tobytes())
    return h.hexdigest()


def rref_digest(r, Q, A):
    """Digest of a reduced echelon form: rank, Q (int64 LE), the m x ldw words
    (rows past the rank zero)."""
    h = hashlib.sha256()
    h.update(np.int64(r).tobytes())
    h.update(np.ascontiguousarray(Q, dtype="<i8").tobytes())
    h.update(np.ascontiguousarray(A, dtype="<u8").tobytes())
    return h.hexdigest()


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        if name in RREF_CASES:
            m, n, seed = RREF_CASES[name]
            A = inputs.bernoulli(m, n, seed)
            t0 = time.time()
            r, P, Q = oracle.ple(A, n)
            oracle.rref_from_ple(A, n, Q, r)
            dt = time.time() - t0
            data[name] = {"m": m, "n": n, "seed": seed, "density": 0.5, "rank": r, "sha256": rref_digest(r, Q, A),
                          "oracle_seconds": round(dt, 1), "oracle_threads": oracle.threads()}
            print(name, data[name], flush=True)
            with open(OUT, "w") as f:
                json.dump(data, f, indent=1, sort_keys=True)
                f.write("\n")
            continue
        m, n, seed = CASES[name]
        A = inputs.bernoulli(m, n, seed)
        t0 = time.time()
        r, P, Q = oracle.ple(A, n)
        dt = time.time() - t0
        data[name] = {"m": m, "n": n, "seed": seed, "density": 0.5, "rank": r, "sha256": ple_digest(r, P, Q, A),
                      "q_sha256": hashlib.sha256(np.ascontiguousarray(Q, dtype="<i8").tobytes()).hexdigest(),
                      "oracle_seconds": round(dt, 1), "oracle_threads": oracle.threads()}
        print(name, data[name], flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
            f.write("\n")


if __name__ == "__main__":
    main(sys.argv[1:] or list(CASES) + list(RREF_CASES))
