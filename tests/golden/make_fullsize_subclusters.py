"""Write fullsize_subclusters.json: digests of the oracle's scaling and
equal sized subclustering (Sec. II, Algorithm 1, landmark recomputed every
round) of the two large synthetic workloads, so that GPU tests can compare
the library's full-size results with the oracle's bit for bit without
re-running the oracle's 128 rounds (minutes at 2^22 x 128).

Calls only the oracle (and the seeded input generators).  Every digest is
SHA-256 of the little-endian bytes of an array:
  x        the float32 input X (detects a different input generation);
  s        the oracle's float32 scaled points S;
  perm     the oracle's int64 permutation;
  offsets  the oracle's int64 offsets;
  landmarks the oracle's float32 landmarks (T x d).

Run:  python tests/golden/make_fullsize_subclusters.py
"""
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
import synth  # noqa: E402


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def record(job) -> dict:
    t0 = time.time()
    S, _, _ = oracle.scale(job.X)
    perm, offs, lms = oracle.subcluster(S, job.N)
    n, d = job.X.shape
    return {"n": n, "d": d, "N": job.N, "x": digest(job.X), "s": digest(S),
            "perm": digest(perm.astype("<i8")), "offsets": digest(offs.astype("<i8")),
            "landmarks": digest(lms.astype("<f4")), "oracle_seconds": round(time.time() - t0, 1)}


def main():
    out = {"what": "SHA-256 digests of the oracle's scaling and Algorithm 1 subclustering "
                   "(landmark recomputed each round, squared Euclidean keys) of the workloads below; "
                   "written by tests/golden/make_fullsize_subclusters.py",
           "mid": record(synth.mid()), "precision": record(synth.precision())}
    with open(os.path.join(HERE, "fullsize_subclusters.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
