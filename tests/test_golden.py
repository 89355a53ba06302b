"""The stored digests of full-size oracle results (tests/golden/) are the
oracle's: the mid workload's are recomputed here from the oracle and the
seeded generator; for the precision workload (minutes of oracle time) the
input digest is checked, so a change of the generator is caught on the CPU."""
import hashlib
import json
import os

import numpy as np

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fullsize_subclusters.json")


def _digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def _gold(name):
    with open(GOLDEN) as f:
        return json.load(f)[name]


def test_mid_digests_are_the_oracles(oracle):
    g = _gold("mid")
    job = synth.mid()
    assert (g["n"], g["d"], g["N"]) == (job.X.shape[0], job.X.shape[1], job.N)
    assert _digest(job.X) == g["x"]
    S, _, _ = oracle.scale(job.X)
    assert _digest(S) == g["s"]
    perm, offs, lms = oracle.subcluster(S, job.N)
    assert _digest(perm.astype("<i8")) == g["perm"]
    assert _digest(offs.astype("<i8")) == g["offsets"]
    assert _digest(lms.astype("<f4")) == g["landmarks"]


def test_precision_input_digest():
    g = _gold("precision")
    job = synth.precision()
    assert (g["n"], g["d"], g["N"]) == (job.X.shape[0], job.X.shape[1], job.N)
    assert _digest(job.X) == g["x"]
