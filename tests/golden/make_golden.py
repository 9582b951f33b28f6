"""Writes the stored oracle values used by the GPU parity tests.

Calls only the seeded generator (tnqe_synth) and the FP64 oracle (oracle/);
nothing here touches the GPU library.  Usage:  python tests/golden/make_golden.py [names...]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import tnqe_synth as synth                     # noqa: E402
from oracle.subspace import pair_element, subspace   # noqa: E402

C5_PAIRS = [(0, 0), (0, 1), (3, 11), (14, 15)]


def digests():
    out = {f"config{k}": synth.problem_digest(synth.make_config(k)) for k in (1, 2, 3, 5)}
    out["batch"] = [synth.problem_digest(p) for p in synth.make_batch()[:8]]
    for rot in VARIANTS.values():
        for k in (2, 3):
            p = synth.make_config(k, rot)
            out[p.name] = synth.problem_digest(p)
    with open(os.path.join(HERE, "digests.json"), "w") as f:
        json.dump(out, f, indent=1)


VARIANTS = {"f": "perm", "lc": "identity"}   # fermionic-swap networks (TNQE-F), no rotations (LC-MPS)


def full(k, rotations="expm"):
    prob = synth.make_config(k, rotations)
    t = time.time()
    H, S, E, c, rep = subspace(prob)
    np.savez(os.path.join(HERE, f"oracle_{prob.name}.npz"), H=H, S=S, E=E, c=c,
             min_rel_gap=rep["min_rel_gap"] or 1.0, max_discarded=rep["max_discarded_weight_sum"],
             seconds=time.time() - t)
    print(k, E, rep, time.time() - t, flush=True)


def c5_pairs():
    prob = synth.make_config(5)
    cache = {}
    out = {}
    for (i, j) in C5_PAIRS:
        t = time.time()
        h, s, st = pair_element(prob, i, j, mpo_cache=cache)
        gaps = [x["gap"] for x in st if x["gap"] is not None]
        out[f"{i}_{j}"] = np.array([h, s, min(gaps) if gaps else 1.0, time.time() - t])
        print(i, j, h, s, time.time() - t, flush=True)
    np.savez(os.path.join(HERE, "oracle_config5_pairs.npz"), **out)


BATCH_SAMPLE = [3, 7, 10, 11, 0]


def batch():
    probs = synth.make_batch()
    res = {}
    for s_ in BATCH_SAMPLE:
        prob = probs[s_]
        t = time.time()
        H, S, E, c, rep = subspace(prob, h_method="mpo")
        res[f"H{s_}"], res[f"S{s_}"], res[f"E{s_}"] = H, S, E
        print("batch", s_, prob.N, prob.chi, prob.M, E, time.time() - t, flush=True)
        np.savez(os.path.join(HERE, "oracle_batch.npz"), **res)


if __name__ == "__main__":
    todo = sys.argv[1:] or ["digests", "1", "2", "3", "c5", "batch", "f2", "f3", "lc2", "lc3"]
    for name in todo:
        if name == "digests":
            digests()
        elif name == "c5":
            c5_pairs()
        elif name == "batch":
            batch()
        elif name.rstrip("0123456789") in VARIANTS:
            v = name.rstrip("0123456789")
            full(int(name[len(v):]), VARIANTS[v])
        else:
            full(int(name))
