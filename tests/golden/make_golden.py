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
    """Sampled pairs of the N = 24 workload.  Each H is computed twice, by the
    block-sparse MPO sweep and by the plain dense sweep (no sector or channel
    grouping), and the two must agree: no sector FCI is possible at N = 24."""
    from oracle.mpo import expectation_plain
    prob = synth.make_config(5)
    cache = {}
    out = {}
    for (i, j) in C5_PAIRS:
        t = time.time()
        h, s, st, ket = pair_element(prob, i, j, mpo_cache=cache, return_ket=True)
        hp, sp = expectation_plain(cache[i], prob.mps[i].sites, ket)
        assert abs(hp - h) <= 1e-12 * max(abs(h), 1e-300) + 1e-14 and abs(sp - s) <= 1e-12 * abs(s) + 1e-16, \
            (h, hp, s, sp)
        gaps = [x["gap"] for x in st if x["gap"] is not None]
        out[f"{i}_{j}"] = np.array([h, s, min(gaps) if gaps else 1.0, time.time() - t, hp, sp])
        print(i, j, h, hp, s, sp, time.time() - t, flush=True)
    np.savez(os.path.join(HERE, "oracle_config5_pairs.npz"), **out)


# sampled subspaces of the batched workload: every chi in {16, 32, 64, 128},
# N from 8 to 15; H by sector FCI wherever N <= 13 (independent of any MPO),
# by the oracle's MPO sweep (cross-checked by the plain dense sweep) above
BATCH_SAMPLE = [3, 7, 11, 19, 16, 10, 9, 23, 13, 49, 0]
FCI_MAX_N = 13


def batch():
    probs = synth.make_batch()
    res = {}
    for s_ in BATCH_SAMPLE:
        prob = probs[s_]
        t = time.time()
        method = "fci" if prob.N <= FCI_MAX_N else "mpo"
        H, S, E, c, rep = subspace(prob, h_method=method)
        if method == "mpo":
            # the block-sparse sweep against the plain dense sweep, pair by pair
            Hp = plain_pencil(prob)
            assert np.abs(Hp - H).max() <= 1e-11 * np.abs(H).max(), np.abs(Hp - H).max()
        res[f"H{s_}"], res[f"S{s_}"], res[f"E{s_}"] = H, S, E
        res[f"rep{s_}"] = np.array([rep["cond_S"], rep["lam_min"], rep["kappa1"], rep["n_dropped"],
                                    rep["min_rel_gap"] or 1.0, rep["max_discarded_weight_sum"]])
        res[f"method{s_}"] = np.array(method)
        print("batch", s_, prob.N, prob.chi, prob.M, method, E, time.time() - t, flush=True)
        np.savez(os.path.join(HERE, "oracle_batch.npz"), **res)


def plain_pencil(prob):
    """H by the plain dense MPO sweep for every pair (the same kets)."""
    from oracle.mpo import build_mpo, expectation_plain
    from oracle.subspace import rotate_integrals, rotate_ket
    H = np.zeros((prob.M, prob.M))
    for i in range(prob.M):
        bi = prob.mps[i]
        hi, Li = rotate_integrals(prob.h, prob.L, bi.U)
        W = build_mpo(hi, np.einsum("kpq,krs->pqrs", Li, Li))
        for j in range(i, prob.M):
            if i == j:
                ket = bi.sites
            else:
                ket, _, _ = rotate_ket(prob.mps[j].sites, prob.mps[j].bond_qn, bi.U.T @ prob.mps[j].U, prob.chi)
            H[i, j] = H[j, i] = expectation_plain(W, bi.sites, ket)[0]   # e_core = 0 in the batch
    return H


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
