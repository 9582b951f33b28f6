"""Writes the stored oracle values of generalized-sweep steps at the
N = 12, chi = 64, M = 8 workload: state 0 at sites 1-2 with the Givens
search, and state 5 at sites 9-10 with the FSWAP test, each with one
single-site mitigation round (400 one-hot states, 407 columns).  The oracle
takes tens of minutes per step here (every one-hot state is a sector-FCI
vector), too long for a test, so its results are stored.

Calls only the seeded generator (tnqe_synth) and the FP64 oracle (oracle/),
with the pencil (H, S) of oracle_config3.npz; nothing here touches the GPU
library.  Usage:  python tests/golden/make_golden_sweep.py [case names...]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import tnqe_synth as synth                     # noqa: E402
from oracle import sweep                       # noqa: E402

# name: (state, left site, rotation, mitigation rounds)
CASES = {"oracle_sweep_config3": (0, 1, "givens", 1), "oracle_sweep_config3_b": (5, 9, "fswap", 1)}
N_SAMPLE = 4000   # sampled off-diagonal entries of the one-hot block H^[ii]


def case(name):
    I_STATE, P_SITE, ROTATION, NREPS = CASES[name]
    prob = synth.make_config(3)
    g = np.load(os.path.join(HERE, "oracle_config3.npz"))
    t0 = time.time()
    o = sweep.sweep_step(prob, g["H"], g["S"], I_STATE, P_SITE, rotation=ROTATION, nreps=NREPS)
    print(f"oracle sweep step: {time.time() - t0:.0f} s", flush=True)
    Hd, Sd, Hc, Sc = o["onehot"]
    n = Hd.shape[0]
    rng = np.random.default_rng(12)
    ra, rb = rng.integers(0, n, N_SAMPLE), rng.integers(0, n, N_SAMPLE)
    p = P_SITE
    two = np.einsum("akm,mlb->aklb", o["sites"][p], o["sites"][p + 1])
    st = o["trunc"]
    mit = o["mitigation"]
    np.savez_compressed(
        os.path.join(HERE, name + ".npz"),
        i=I_STATE, p=P_SITE, nreps=NREPS, rotation=ROTATION,
        E_old=o["E_old"], E1=o["E1"], E_new=o["E_new"], accepted=int(o["accepted"]),
        n_onehot=o["n_onehot"], n_columns=len(o["keep"]), n_kept=int(o["keep"].sum()),
        n_dropped_S=o["n_dropped_S"], t_new=o["t_new"], theta=o["theta"], xi_none=o["xi_none"], xi=o["xi"],
        new_bond=st["kept"], discarded=st["discarded"], gap=np.nan if st["gap"] is None else st["gap"],
        mit_columns=mit["n_columns"], mit_kept=mit["n_kept"], two_site=two, U=o["U"],
        qn=np.concatenate(o["qn"]),
        qn_len=np.array([q.shape[0] for q in o["qn"]]),
        index=np.array(o["index"], dtype=np.int32), Hd_diag=np.diag(Hd).copy(),
        Hd_rows=ra, Hd_cols=rb, Hd_vals=Hd[ra, rb], Sd_dev=np.abs(Sd - np.eye(n)).max(), Hc=Hc, Sc=Sc)
    print("written", name, flush=True)


if __name__ == "__main__":
    for name in sys.argv[1:] or list(CASES):
        case(name)
