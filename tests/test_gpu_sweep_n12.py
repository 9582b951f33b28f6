"""The expanded one-hot pencil (Sec. II.E eq. subs_exp, App. A1) and one
generalized-sweep step (Alg. A.1 with one single-site mitigation round,
App. A4) at the N = 12, chi = 64, M = 8 workload, against stored oracle
values (tests/golden/make_golden_sweep.py: state 0 at sites 1-2 with the
Givens search, state 5 at sites 9-10 with the FSWAP test; 400 one-hot states
and 407 columns each, so the dense eigensolves take the chip-wide Jacobi).
The oracle needs about 20 minutes per step here, so its results are stored:
the one-hot block's diagonal and 4000 sampled entries, the state columns, and
the step's outcome."""
import os

import numpy as np
import pytest

import paper_2404_10223_amd as T
import tnqe_synth as synth

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")
TOL = 1e-10


@pytest.fixture(scope="module")
def ctx():
    c = T.Context(0)
    yield c
    c.close()


CASES = ["oracle_sweep_config3", "oracle_sweep_config3_b"]


def _gold(name):
    g = np.load(os.path.join(GOLD, name + ".npz"))
    return {k: g[k] for k in g.files}


@pytest.mark.parametrize("name", CASES)
def test_onehot_pencil_n12(ctx, name):
    gold = _gold(name)
    prob = synth.make_config(3)
    i, p = int(gold["i"]), int(gold["p"])
    print(f"N = 12 one-hot pencil, state {i}, sites ({p}, {p + 1})", flush=True)
    idx, Hd, Sd, Hc, Sc, rep = ctx.onehot_pencil(prob, i, p, chi=prob.chi)
    np.testing.assert_array_equal(idx, gold["index"])
    h = np.abs(gold["Hd_diag"]).max()
    assert np.abs(np.diag(Hd) - gold["Hd_diag"]).max() <= TOL * h
    assert np.abs(Hd[gold["Hd_rows"], gold["Hd_cols"]] - gold["Hd_vals"]).max() <= TOL * h
    assert np.abs(Hc - gold["Hc"]).max() <= TOL * h
    assert np.abs(Sc - gold["Sc"]).max() <= TOL
    np.testing.assert_allclose(Sd, np.eye(len(idx)), atol=1e-12)
    np.testing.assert_allclose(Hd, Hd.T, atol=1e-12 * h)


@pytest.mark.parametrize("name", CASES)
def test_sweep_step_n12(ctx, name):
    gold = _gold(name)
    prob = synth.make_config(3)
    H0 = np.load(os.path.join(GOLD, "oracle_config3.npz"))
    i, p, nreps, rotation = int(gold["i"]), int(gold["p"]), int(gold["nreps"]), str(gold["rotation"])
    print(f"N = 12 sweep step, state {i}, sites ({p}, {p + 1}), {rotation}, nreps {nreps}", flush=True)
    res, (sites, qn, U), t, rep = ctx.sweep_step(prob, H0["H"], H0["S"], i, p, rotation=rotation, nreps=nreps,
                                                 chi=prob.chi)
    print(f"E1 {res['E1']:.12f} ({float(gold['E1']):.12f}) E_new {res['E_new']:.12f} "
          f"columns {res['n_columns']} kept {res['n_kept']}", flush=True)
    assert res["n_onehot"] == gold["n_onehot"] and res["n_columns"] == gold["n_columns"]
    assert res["n_kept"] == gold["n_kept"] and res["n_dropped_S"] == gold["n_dropped_S"]
    assert abs(res["E_old"] - gold["E_old"]) <= 1e-12 * abs(gold["E_old"])
    assert abs(res["E1"] - gold["E1"]) <= TOL * abs(gold["E1"])
    assert abs(res["E_new"] - gold["E_new"]) <= TOL * abs(gold["E_new"])
    assert res["accepted"] == gold["accepted"]
    np.testing.assert_allclose(t, gold["t_new"], atol=1e-8)
    assert abs(res["xi_none"] - gold["xi_none"]) <= 1e-12
    assert res["theta"] == gold["theta"] and abs(res["xi"] - gold["xi"]) <= 1e-12
    assert res["new_bond"] == gold["new_bond"] and abs(res["discarded"] - gold["discarded"]) <= 1e-12
    assert res["mit_columns"] == gold["mit_columns"] and res["mit_kept"] == gold["mit_kept"]
    qo = np.split(gold["qn"], np.cumsum(gold["qn_len"])[:-1])
    for b in range(prob.N + 1):
        np.testing.assert_array_equal(qn[b], qo[b])
    two = np.einsum("akm,mlb->aklb", sites[p], sites[p + 1])
    np.testing.assert_allclose(two, gold["two_site"], atol=1e-8)
    A = sites[p].reshape(-1, sites[p].shape[2])
    np.testing.assert_allclose(A.T @ A, np.eye(A.shape[1]), atol=1e-12)
    np.testing.assert_allclose(U, gold["U"], atol=1e-10)
