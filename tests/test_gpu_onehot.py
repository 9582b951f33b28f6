"""Expanded one-hot pencil (Sec. II.E eq. subs_exp, App. A1) on the MI355X
against the oracle's sector-FCI values, element by element."""
import numpy as np
import pytest

import paper_2404_10223_amd as T
import tnqe_synth as synth
from oracle.onehot import expanded_gep, onehot_pencil
from oracle.subspace import subspace

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module")
def ctx():
    c = T.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("k,i,p", [(1, 1, 1), (1, 0, 2), (2, 2, 3), (2, 0, 0), (2, 3, 5)])
def test_onehot_blocks_match_oracle(ctx, k, i, p):
    prob = synth.make_config(k)
    idx, Hd, Sd, Hc, Sc, rep = ctx.onehot_pencil(prob, i, p, chi=prob.chi)
    oidx, oHd, oSd, oHc, oSc, t = onehot_pencil(prob, i, p)
    print(f"config {k}, state {i}, sites ({p},{p + 1}): {len(idx)} one-hot states, "
          f"{rep['env_kernel_ms']:.2f} ms, {rep['env_flops'] / 1e9:.2f} GFLOP", flush=True)
    np.testing.assert_array_equal(idx, np.array(oidx, dtype=np.int32).reshape(-1, 4))
    h = np.abs(oHd).max()
    assert np.abs(Hd - oHd).max() <= TOL * h
    assert np.abs(Hc - oHc).max() <= TOL * h
    assert np.abs(Sd - oSd).max() <= TOL
    assert np.abs(Sc - oSc).max() <= TOL
    np.testing.assert_allclose(Sd, np.eye(len(idx)), atol=1e-12)
    np.testing.assert_allclose(Hd, Hd.T, atol=1e-12 * h)
    # the expanded eigenproblem from the device blocks and the device pencil
    H, S, E, c, _ = ctx.subspace(prob, chi=prob.chi)
    Ex, tn = expanded_gep(H, S, Hd, Sd, Hc, Sc, i)
    Eo, tno = expanded_gep(H, S, oHd, oSd, oHc, oSc, i)
    assert abs(Ex - Eo) <= 1e-9 * max(1.0, abs(Eo))


def test_onehot_single_state_is_two_site_update(ctx):
    """M = 1: the expanded pencil is the two-site effective Hamiltonian, whose
    lowest eigenvalue is at most the state's energy."""
    base = synth.make_config(2)
    one = synth.Problem(**{**base.__dict__, "mps": [base.mps[1]]})
    idx, Hd, Sd, Hc, Sc, rep = ctx.onehot_pencil(one, 0, 2, chi=one.chi)
    t = Sc[:, 0]
    assert abs(t @ t - 1.0) < 1e-12
    e = t @ Hd @ t
    H, S, E, c, _ = ctx.subspace(one, chi=one.chi)
    assert abs(e - H[0, 0]) < 1e-10 * abs(H[0, 0])
    assert np.linalg.eigvalsh(Hd)[0] <= e + 1e-12
