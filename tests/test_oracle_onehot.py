"""Pins of the expanded one-hot pencil (Sec. II.E eq. oht_exp / eq. subs_exp,
App. A1): orthonormality and completeness of the one-hot states, the 4^N
Fock space, and the variational property of the expanded eigenproblem."""
import numpy as np
import pytest

import tnqe_synth as synth
from oracle import fock
from oracle.onehot import canonical_at, expanded_gep, onehot_index, onehot_pencil, onehot_state
from oracle.subspace import rotate_integrals, subspace


@pytest.mark.parametrize("k,i,p", [(1, 0, 1), (1, 1, 0), (1, 1, 2), (2, 2, 3)])
def test_onehot_states_orthonormal_and_complete(k, i, p):
    prob = synth.make_config(k)
    index, Hd, Sd, Hc, Sc, t = onehot_pencil(prob, i, p)
    n = len(index)
    assert n > 0
    np.testing.assert_allclose(Sd, np.eye(n), atol=1e-13)        # <varphi_m|varphi_n> = delta
    assert abs(t @ t - 1.0) < 1e-12                                 # sum |t_m|^2 = 1
    # phi_i = sum_m t_m varphi_m, so its column is Hd t (and Sd t = t)
    np.testing.assert_allclose(Hc[:, i], Hd @ t, atol=1e-11 * np.abs(Hd).max())
    np.testing.assert_allclose(Hd, Hd.T, atol=1e-12 * np.abs(Hd).max())
    # the one-hot entries conserve particle numbers; none is missing
    sites, qn = canonical_at(prob.mps[i].sites, prob.mps[i].bond_qn, p)
    T = np.einsum("akm,mlb->aklb", sites[p], sites[p + 1])
    mask = np.zeros(T.shape, dtype=bool)
    for (l, kp, kq, r) in index:
        mask[l, kp, kq, r] = True
    assert np.abs(T[~mask]).max(initial=0.0) < 1e-13
    np.testing.assert_allclose(T[mask], t, atol=1e-13)


def test_onehot_pencil_equals_fock_space():
    """Config 1 without truncation: every block against the 4^N Fock space
    (Jordan-Wigner operators and the determinant form of the rotations)."""
    prob = synth.make_config(1)
    i, p = 1, 1
    index, Hd, Sd, Hc, Sc, t = onehot_pencil(prob, i, p, chi_cap=10 ** 6)
    bi = prob.mps[i]
    hi, Li = rotate_integrals(prob.h, prob.L, bi.U)
    Hf = fock.hamiltonian_fock(hi, np.einsum("kpq,krs->pqrs", Li, Li), prob.e_core)
    sites, qn = canonical_at(bi.sites, bi.bond_qn, p)
    V = np.array([fock.mps_to_vector(onehot_state(sites, p, m)) for m in index])
    np.testing.assert_allclose(Hd, V @ (Hf @ V.T), atol=1e-12)
    for kk in range(prob.M):
        bk = prob.mps[kk]
        vk = fock.rotation_matrix_fock(bi.U.T @ bk.U) @ fock.mps_to_vector(bk.sites)
        np.testing.assert_allclose(Hc[:, kk], V @ (Hf @ vk), atol=1e-12)
        np.testing.assert_allclose(Sc[:, kk], V @ vk, atol=1e-13)


def test_expanded_eigenvalue_is_variational():
    """The expanded space contains every original state, so its lowest root
    is at most the pencil's (exact rotations); with one state it is the
    lowest eigenvalue of the two-site block (the DMRG two-site update)."""
    prob = synth.make_config(2)
    H, S, E, c, rep = subspace(prob, chi_cap=10 ** 6)
    for i, p in [(0, 2), (3, 4)]:
        index, Hd, Sd, Hc, Sc, t = onehot_pencil(prob, i, p, chi_cap=10 ** 6)
        Ex, tnew = expanded_gep(H, S, Hd, Sd, Hc, Sc, i)
        assert Ex <= E + 1e-10
        assert abs(tnew @ tnew - 1.0) < 1e-12
    one = synth.Problem(**{**prob.__dict__, "mps": [prob.mps[1]]})
    index, Hd, Sd, Hc, Sc, t = onehot_pencil(one, 0, 3)
    Ex, tnew = expanded_gep(np.array([[Hc[:, 0] @ t]]), np.eye(1), Hd, Sd, Hc, Sc, 0)
    assert abs(Ex - np.linalg.eigvalsh(Hd)[0]) < 1e-10
    assert Ex <= t @ Hd @ t + 1e-12


def test_onehot_index_counts():
    prob = synth.make_config(2)
    sites, qn = canonical_at(prob.mps[0].sites, prob.mps[0].bond_qn, 3)
    idx = onehot_index(qn, 3)
    dense = qn[3].shape[0] * 16 * qn[5].shape[0]
    assert 0 < len(idx) < dense
    assert idx == sorted(idx)
