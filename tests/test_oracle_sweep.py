"""Pins of the generalized-sweep step oracle (Alg. A.1; App. A1-A3) against
what the mathematics fixes: full-span expansions reduce to exact
diagonalisation, the updated state reproduces the expanded root, merging a
rotation into the orbital basis leaves the state unchanged, the blocked
truncation error equals the dense SVD's, and the discard rule equals an
explicit least-squares projection."""
import copy

import numpy as np
import pytest

import tnqe_synth as synth
from oracle import fock, gates, sweep
from oracle.subspace import subspace as oracle_subspace


def _with_state(prob, i, sites, qn, U):
    p2 = copy.copy(prob)
    p2.mps = list(prob.mps)
    p2.mps[i] = synth.MPS([s.copy() for s in sites], [q.copy() for q in qn], U.copy())
    return p2


def _fci_ground(prob):
    """Lowest eigenvalue of the 4^N Fock Hamiltonian in the particle sector."""
    Hf = fock.hamiltonian_fock(prob.h, prob.g(), prob.e_core).toarray()
    na_op, nb_op = fock.number_ops(prob.N)
    sel = np.isclose(na_op.diagonal(), prob.n_alpha) & np.isclose(nb_op.diagonal(), prob.n_beta)
    return float(np.linalg.eigvalsh(Hf[np.ix_(sel, sel)])[0])


def test_discard_rule_against_least_squares():
    r = np.random.default_rng(5)
    V = r.normal(size=(9, 6))
    V[:, 3] = V[:, 0] - 2.0 * V[:, 1] + 1e-3 * r.normal(size=9)   # nearly dependent
    V[:, 5] = 0.5 * V[:, 2] + V[:, 4]                              # exactly dependent
    V /= np.linalg.norm(V, axis=0)[None, :]
    S = V.T @ V
    # (tolerances above the resolution of the overlap form, ~eps cond(S_kept))
    for tol in (1e-3, 1e-6):
        keep = sweep.discard_dependent(S, tol)
        # brute force: the squared residual of each column after a least-squares
        # fit by the kept earlier columns
        want, kept = [], []
        for c in range(6):
            res = V[:, c] - V[:, kept] @ np.linalg.lstsq(V[:, kept], V[:, c], rcond=None)[0] if kept else V[:, c]
            ok = res @ res >= tol
            want.append(ok)
            if ok:
                kept.append(c)
        assert list(keep) == want, (tol, keep, want)
    assert list(sweep.discard_dependent(S, 1e-3)) == [True, True, True, False, True, False]


@pytest.mark.parametrize("N,p", [(2, 0), (3, 0), (3, 1), (4, 1)])
def test_full_span_expansion_is_exact_diagonalisation(N, p):
    """M = 1 and a two-site block whose one-hot states span the whole particle
    sector (the bonds around it are full): the expanded root is the exact
    ground energy (App. A1)."""
    from oracle.fock import sector_dim
    na, nb = (N + 1) // 2, N // 2
    prob = synth.make_problem(N, na, nb, 16, 1, N, (77, N, p))
    H, S, E, c, rep = oracle_subspace(prob)
    r = sweep.sweep_step(prob, H, S, 0, p)
    assert r["n_onehot"] == sector_dim(N, na, nb)
    assert abs(r["E1"] - _fci_ground(prob)) < 1e-10 * (1 + abs(r["E1"]))
    assert r["E1"] <= r["E_old"] + 1e-12


@pytest.mark.parametrize("k,i,p", [(1, 0, 1), (1, 1, 0), (1, 1, 2), (2, 2, 3)])
def test_updated_state_reproduces_expanded_root(k, i, p):
    """eq. param_upd: the subspace with state i replaced by its updated
    (untruncated) state has the expanded root as its lowest root -- the
    expanded optimum lies in the span of the other states and the updated
    one.  Lossless rotations (chi_cap far above every bond) on both sides."""
    prob = synth.make_config(k)
    big = 4 ** prob.N
    H, S, E, c, _ = oracle_subspace(prob, chi_cap=big)
    r = sweep.sweep_step(prob, H, S, i, p, chi_cap=big, tau_w=0.0)
    assert abs(np.linalg.norm(r["t_new"]) - 1.0) < 1e-12
    assert r["t_new"] @ r["t_old"] >= 0.0
    assert r["E1"] <= r["E_old"] + 1e-12
    p2 = _with_state(prob, i, r["sites"], r["qn"], r["U"])
    H2, S2, E2, _, _ = oracle_subspace(p2, chi_cap=big)
    assert abs(E2 - r["E1"]) < 1e-9 * (1 + abs(E2)), (E2, r["E1"])


@pytest.mark.parametrize("rotation,theta", [("givens", 0.37), ("givens", -1.2), ("fswap", np.pi / 2)])
def test_rotation_merge_keeps_the_state(rotation, theta):
    """A rotation applied to the two-site tensor and merged into U_i
    (U_i <- U_i R_p(theta)^T, FSWAP: columns exchanged) leaves the state
    G(U_i)|Phi> unchanged before truncation (C3: G(A)G(B) = G(AB))."""
    prob = synth.make_config(1)
    H, S, E, c, _ = oracle_subspace(prob)
    i, p = 1, 1
    r = sweep.sweep_step(prob, H, S, i, p)
    big = 4 ** prob.N
    s0, q0, U0, _, _ = sweep.finish(r["T4"], r["canon_sites"], r["canon_qn"], prob.mps[i].U, p, "none", 0.0,
                                    big, 0.0)
    s1, q1, U1, _, _ = sweep.finish(r["T4"], r["canon_sites"], r["canon_qn"], prob.mps[i].U, p, rotation, theta,
                                    big, 0.0)
    v0 = fock.rotation_matrix_fock(U0) @ fock.mps_to_vector(s0)
    v1 = fock.rotation_matrix_fock(U1) @ fock.mps_to_vector(s1)
    np.testing.assert_allclose(v1, v0, atol=1e-12)
    assert np.abs(U1.T @ U1 - np.eye(prob.N)).max() < 1e-14


def _step_tensor(k=2, i=1, p=3):
    prob = synth.make_config(k)
    H, S, E, c, _ = oracle_subspace(prob)
    return prob, sweep.sweep_step(prob, H, S, i, p)


def test_blocked_xi_equals_dense_svd():
    prob, r = _step_tensor()
    T4, qn, p = r["T4"], r["canon_qn"], 3
    dl, dr = T4.shape[0], T4.shape[3]
    for G in (np.eye(16), gates.f4(), gates.g4(0.8)):
        T = sweep.apply_gate(T4, G)
        s = np.linalg.svd(T.reshape(dl * 4, 4 * dr), compute_uv=False)
        for chi in (1, 5, prob.chi):
            assert abs(sweep.xi(T, qn[p], qn[p + 2], chi) - (1.0 - np.sum(s[:chi] ** 2))) < 1e-13


def test_theta_opt_minimises_xi_and_period():
    prob, r = _step_tensor()
    T4, qn, p = r["T4"], r["canon_qn"], 3
    th, xv, x0 = sweep.optimise_theta(T4, qn[p], qn[p + 2], prob.chi)
    f = lambda t: sweep.xi(sweep.apply_gate(T4, gates.g4(t)), qn[p], qn[p + 2], prob.chi)
    scan = [f(t) for t in np.linspace(-np.pi / 2, np.pi / 2, 721)]
    assert xv <= min(scan) + 1e-12 and xv <= x0
    assert abs(f(th) - xv) < 1e-15
    for t in (0.3, -1.0):
        assert abs(f(t + np.pi) - f(t)) < 1e-13


def test_truncation_is_best_low_rank():
    """The split at chi equals the dense Eckart-Young projection of the whole
    two-site matrix (the blocks carry a gap at the cut here)."""
    prob, r = _step_tensor()
    T4, qn, p = r["T4"], r["canon_qn"], 3
    dl, dr = T4.shape[0], T4.shape[3]
    for chi in (3, 8):
        Ap, Aq, newq, st = sweep.truncate_two_site(T4, qn[p], qn[p + 2], chi, 1e-13)
        Tm = T4.reshape(dl * 4, 4 * dr)
        u, s, vt = np.linalg.svd(Tm)
        assert st["gap"] is None or st["gap"] > 1e-6
        best = (u[:, :st["kept"]] * s[:st["kept"]]) @ vt[:st["kept"]]
        got = Ap.reshape(dl * 4, -1) @ Aq.reshape(Aq.shape[0], -1)
        np.testing.assert_allclose(got, best, atol=1e-13)
        A = Ap.reshape(dl * 4, -1)
        np.testing.assert_allclose(A.T @ A, np.eye(A.shape[1]), atol=1e-13)


def test_fswap_decision_and_acceptance():
    prob, r = _step_tensor()
    H, S, E, c, _ = oracle_subspace(prob)
    rf = sweep.sweep_step(prob, H, S, 1, 3, rotation="fswap")
    T4, qn, p = rf["T4"], rf["canon_qn"], 3
    xs = sweep.xi(sweep.apply_gate(T4, gates.f4()), qn[p], qn[p + 2], prob.chi)
    assert (rf["theta"] != 0.0) == (xs < rf["xi_none"] - 1e-12)
    assert rf["xi"] == (xs if rf["theta"] != 0.0 else rf["xi_none"])
    assert rf["accepted"] == (rf["E1"] < rf["E_old"])


# ------------------------------------------------ single-site mitigation (App. A4)
def test_onehot_gate_matrix_gives_the_rotated_basis():
    """The rotation in the one-hot basis (App. A4) maps the expanded pencil to
    the one computed directly in the merged orbital basis: G^T H^[ii] G equals
    the diagonal block of the state with U_i R_p(theta)^T, and G is
    orthogonal."""
    from oracle.onehot import onehot_pencil
    prob = synth.make_config(2)
    H, S, E, c, _ = oracle_subspace(prob)
    i, p = 3, 2
    r = sweep.sweep_step(prob, H, S, i, p, rotation="givens")
    assert r["theta"] != 0.0
    Hd, Sd, Hc, Sc = r["onehot"]
    G = sweep.onehot_gate_matrix(r["index"], gates.g4(r["theta"]))
    np.testing.assert_allclose(G.T @ G, np.eye(len(G)), atol=1e-13)
    # the same environments (canonical form of the same state), integrals in
    # the merged basis
    p2 = _with_state(prob, i, prob.mps[i].sites, prob.mps[i].bond_qn, r["U"])
    idx2, Hd2, Sd2, _, _, _ = onehot_pencil(p2, i, p)
    assert idx2 == r["index"]
    np.testing.assert_allclose(G.T @ Hd @ G, Hd2, atol=1e-11)
    np.testing.assert_allclose(Sd2, np.eye(len(G)), atol=1e-13)


@pytest.mark.parametrize("nreps", [1, 2])
def test_mitigated_state_reproduces_last_root(nreps):
    """Lossless rotations: the state after the single-site expansions, put
    back into an independent subspace evaluation, has the last root as its
    lowest root (its optimum lies in the span of the other states and the
    updated one)."""
    prob = synth.make_config(1)
    big = 4 ** prob.N
    H, S, E, c, _ = oracle_subspace(prob, chi_cap=big)
    r = sweep.sweep_step(prob, H, S, 1, 1, rotation="givens", chi_cap=big, tau_w=0.0, nreps=nreps)
    assert r["mitigation"] is not None
    p2 = _with_state(prob, 1, r["sites"], r["qn"], r["U"])
    H2, S2, E2, _, _ = oracle_subspace(p2, chi_cap=big)
    assert abs(E2 - r["E_new"]) < 1e-9 * (1 + abs(E2)), (E2, r["E_new"])
    assert r["E_new"] >= r["E1"] - 1e-10
    A = r["sites"][1].reshape(-1, r["sites"][1].shape[2])
    np.testing.assert_allclose(A.T @ A, np.eye(A.shape[1]), atol=1e-12)


def test_mitigation_improves_on_the_truncated_state():
    """With a cut at the bond, the first single-site expansion contains the
    truncated state itself, so the mitigated root is not above the truncated
    state's energy in the same expanded pencil, nor below the two-site root."""
    prob = synth.make_config(2)
    H, S, E, c, _ = oracle_subspace(prob)
    i, p = 3, 2
    r = sweep.sweep_step(prob, H, S, i, p, rotation="givens", nreps=1)
    Hd, Sd, Hc, Sc = r["onehot"]
    G = sweep.onehot_gate_matrix(r["index"], gates.g4(r["theta"]))
    s_t, _, _, _, st = sweep.finish(r["T4"], r["canon_sites"], r["canon_qn"], prob.mps[i].U, p, "givens",
                                    r["theta"], prob.chi, 1e-13)
    assert st["discarded"] > 1e-8
    T2 = np.einsum("akm,mlb->aklb", s_t[p], s_t[p + 1])
    x = np.array([T2[e] for e in r["index"]])
    Hr, Sr = H.copy(), S.copy()
    Hr[i, i], Sr[i, i] = x @ (G.T @ Hd @ G) @ x, x @ (G.T @ Sd @ G) @ x
    for k in range(prob.M):
        if k != i:
            Hr[i, k] = Hr[k, i] = x @ (G.T @ Hc[:, k])
            Sr[i, k] = Sr[k, i] = x @ (G.T @ Sc[:, k])
    from oracle.gep import solve_projection
    E_trunc = solve_projection(Hr, Sr)["E"]
    print(r["E1"], r["E_new"], E_trunc)
    assert r["E_new"] <= E_trunc + 1e-12
    assert r["E_new"] >= r["E1"] - 1e-12
