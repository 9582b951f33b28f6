"""Pins of the whole pencil: brute force (P5), invariants (P8), eigensolver (P10)."""
import numpy as np
import pytest
import scipy.linalg

import tnqe_synth as synth
from oracle import fock, gates, givens, gep, mps as M
from oracle.subspace import pair_element, rotate_integrals, rotate_ket, subspace


@pytest.fixture(scope="module")
def c1():
    return synth.make_config(1)


@pytest.fixture(scope="module")
def c2():
    return synth.make_config(2)


def _exact_pencil_fock(prob):
    """C6 by brute force: 4^N Fock space, determinant-formula rotation."""
    Mn = prob.M
    H = np.zeros((Mn, Mn))
    S = np.zeros((Mn, Mn))
    for i in range(Mn):
        bi = prob.mps[i]
        hi, Li = rotate_integrals(prob.h, prob.L, bi.U)
        Hf = fock.hamiltonian_fock(hi, np.einsum("kpq,krs->pqrs", Li, Li), prob.e_core)
        vi = fock.mps_to_vector(bi.sites)
        for j in range(Mn):
            bj = prob.mps[j]
            vj = fock.rotation_matrix_fock(bi.U.T @ bj.U) @ fock.mps_to_vector(bj.sites)
            S[i, j] = vi @ vj
            H[i, j] = vi @ (Hf @ vj)
    return H, S


def test_lossless_equals_brute_force(c1):
    Hx, Sx = _exact_pencil_fock(c1)
    for method in ("fci", "mpo"):
        H, S, E, c, rep = subspace(c1, chi_cap=10 ** 6, h_method=method)
        assert np.abs(H - Hx).max() <= 1e-12 * np.abs(Hx).max()
        assert np.abs(S - Sx).max() <= 1e-12
        assert rep["max_discarded_weight_sum"] < 1e-25
    # the exact pencil's lowest root is a variational upper bound of the FCI energy
    f = fock.SectorFCI(c1.N, c1.n_alpha, c1.n_beta)
    e_fci = np.linalg.eigvalsh(f.hamiltonian_dense(c1.h, c1.L))[0]
    assert E >= e_fci - 1e-12


@pytest.mark.parametrize("cfg", [1, 2])
def test_truncated_pencil_within_error_bound(cfg, c1, c2):
    prob = c1 if cfg == 1 else c2
    H, S, E, c, rep = subspace(prob)
    Hl, Sl, El, cl, _ = subspace(prob, chi_cap=10 ** 6)
    f = fock.SectorFCI(prob.N, prob.n_alpha, prob.n_beta)
    for i in range(prob.M):
        for j in range(i + 1, prob.M):
            _, _, st = pair_element(prob, i, j)
            bound = sum(np.sqrt(x["discarded"]) for x in st)
            hi, Li = rotate_integrals(prob.h, prob.L, prob.mps[i].U)
            vi = f.from_mps(prob.mps[i].sites)
            Hvi = f.apply_one_body(hi - 0.5 * np.einsum("prrq->pq", np.einsum("kpq,krs->pqrs", Li, Li)), vi)
            for k in range(Li.shape[0]):
                Hvi = Hvi + 0.5 * f.apply_one_body(Li[k], f.apply_one_body(Li[k], vi))
            normH = np.linalg.norm(Hvi)
            assert abs(S[i, j] - Sl[i, j]) <= bound + 1e-12
            assert abs(H[i, j] - Hl[i, j]) <= normH * bound + 1e-11
    np.testing.assert_allclose(np.diag(S), 1.0, atol=1e-12)


def test_lossless_hermiticity_two_bases(c2):
    # H_ij with j rotated into i equals H_ji with i rotated into j (G(W)^T = G(W^T))
    for (i, j) in [(0, 1), (1, 3)]:
        hij, sij, _ = pair_element(c2, i, j, chi_cap=10 ** 6)
        hji, sji, _ = pair_element(c2.__class__(**{**c2.__dict__, "mps": [c2.mps[j], c2.mps[i]]}), 0, 1,
                                   chi_cap=10 ** 6)
        assert abs(hij - hji) < 1e-12
        assert abs(sij - sji) < 1e-13


def test_global_rotation_invariance(c1):
    # U_j -> Q^T U_j for all j with h -> Q^T h Q, L -> Q^T L Q leaves H and S unchanged
    r = np.random.default_rng(5)
    Q, _ = np.linalg.qr(r.normal(size=(c1.N, c1.N)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    rot = synth.Problem(N=c1.N, n_alpha=c1.n_alpha, n_beta=c1.n_beta, h=Q.T @ c1.h @ Q,
                        L=np.einsum("pa,kpq,qb->kab", Q, c1.L, Q), e_core=0.0, chi=c1.chi,
                        mps=[synth.MPS(m.sites, m.bond_qn, Q.T @ m.U) for m in c1.mps])
    H0, S0, E0, _, _ = subspace(c1, chi_cap=10 ** 6)
    H1, S1, E1, _, _ = subspace(rot, chi_cap=10 ** 6)
    np.testing.assert_allclose(H1, H0, atol=1e-12)
    np.testing.assert_allclose(S1, S0, atol=1e-13)


def test_fci_spectrum_independent_of_basis(c1):
    f = fock.SectorFCI(c1.N, c1.n_alpha, c1.n_beta)
    e0 = np.linalg.eigvalsh(f.hamiltonian_dense(c1.h, c1.L))
    hi, Li = rotate_integrals(c1.h, c1.L, c1.mps[1].U)
    e1 = np.linalg.eigvalsh(f.hamiltonian_dense(hi, Li))
    np.testing.assert_allclose(e1, e0, atol=1e-12)


def test_rotated_ket_conserves_particle_number(c1):
    N = c1.N
    ket, kqn, st = rotate_ket(c1.mps[1].sites, c1.mps[1].bond_qn, c1.mps[0].U.T @ c1.mps[1].U, c1.chi)
    v = fock.mps_to_vector(ket)
    nu, nd = fock.number_ops(N)
    nrm = v @ v
    assert abs(v @ (nu @ v) - c1.n_alpha * nrm) < 1e-12
    assert abs(v @ (nd @ v) - c1.n_beta * nrm) < 1e-12
    assert M.check_qn(ket, kqn) == 0.0


def test_gep_closed_forms():
    r = np.random.default_rng(0)
    # M = 1: Rayleigh quotient
    sol = gep.solve_projection(np.array([[-3.2]]), np.array([[0.7]]))
    assert abs(sol["E"] - (-3.2 / 0.7)) < 1e-14
    # M = 2 with S_ii = 1: lowest root of (1-s^2)E^2 - (H11+H22-2sH12)E + (H11H22-H12^2)
    H = np.array([[-1.3, 0.2], [0.2, -0.9]])
    s = 0.35
    S = np.array([[1.0, s], [s, 1.0]])
    a, b, c = 1 - s * s, -(H[0, 0] + H[1, 1] - 2 * s * H[0, 1]), H[0, 0] * H[1, 1] - H[0, 1] ** 2
    want = (-b - np.sqrt(b * b - 4 * a * c)) / (2 * a)
    assert abs(gep.solve_projection(H, S)["E"] - want) < 1e-14
    # textbook dsygv when nothing is dropped, and inversion agrees with projection
    for n in (3, 6, 16):
        A = r.normal(size=(n, n))
        Sx = A @ A.T / n + np.eye(n)
        Hx = r.normal(size=(n, n))
        Hx = Hx + Hx.T
        e_ref = scipy.linalg.eigh(Hx, Sx, eigvals_only=True)[0]
        p = gep.solve_projection(Hx, Sx)
        q = gep.solve_inversion(Hx, Sx)
        assert p["n_dropped"] == 0
        assert abs(p["E"] - e_ref) < 1e-12 * max(1, abs(e_ref))
        assert abs(q["E"] - e_ref) < 1e-10 * max(1, abs(e_ref))
        assert abs(p["c"] @ Sx @ p["c"] - 1.0) < 1e-12


def test_gep_report_hand_solved():
    """kappa_1 (App. A2), cond(S), lambda_min(S) and the dropped count on
    pencils solved by hand."""
    # H = [[0, 1], [1, 0]], S = [[1, 1/2], [1/2, 1]]: det(H - E S) = 0 reads
    # (3/4) E^2 + E - 1 = 0, roots -2 and 2/3; at E = -2, H + 2 S = [[2, 2], [2, 2]]
    # so c = (1, -1) (c^T S c = 1 + 1 - 1 = 1 already), |c|^2 = 2,
    # kappa_1 = 2 / sqrt(5); eigenvalues of S are 3/2 and 1/2
    sol = gep.solve_projection(np.array([[0.0, 1.0], [1.0, 0.0]]), np.array([[1.0, 0.5], [0.5, 1.0]]))
    assert abs(sol["E"] + 2.0) < 1e-14
    assert abs(abs(sol["c"][0]) - 1.0) < 1e-14 and abs(sol["c"][0] + sol["c"][1]) < 1e-14
    assert abs(sol["kappa1"] - 2.0 / np.sqrt(5.0)) < 1e-14
    assert abs(sol["cond_S"] - 3.0) < 1e-13
    assert abs(sol["lam_min"] - 0.5) < 1e-14
    assert sol["n_dropped"] == 0
    # diagonal S = diag(4, 1e-3, 1e-14) with H = diag(-8, 1, 5): the third
    # eigenvalue is below 1e-12 * 4 and is dropped; the reduced problem is
    # diag(-8/4, 1/1e-3) so E = -2, c = (1/2, 0, 0), kappa_1 = (1/4) / sqrt(5)
    sol = gep.solve_projection(np.diag([-8.0, 1.0, 5.0]), np.diag([4.0, 1e-3, 1e-14]))
    assert sol["n_dropped"] == 1
    assert abs(sol["E"] + 2.0) < 1e-14
    np.testing.assert_allclose(np.abs(sol["c"]), [0.5, 0.0, 0.0], atol=1e-15)
    assert abs(sol["kappa1"] - 0.25 / np.sqrt(5.0)) < 1e-15
    assert abs(sol["cond_S"] - 4.0 / 1e-3) < 1e-9
    assert sol["lam_min"] == 1e-14
    # a negative eigenvalue of S (possible under truncation) is reported and dropped
    sol = gep.solve_projection(np.diag([-1.0, 2.0]), np.diag([1.0, -1e-9]))
    assert sol["n_dropped"] == 1 and sol["lam_min"] == -1e-9 and abs(sol["E"] + 1.0) < 1e-15
    assert abs(sol["kappa1"] - 1.0 / np.sqrt(2.0)) < 1e-15


def test_duplicated_mps_singular_overlap(c1):
    dup = synth.Problem(**{**c1.__dict__, "mps": [c1.mps[0], c1.mps[1], c1.mps[1]]})
    H2, S2, E2, _, rep2 = subspace(c1, chi_cap=10 ** 6)
    H3, S3, E3, _, rep3 = subspace(dup, chi_cap=10 ** 6)
    assert rep3["n_dropped"] == 1
    assert abs(E3 - E2) < 1e-10
