"""Pins of the two-site gates and the Givens plan (App. A3, App. D, Sec. II.B)."""
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import fock, gates, givens

GOLD = os.path.join(os.path.dirname(__file__), "golden", "app_a3_gates.txt")


def _printed(name, theta=0.0):
    c, s, r = np.cos(theta), np.sin(theta), 1.0 / np.sqrt(2.0)
    for line in open(GOLD):
        if line.startswith(name + ":"):
            vals = [{"c": c, "s": s, "-s": -s, "r": r, "-r": -r}.get(t, None) for t in line.split()[1:]]
            vals = [float(t) if v is None else v for t, v in zip(line.split()[1:], vals)]
            return np.array(vals).reshape(4, 4)
    raise KeyError(name)


def test_d2_gates_match_paper():
    np.testing.assert_array_equal(gates.F2, _printed("fswap"))
    for th in (0.0, 0.3, -1.1, 2.5):
        np.testing.assert_allclose(gates.g2(th), _printed("givens", th), atol=1e-15)
    np.testing.assert_allclose(gates.g2(np.pi / 4), _printed("givens_pi4"), atol=1e-15)


def test_phased_fswap_is_givens_pi_half():
    Z = np.diag([1.0, -1.0])
    np.testing.assert_allclose(np.kron(np.eye(2), Z) @ gates.F2, gates.g2(np.pi / 2), atol=1e-15)


def test_g4_group_and_symmetry():
    np.testing.assert_allclose(gates.g4(0.0), np.eye(16), atol=0)
    a, b = 0.37, -1.21
    np.testing.assert_allclose(gates.g4(a) @ gates.g4(b), gates.g4(a + b), atol=1e-14)
    G = gates.g4(0.7)
    np.testing.assert_allclose(G.T @ G, np.eye(16), atol=1e-14)
    assert np.count_nonzero(np.abs(G) > 1e-14) == 36
    # conserves n_up and n_dn of the pair
    nup = np.array([(k1 & 1) + (k2 & 1) for k1 in range(4) for k2 in range(4)])
    ndn = np.array([(k1 >> 1) + (k2 >> 1) for k1 in range(4) for k2 in range(4)])
    nz = np.abs(G) > 1e-14
    assert np.all(nup[:, None] == nup[None, :], where=nz)
    assert np.all(ndn[:, None] == ndn[None, :], where=nz)


def test_g4_equals_exponential_generator():
    # exp[theta sum_s (a+_{p s} a_{p+1 s} - h.c.)] built from Jordan-Wigner creation ops
    cr = fock.creation_ops(2)
    Gen = sum(cr[s] @ cr[2 + s].T - cr[2 + s] @ cr[s].T for s in (0, 1)).toarray()
    for th in (0.1, 0.9, -2.3):
        np.testing.assert_allclose(gates.g4(th), scipy.linalg.expm(th * Gen), atol=1e-14)


def test_g4_worked_column():
    # g4|updn, 0> = c^2|updn,0> - cs|up,dn> + cs|dn,up> + s^2|0,updn>
    th = 0.61
    c, s = np.cos(th), np.sin(th)
    col = gates.g4(th)[:, 3 * 4 + 0]
    want = np.zeros(16)
    want[3 * 4 + 0] = c * c
    want[1 * 4 + 2] = -c * s
    want[2 * 4 + 1] = c * s
    want[0 * 4 + 3] = s * s
    np.testing.assert_allclose(col, want, atol=1e-15)
    # same-spin pairs are invariant
    G = gates.g4(th)
    for k1, k2 in ((1, 1), (2, 2), (3, 3), (0, 0)):
        e = np.zeros(16)
        e[k1 * 4 + k2] = 1.0
        np.testing.assert_allclose(G @ e, e, atol=1e-15)


def test_f4_is_fermionic_site_swap():
    F = gates.f4()
    for k1 in range(4):
        for k2 in range(4):
            n1, n2 = bin(k1).count("1"), bin(k2).count("1")
            e = np.zeros(16)
            e[k1 * 4 + k2] = 1.0
            want = np.zeros(16)
            want[k2 * 4 + k1] = (-1.0) ** (n1 * n2)
            np.testing.assert_allclose(F @ e, want, atol=1e-15)


def _random_orthogonal(N, seed, det=1):
    r = np.random.default_rng(seed)
    Q, R = np.linalg.qr(r.normal(size=(N, N)))
    Q = Q * np.sign(np.diag(R))[None, :]
    if np.linalg.det(Q) * det < 0:
        Q[:, 0] = -Q[:, 0]
    return Q


@pytest.mark.parametrize("N", [2, 3, 5, 8, 24])
@pytest.mark.parametrize("det", [1, -1])
def test_plan_reproduces_rotation(N, det):
    W = _random_orthogonal(N, 10 * N + (det > 0), det)
    gl, ds = givens.plan(W)
    assert len(gl) == N * (N - 1) // 2
    assert ds == det
    np.testing.assert_allclose(givens.compose(N, gl, ds), W, atol=1e-13)


def test_plan_column_order():
    # application order = column groups c = N-2 .. 0, each a left-to-right run
    N = 5
    gl, _ = givens.plan(_random_orthogonal(N, 3))
    want = [a for c in range(N - 2, -1, -1) for a in range(c, N - 1)]
    assert [a for a, _ in gl] == want


@pytest.mark.parametrize("det", [1, -1])
def test_network_equals_determinant_formula(det):
    N = 4
    W = _random_orthogonal(N, 7, det)
    gl, ds = givens.plan(W)
    Gdet = fock.rotation_matrix_fock(W)
    psi = np.random.default_rng(1).normal(size=4 ** N)
    v = psi.copy()
    if ds < 0:
        v = fock.apply_site_gate(v, N, N - 1, gates.parity_gate())
    for a, th in gl:
        v = fock.apply_two_site_gate(v, N, a, gates.g4(th))
    np.testing.assert_allclose(v, Gdet @ psi, atol=1e-13)


def test_determinant_formula_is_a_representation():
    N = 3
    A, B = _random_orthogonal(N, 1), _random_orthogonal(N, 2, -1)
    GA, GB = fock.rotation_matrix_fock(A), fock.rotation_matrix_fock(B)
    np.testing.assert_allclose(GA @ GB, fock.rotation_matrix_fock(A @ B), atol=1e-13)
    np.testing.assert_allclose(GA.T, fock.rotation_matrix_fock(A.T), atol=1e-13)
    # a single Givens rotation R_p(theta) is the gate g4(theta) on sites (p, p+1)
    th = 0.83
    G = fock.rotation_matrix_fock(givens.rot(N, 1, th))
    v = np.random.default_rng(3).normal(size=4 ** N)
    np.testing.assert_allclose(G @ v, fock.apply_two_site_gate(v, N, 1, gates.g4(th)), atol=1e-14)


def test_plan_ignores_rounding_noise():
    # W = I + noise plans as an identity network; a signed permutation still reproduces W
    r = np.random.default_rng(9)
    N = 6
    W = np.eye(N) + 1e-16 * r.normal(size=(N, N))
    gl, ds = givens.plan(W)
    assert ds == 1 and all(th == 0.0 for _, th in gl)
    P = np.eye(N)[[2, 0, 1, 5, 3, 4]]
    P[:, 1] *= -1
    P[:, 4] *= -1
    gl, ds = givens.plan(P)
    np.testing.assert_allclose(givens.compose(N, gl, ds), P, atol=1e-13)
