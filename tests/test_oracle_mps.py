"""Pins of the MPS layer: canonical form, gate + truncation, error bound, App. D."""
import numpy as np
import pytest

import tnqe_synth as synth
from oracle import fock, gates, givens, mps as M
from oracle.subspace import rotate_ket


def _vec(sites):
    return fock.mps_to_vector(sites)


@pytest.fixture(scope="module")
def c1():
    return synth.make_config(1)


@pytest.fixture(scope="module")
def c2():
    return synth.make_config(2)


def test_generated_mps_are_sector_states(c1, c2):
    for prob in (c1, c2):
        for m in prob.mps:
            assert M.check_qn(m.sites, m.bond_qn) == 0.0
            assert abs(M.overlap(m.sites, m.sites) - 1.0) < 1e-13
            np.testing.assert_allclose(m.U.T @ m.U, np.eye(prob.N), atol=1e-13)
    # particle number: <N_up> = n_alpha, <N_dn> = n_beta (Fock space, N = 4)
    nu, nd = fock.number_ops(c1.N)
    v = _vec(c1.mps[0].sites)
    assert abs(v @ (nu @ v) - c1.n_alpha) < 1e-12
    assert abs(v @ (nd @ v) - c1.n_beta) < 1e-12


def test_canonical_moves_are_exact(c2):
    m = c2.mps[1]
    s, q = M.copy_mps(m.sites, m.bond_qn)
    v0 = _vec(s)
    # scramble the gauge first: push the centre to the left end
    c = M.move_centre(s, q, len(s) - 1, 0)
    np.testing.assert_allclose(_vec(s), v0, atol=1e-13)
    for A in s[1:]:               # right-orthonormal
        np.testing.assert_allclose(np.einsum("akb,ckb->ac", A, A), np.eye(A.shape[0]), atol=1e-13)
    M.move_centre(s, q, c, 3)
    for A in s[:3]:               # left-orthonormal
        np.testing.assert_allclose(np.einsum("akb,akc->bc", A, A), np.eye(A.shape[2]), atol=1e-13)
    np.testing.assert_allclose(_vec(s), v0, atol=1e-13)
    assert M.check_qn(s, q) == 0.0


def test_gate_without_truncation_is_exact(c2):
    m = c2.mps[2]
    s, q = M.copy_mps(m.sites, m.bond_qn)
    c = M.left_canonicalize(s, q)
    M.move_centre(s, q, c, 2)
    v0 = _vec(s)
    st = M.gate_and_truncate(s, q, 2, gates.g4(0.45), 10 ** 6, 0.0)
    np.testing.assert_allclose(_vec(s), fock.apply_two_site_gate(v0, c2.N, 2, gates.g4(0.45)), atol=1e-13)
    assert st["discarded"] < 1e-28
    assert M.check_qn(s, q) == 0.0


def test_block_svd_equals_dense_svd(c2):
    m = c2.mps[0]
    s, q = M.copy_mps(m.sites, m.bond_qn)
    c = M.left_canonicalize(s, q)
    M.move_centre(s, q, c, 3)
    A, B = s[3], s[4]
    T = np.einsum("akm,mlb->aklb", A, B).reshape(A.shape[0], 16, B.shape[2])
    T = np.einsum("xy,ayb->axb", gates.g4(0.3), T).reshape(A.shape[0] * 4, 4 * B.shape[2])
    dense = np.linalg.svd(T, compute_uv=False)
    st = M.gate_and_truncate(s, q, 3, gates.g4(0.3), 10 ** 6, 0.0)
    blocks = np.linalg.svd(s[4].reshape(s[4].shape[0], -1), compute_uv=False)   # A_{p+1} = Sigma V^T
    n = len(blocks)
    np.testing.assert_allclose(np.sort(blocks)[::-1], dense[:n], atol=1e-13)
    assert np.all(dense[n:] < 1e-12)


def test_truncation_is_orthogonal_projection(c2):
    m = c2.mps[3]
    s, q = M.copy_mps(m.sites, m.bond_qn)
    c = M.left_canonicalize(s, q)
    M.move_centre(s, q, c, 3)
    v_full = fock.apply_two_site_gate(_vec(s), c2.N, 3, gates.g4(1.0))
    st = M.gate_and_truncate(s, q, 3, gates.g4(1.0), 5, 1e-13)
    v_tr = _vec(s)
    assert st["kept"] == 5 and st["discarded"] > 1e-6
    # projection: <v_tr | v_full - v_tr> = 0 and norms add up
    assert abs(v_tr @ (v_full - v_tr)) < 1e-13
    assert abs(v_full @ v_full - v_tr @ v_tr - st["discarded"]) < 1e-13


def _exact_rotated(prob, i, j):
    """G(U_i^T U_j)|Phi_j> on the full Fock space, by exact gates."""
    N = prob.N
    W = prob.mps[i].U.T @ prob.mps[j].U
    gl, ds = givens.plan(W)
    v = _vec(prob.mps[j].sites)
    if ds < 0:
        v = fock.apply_site_gate(v, N, N - 1, gates.parity_gate())
    for a, th in gl:
        v = fock.apply_two_site_gate(v, N, a, gates.g4(th))
    return v


@pytest.mark.parametrize("cfg", [1, 2])
def test_error_bound_of_sequential_truncation(cfg, c1, c2):
    prob = c1 if cfg == 1 else c2
    for (i, j) in [(0, 1)] + ([(1, 3), (2, 3)] if cfg == 2 else []):
        exact = _exact_rotated(prob, i, j)
        ket, kqn, st = rotate_ket(prob.mps[j].sites, prob.mps[j].bond_qn,
                                  prob.mps[i].U.T @ prob.mps[j].U, prob.chi)
        err = np.linalg.norm(_vec(ket) - exact)
        bound = sum(np.sqrt(x["discarded"]) for x in st)
        assert bound > 1e-3                 # the workload does truncate
        assert err <= bound * (1 + 1e-12) + 1e-13
        assert M.check_qn(ket, kqn) == 0.0


def test_lossless_rotation_is_exact(c1):
    exact = _exact_rotated(c1, 0, 1)
    ket, _, st = rotate_ket(c1.mps[1].sites, c1.mps[1].bond_qn, c1.mps[0].U.T @ c1.mps[1].U, 10 ** 6)
    np.testing.assert_allclose(_vec(ket), exact, atol=1e-13)
    assert max(x["kept"] for x in st) <= 16        # maximal Schmidt rank of the (2,2) sector at N = 4


def _app_d_network(N):
    """pi/4 and pi/2 rotations of App. D taking |1..1 0..0> to a maximally entangled state."""
    m = N // 2
    seq = []
    for t in range(m):
        seq.append((m - 1, np.pi / 4))
        seq += [(a, np.pi / 2) for a in range(m, N - 1 - t)]          # particle to the right end
        seq += [(a, np.pi / 2) for a in range(m - 2, t - 1, -1)]      # hole to the left end
    return seq


def _closed_shell_mps(N):
    """chi = 1 MPS of the determinant with sites 0..N/2-1 doubly occupied."""
    sites, qn = [], [np.zeros((1, 2), dtype=np.int64)]
    acc = np.zeros(2, dtype=np.int64)
    for p in range(N):
        A = np.zeros((1, 4, 1))
        k = 3 if p < N // 2 else 0
        A[0, k, 0] = 1.0
        acc = acc + M.QK[k]
        sites.append(A)
        qn.append(acc.reshape(1, 2).copy())
    return sites, qn


@pytest.mark.parametrize("N", [4, 6])
def test_app_d_maximal_entanglement(N):
    sites, qn = _closed_shell_mps(N)
    centre = M.left_canonicalize(sites, qn)
    for a, th in _app_d_network(N):
        centre = M.move_centre(sites, qn, centre, a)
        M.gate_and_truncate(sites, qn, a, gates.g4(th), 10 ** 6, 1e-13)
        centre = a + 1
    v = _vec(sites)
    sv = np.linalg.svd(v.reshape(4 ** (N // 2), -1), compute_uv=False)
    rank = int((sv > 1e-12).sum())
    assert rank == 2 ** N                                # (2^(N/2))^2 for the two spins
    np.testing.assert_allclose(sv[:rank], 2.0 ** (-N / 2), atol=1e-12)
    # one truncation at the centre to chi discards exactly 1 - chi 2^-N
    centre = M.move_centre(sites, qn, centre, N // 2 - 1)
    chi = 4
    st = M.gate_and_truncate(sites, qn, N // 2 - 1, np.eye(16), chi, 1e-13)
    assert abs(st["discarded"] - (1 - chi * 2.0 ** (-N))) < 1e-12
    assert st["gap"] == pytest.approx(0.0, abs=1e-12)     # the all-ties case


def test_select_kept_is_best_subset_brute_force():
    """The truncation rule of App. A1 against exhaustive search on tiny lists:
    among all index sets of the kept size, the one with the largest retained
    weight (ties: the lexicographically smallest index set, i.e. equal values
    kept in list order), the kept size being min(chi, #{s^2 > tau sum s^2})."""
    from itertools import combinations
    rng = np.random.default_rng(7)
    for case in range(300):
        n = int(rng.integers(1, 8))
        # few distinct values so that ties are frequent; some exact zeros
        sv = rng.choice([0.0, 0.1, 0.25, 0.5, 1.0, 2.0], size=n)
        chi = int(rng.integers(1, n + 2))
        tau = float(rng.choice([0.0, 1e-3, 0.02, 0.3]))
        mask, keep, nnz, gap, disc, total = M.select_kept(sv, chi, tau)
        w2 = sv ** 2
        assert total == pytest.approx(w2.sum(), abs=0)
        above = sum(1 for x in w2 if x > tau * w2.sum())
        assert nnz == above and keep == min(chi, above)
        best = None
        for S in combinations(range(n), keep):          # lexicographic order
            w = sum(w2[i] for i in S)
            if best is None or w > best[0] + 1e-12:       # ties differ only by rounding
                best = (w, S)
        want = np.zeros(n, dtype=bool)
        want[list(best[1])] = True
        assert (mask == want).all(), (sv, chi, tau)
        assert disc == pytest.approx(w2[~want].sum(), abs=1e-15)
        if 0 < keep < n:
            s_in = min(sv[want])
            s_out = max(sv[~want])
            assert gap == pytest.approx((s_in - s_out) / s_in)
        else:
            assert gap is None


def test_renormalized_network_is_the_normalized_projection():
    """With renormalisation after every cut the rotated ket has unit norm and
    equals the plain (projected) ket divided by its norm: the kept subspace of
    a cut does not depend on the scale of the state, so rescaling commutes
    with every later gate and cut."""
    import tnqe_synth as synth
    from oracle.subspace import pair_element, rotate_ket
    prob = synth.make_config(2)
    bi, bj = prob.mps[0], prob.mps[2]
    W = bi.U.T @ bj.U
    plain, _, st = rotate_ket(bj.sites, bj.bond_qn, W, prob.chi)
    ren, _, st_r = rotate_ket(bj.sites, bj.bond_qn, W, prob.chi, renormalize=True)
    assert sum(x["discarded"] for x in st) > 1e-6          # the network does cut
    n2 = M.overlap(plain, plain)
    assert abs(M.overlap(ren, ren) - 1.0) < 1e-12
    assert abs(M.overlap(bi.sites, ren) - M.overlap(bi.sites, plain) / np.sqrt(n2)) < 1e-12
    h, s, _ = pair_element(prob, 0, 2)
    hr, sr, _ = pair_element(prob, 0, 2, renormalize=True)
    assert abs(hr - h / np.sqrt(n2)) < 1e-11 * max(1.0, abs(h))
    assert abs(sr - s / np.sqrt(n2)) < 1e-13
