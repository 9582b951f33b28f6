"""Pins of the Hamiltonian MPO and its environment sweep (P7)."""
import numpy as np
import pytest

import tnqe_synth as synth
from oracle import fock, mpo, mps as M
from oracle.fock import SectorFCI


def _random_integrals(N, K, seed):
    r = np.random.default_rng(seed)
    h = r.normal(size=(N, N))
    h = 0.5 * (h + h.T)
    L = r.normal(size=(K, N, N)) * 0.3
    L = 0.5 * (L + L.transpose(0, 2, 1))
    return h, L, np.einsum("kpq,krs->pqrs", L, L)


@pytest.mark.parametrize("N", [2, 3, 4, 5])
def test_mpo_contracts_to_fock_hamiltonian(N):
    h, L, g = _random_integrals(N, 3, N)
    W = mpo.build_mpo(h, g)
    Hd, Id = W.to_dense()
    Hf = fock.hamiltonian_fock(h, g).toarray()
    np.testing.assert_allclose(Hd, Hf, atol=1e-12)
    np.testing.assert_array_equal(Id, np.eye(4 ** N))


def test_mpo_bond_dimension_is_quadratic():
    h, L, g = _random_integrals(12, 2, 0)
    d = mpo.build_mpo(h, g).bond_dims()
    assert max(d) <= 2 + 4 * 12 + 8 * 6 * 6
    assert d[0] == 1 and d[-1] == 2


# N = 10 and 12 reach every channel path of the builder at sizes where the
# two-operator channels switch from normal to complementary form at the centre
@pytest.mark.parametrize("N,na,nb,chi", [(6, 3, 2, 12), (7, 4, 4, 10), (8, 4, 4, 20), (10, 5, 5, 16),
                                         (12, 6, 5, 12)])
def test_sweep_equals_sector_fci(N, na, nb, chi):
    h, L, g = _random_integrals(N, 4, 100 + N)
    W = mpo.build_mpo(h, g)
    f = SectorFCI(N, na, nb)
    bra, bq = synth.make_mps(N, na, nb, chi, (7,), 0)
    ket, kq = synth.make_mps(N, na, nb, chi // 2 + 1, (7,), 1)
    H, S = mpo.expectation(W, bra, bq, ket, kq)
    vb, vk = f.from_mps(bra), f.from_mps(ket)
    assert abs(S - np.sum(vb * vk)) < 1e-13
    assert abs(H - f.expectation(h, L, 0.0, vb, vk)) < 1e-11 * max(1.0, abs(H))


def _det_mps(N, occ):
    """chi = 1 MPS of a determinant; occ = set of spin-orbitals 2p + s."""
    sites, qn = [], [np.zeros((1, 2), dtype=np.int64)]
    acc = np.zeros(2, dtype=np.int64)
    for p in range(N):
        k = (1 if 2 * p in occ else 0) + (2 if 2 * p + 1 in occ else 0)
        A = np.zeros((1, 4, 1))
        A[0, k, 0] = 1.0
        acc = acc + M.QK[k]
        sites.append(A)
        qn.append(acc.reshape(1, 2).copy())
    return sites, qn


def _phase(occ_ket, ops):
    """<D| ops |D'> sign for a product of single-mode ops applied right to left."""
    occ = sorted(occ_ket)
    sign = 1
    for m, dag in reversed(ops):
        pos = sum(1 for x in occ if x < m)
        if dag:
            assert m not in occ
            occ = sorted(occ + [m])
        else:
            assert m in occ
            occ.remove(m)
        sign *= (-1) ** pos
    return sign, set(occ)


def _slater_condon(h, g, occ_bra, occ_ket):
    """<D|H|D'> by the Slater-Condon rules (interleaved mode order)."""
    sp = lambda m: m % 2
    o = lambda m: m // 2
    diff_k = sorted(set(occ_ket) - set(occ_bra))
    diff_b = sorted(set(occ_bra) - set(occ_ket))
    if not diff_k:
        e = sum(h[o(i), o(i)] for i in occ_ket)
        for i in occ_ket:
            for j in occ_ket:
                e += 0.5 * g[o(i), o(i), o(j), o(j)]
                if sp(i) == sp(j):
                    e -= 0.5 * g[o(i), o(j), o(j), o(i)]
        return e
    if len(diff_k) == 1:
        i, a = diff_k[0], diff_b[0]
        if sp(i) != sp(a):
            return 0.0
        sign, res = _phase(occ_ket, [(a, 1), (i, 0)])
        assert res == set(occ_bra)
        v = h[o(a), o(i)]
        for j in occ_ket:
            v += g[o(a), o(i), o(j), o(j)]
            if sp(j) == sp(i):
                v -= g[o(a), o(j), o(j), o(i)]
        return sign * v
    if len(diff_k) == 2:
        i, j = diff_k
        a, b = diff_b
        sign, res = _phase(occ_ket, [(a, 1), (b, 1), (j, 0), (i, 0)])
        assert res == set(occ_bra)
        v = 0.0
        if sp(a) == sp(i) and sp(b) == sp(j):
            v += g[o(a), o(i), o(b), o(j)]
        if sp(a) == sp(j) and sp(b) == sp(i):
            v -= g[o(a), o(j), o(b), o(i)]
        return sign * v
    return 0.0


@pytest.mark.parametrize("N", [6, 24])
def test_sweep_matches_slater_condon(N):
    prob = synth.make_problem(N, N // 2, N // 2, 4, 1, max(2, N // 3), (9, N))
    h, g = prob.h, prob.g()
    W = mpo.build_mpo(h, g)
    r = np.random.default_rng(N)
    occ = set(r.choice(np.arange(0, 2 * N, 2), N // 2, replace=False)) | \
        set(r.choice(np.arange(1, 2 * N, 2), N // 2, replace=False))
    occ = {int(x) for x in occ}
    up_occ = sorted(m for m in occ if m % 2 == 0)
    up_vir = sorted(m for m in range(0, 2 * N, 2) if m not in occ)
    dn_occ = sorted(m for m in occ if m % 2 == 1)
    dn_vir = sorted(m for m in range(1, 2 * N, 2) if m not in occ)
    kets = [occ,
            (occ - {up_occ[0]}) | {up_vir[-1]},                               # single, up
            (occ - {dn_occ[-1]}) | {dn_vir[0]},                               # single, down
            (occ - {up_occ[1], dn_occ[0]}) | {up_vir[0], dn_vir[-1]},         # double, opposite spins
            (occ - {up_occ[0], up_occ[-1]}) | {up_vir[0], up_vir[-1]}]        # double, same spin
    bs, bq = _det_mps(N, occ)
    for ket_occ in kets:
        ks, kq = _det_mps(N, ket_occ)
        H, S = mpo.expectation(W, bs, bq, ks, kq)
        want = _slater_condon(h, g, sorted(occ), sorted(ket_occ))
        assert abs(H - want) < 1e-12 * max(1.0, abs(want)), (sorted(ket_occ), H, want)
        assert S == (1.0 if ket_occ == occ else 0.0)


@pytest.mark.parametrize("N,na,nb,chi", [(5, 2, 3, 6), (8, 4, 4, 20)])
def test_plain_contraction_equals_sector_fci(N, na, nb, chi):
    """The ungrouped dense sweep (used to cross-check the full-size values)
    against sector FCI, independently of the block-sparse sweep."""
    h, L, g = _random_integrals(N, 4, 200 + N)
    W = mpo.build_mpo(h, g)
    f = SectorFCI(N, na, nb)
    bra, bq = synth.make_mps(N, na, nb, chi, (8,), 0)
    ket, kq = synth.make_mps(N, na, nb, chi // 2 + 1, (8,), 1)
    H, S = mpo.expectation_plain(W, bra, ket)
    vb, vk = f.from_mps(bra), f.from_mps(ket)
    assert abs(S - np.sum(vb * vk)) < 1e-13
    assert abs(H - f.expectation(h, L, 0.0, vb, vk)) < 1e-11 * max(1.0, abs(H))
