"""Brute-force Fock space and sector FCI (eq. ham_def, eq. fci of arXiv 2404.10223).

Conventions (the paper leaves them open; Sec. II.A only names the local labels):

* Spatial-orbital sites p = 0..N-1, local index k = n_up + 2 n_dn.
* Fermionic mode order (Jordan-Wigner order) (0 up, 0 dn, 1 up, 1 dn, ...).
* |k_0 ... k_{N-1}> = prod_p (a+_{p up})^{n_p up} (a+_{p dn})^{n_p dn} |vac>,
  site 0 leftmost; Fock index sum_p k_p 4^(N-1-p).
* H = sum_{pq,s} h_pq a+_{ps} a_{qs}
      + 1/2 sum_{pqrs,st} g_pqrs a+_{ps} a+_{rt} a_{st} a_{qs} + e_core,
  with g in chemists' notation (pq|rs).  The paper's eq. ham_def gives only a
  generic two-body sum; this is the standard spin-summed reading.

Creation operators here are built by counting occupied modes that precede the
target mode (plain Jordan-Wigner), not from per-site 4x4 matrices.
"""
from itertools import combinations
from math import comb

import numpy as np
import scipy.sparse as sp


# ---------------------------------------------------------------- full Fock space
def _occupations(N):
    """occ[state, mode] for all 4^N states (mode = 2p + spin)."""
    idx = np.arange(4 ** N)
    occ = np.zeros((4 ** N, 2 * N), dtype=np.int64)
    for p in range(N):
        k = (idx // 4 ** (N - 1 - p)) % 4
        occ[:, 2 * p] = k & 1
        occ[:, 2 * p + 1] = k >> 1
    return occ


def _index(occ, N):
    k = occ[:, 0::2] + 2 * occ[:, 1::2]
    w = 4 ** (N - 1 - np.arange(N))
    return (k * w).sum(axis=1)


def creation_ops(N):
    """List of sparse a+_m (m = 2p + spin) on the 4^N Fock space."""
    occ = _occupations(N)
    D = 4 ** N
    ops = []
    for m in range(2 * N):
        ok = occ[:, m] == 0
        src = np.nonzero(ok)[0]
        new = occ[src].copy()
        new[:, m] = 1
        sign = (-1.0) ** occ[src, :m].sum(axis=1)
        ops.append(sp.csr_matrix((sign, (_index(new, N), src)), shape=(D, D)))
    return ops


def hamiltonian_fock(h, g, e_core=0.0):
    """Sparse second-quantised H on the full 4^N Fock space."""
    N = h.shape[0]
    cr = creation_ops(N)
    an = [c.T.tocsr() for c in cr]
    D = 4 ** N
    H = sp.csr_matrix((D, D))
    for p in range(N):
        for q in range(N):
            for s in (0, 1):
                if h[p, q] != 0.0:
                    H = H + h[p, q] * (cr[2 * p + s] @ an[2 * q + s])
    for p in range(N):
        for q in range(N):
            for r in range(N):
                for s_ in range(N):
                    v = 0.5 * g[p, q, r, s_]
                    if v == 0.0:
                        continue
                    for sg in (0, 1):
                        for tu in (0, 1):
                            H = H + v * (cr[2 * p + sg] @ cr[2 * r + tu] @ an[2 * s_ + tu] @ an[2 * q + sg])
    if e_core:
        H = H + e_core * sp.identity(D, format="csr")
    return H


def number_ops(N):
    cr = creation_ops(N)
    nu = sum(cr[2 * p] @ cr[2 * p].T for p in range(N))
    nd = sum(cr[2 * p + 1] @ cr[2 * p + 1].T for p in range(N))
    return nu, nd


def apply_two_site_gate(psi, N, p, G16):
    """Apply a 16x16 gate on sites (p, p+1) of a full Fock vector."""
    t = psi.reshape((4 ** p, 16, 4 ** (N - p - 2)))
    return np.einsum("ij,ajb->aib", G16, t).reshape(-1)


def apply_site_gate(psi, N, p, G4):
    t = psi.reshape((4 ** p, 4, 4 ** (N - p - 1)))
    return np.einsum("ij,ajb->aib", G4, t).reshape(-1)


# ------------------------------------------------ determinant form of G(W) (Thouless)
def _eps(occ_up, occ_dn):
    """Sign taking the interleaved mode order to (all up ascending)(all dn ascending)."""
    s = 0
    for q in occ_dn:
        s += sum(1 for pu in occ_up if pu > q)
    return -1.0 if s % 2 else 1.0


def rotation_matrix_fock(W):
    """<k'| G(W) |k> with G(W) a+_p G^+ = sum_q W_qp a+_q (dense, N <= 5)."""
    N = W.shape[0]
    occ = _occupations(N)
    D = 4 ** N
    G = np.zeros((D, D))
    ups = [tuple(np.nonzero(occ[i, 0::2])[0]) for i in range(D)]
    dns = [tuple(np.nonzero(occ[i, 1::2])[0]) for i in range(D)]

    def det(rows, cols):
        if len(rows) == 0:
            return 1.0
        return np.linalg.det(W[np.ix_(rows, cols)])

    for i in range(D):
        for j in range(D):
            if len(ups[i]) != len(ups[j]) or len(dns[i]) != len(dns[j]):
                continue
            G[i, j] = (_eps(ups[i], dns[i]) * _eps(ups[j], dns[j])
                       * det(list(ups[i]), list(ups[j])) * det(list(dns[i]), list(dns[j])))
    return G


# ----------------------------------------------------------------- MPS <-> vectors
def mps_to_vector(sites):
    """Contract an MPS (list of [dl, 4, dr]) to its 4^N Fock vector."""
    v = sites[0][0]                       # [4, dr]
    for A in sites[1:]:
        dl, _, dr = A.shape
        v = (v @ A.reshape(dl, 4 * dr)).reshape(-1, dr)
    return v[:, 0].copy()


# ------------------------------------------------------------------ sector FCI
class SectorFCI:
    """Determinant space with fixed (N_alpha, N_beta), vectors as V[alpha, beta].

    H = sum_pq h'_pq E_pq + 1/2 sum_k Lhat_k^2 + e_core, h' = h - 1/2 sum_r g_prrq,
    Lhat_k = sum_pq L^k_pq E_pq, E_pq = sum_s a+_ps a_qs (the Cholesky form of
    the two-electron operator; E_pq acts on alpha strings from the left and on
    beta strings from the right of V).
    """

    def __init__(self, N, na, nb):
        self.N, self.na, self.nb = N, na, nb
        self.sa = [tuple(c) for c in combinations(range(N), na)]
        self.sb = [tuple(c) for c in combinations(range(N), nb)]
        self.ia = {s: i for i, s in enumerate(self.sa)}
        self.ib = {s: i for i, s in enumerate(self.sb)}
        self.Ea = self._epq(self.sa, self.ia)
        self.Eb = self._epq(self.sb, self.ib)

    def _epq(self, strings, index):
        """Transitions of E_pq = a+_p a_q on one spin species: (p, q, row, col, sign)."""
        N = self.N
        out = []
        for j, st in enumerate(strings):
            st = list(st)
            for sq, q in enumerate(st):           # a_q: sign (-1)^(#occupied before q)
                rest = st[:sq] + st[sq + 1:]
                for p in range(N):
                    if p in rest:
                        continue
                    sp_ = sum(1 for r in rest if r < p)
                    new = tuple(sorted(rest + [p]))
                    out.append((p, q, index[new], j, (-1.0) ** (sq + sp_)))
        a = np.array(out, dtype=float).reshape(-1, 5)
        return (a[:, 0].astype(int), a[:, 1].astype(int), a[:, 2].astype(int),
                a[:, 3].astype(int), a[:, 4], len(strings))

    def dim(self):
        return len(self.sa) * len(self.sb)

    def _maps(self):
        if not hasattr(self, "_idx"):
            N = self.N
            w = 4 ** (N - 1 - np.arange(N))
            oa = np.zeros((len(self.sa), N), dtype=np.int64)
            for i, a in enumerate(self.sa):
                oa[i, list(a)] = 1
            ob = np.zeros((len(self.sb), N), dtype=np.int64)
            for i, b in enumerate(self.sb):
                ob[i, list(b)] = 1
            self._idx = (oa @ w)[:, None] + 2 * (ob @ w)[None, :]
            # number of alpha electrons strictly to the right of each orbital
            greater = np.cumsum(oa[:, ::-1], axis=1)[:, ::-1] - oa
            self._sgn = 1.0 - 2.0 * ((greater @ ob.T) % 2)
        return self._idx, self._sgn

    def from_fock(self, psi):
        """Fock vector (site basis) -> V[alpha, beta] in the (up-block)(dn-block) basis."""
        idx, sgn = self._maps()
        return sgn * psi[idx]

    def from_mps(self, sites):
        return self.from_fock(mps_to_vector(sites))

    def one_body(self, t):
        """Sparse matrices of sum_pq t_pq E_pq on alpha and on beta strings."""
        mats = []
        for p, q, r, c, s, n in (self.Ea, self.Eb):
            mats.append(sp.csr_matrix((t[p, q] * s, (r, c)), shape=(n, n)))
        return mats[0], mats[1]

    def apply_one_body(self, t, V):
        Aa, Ab = self.one_body(t)
        return Aa @ V + (Ab @ V.T).T

    def expectation(self, h, L, e_core, Vbra, Vket):
        """<bra| H |ket> with H in Cholesky form (g = sum_k L^k x L^k)."""
        g = np.einsum("kpq,krs->pqrs", L, L)
        hp = h - 0.5 * np.einsum("prrq->pq", g)
        val = np.sum(Vbra * self.apply_one_body(hp, Vket))
        for k in range(L.shape[0]):
            val += 0.5 * np.sum(self.apply_one_body(L[k], Vbra) * self.apply_one_body(L[k], Vket))
        return val + e_core * np.sum(Vbra * Vket)

    def hamiltonian_dense(self, h, L, e_core=0.0):
        """Dense sector Hamiltonian (small sectors only)."""
        n = self.dim()
        H = np.zeros((n, n))
        for j in range(n):
            e = np.zeros(n)
            e[j] = 1.0
            V = e.reshape(len(self.sa), len(self.sb))
            g = np.einsum("kpq,krs->pqrs", L, L)
            hp = h - 0.5 * np.einsum("prrq->pq", g)
            W = self.apply_one_body(hp, V)
            for k in range(L.shape[0]):
                W = W + 0.5 * self.apply_one_body(L[k], self.apply_one_body(L[k], V))
            H[:, j] = W.reshape(-1) + e_core * e
        return H


def sector_dim(N, na, nb):
    return comb(N, na) * comb(N, nb)
