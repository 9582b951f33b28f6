"""Expanded one-hot pencil of one state (Sec. II.E eq. oht_exp and
eq. subs_exp; App. A1) -- test infrastructure only, like the whole package.

The state phi_i is put in canonical form centred on sites (p, p+1): sites
left of p left-orthonormal, sites right of p+1 right-orthonormal (App. A1,
eq. orth_l / orth_r).  Its two-site tensor T[l, k_p, k_{p+1}, r] is then a sum
of one-hot tensors e_m with weights t_m, and replacing T by e_m gives the
one-hot state |varphi_m>; these are orthonormal and phi_i = sum_m t_m varphi_m
(eq. oht_exp).  Only entries that conserve the particle numbers are one-hot
states (the block-sparse structure the paper enforces): qn(l) + q(k_p) +
q(k_{p+1}) = qn(r); they are numbered in row-major order of T.

Expanding state i alone (App. A1: "by expanding a chosen reference state"),
the pencil gains

  H'[im, in] = <varphi_m|H|varphi_n>,  S'[im, in] = <varphi_m|varphi_n> (= delta_mn),
  H'[im, k]  = <varphi_m|H|phi_k>,      S'[im, k]  = <varphi_m|phi_k>   (every k),

with every state taken into basis i: H is H^(i) (integrals rotated into basis
i) and phi_k (k != i) is the ket k rotated into basis i by its Givens network
with truncation to chi, as for the pencil itself (here also for k < i).

Everything is computed from the definition: each one-hot state and each ket
is contracted to its sector-FCI vector and H^(i) is applied in the Cholesky
form (oracle.fock.SectorFCI); no MPO is involved.  Small N only.
"""
import numpy as np

from . import mps as mpsops
from .fock import SectorFCI
from .subspace import rotate_integrals, rotate_ket

QK = mpsops.QK


def canonical_at(sites, qn, p):
    """Copy of the MPS with its orthogonality centre on site p."""
    s, q = mpsops.copy_mps(sites, qn)
    c = mpsops.left_canonicalize(s, q)
    mpsops.move_centre(s, q, c, p)
    return s, q


def onehot_index(qn, p):
    """Allowed one-hot entries (l, k_p, k_{p+1}, r) of the two-site tensor at
    (p, p+1), in row-major order of T[l, k_p, k_{p+1}, r]."""
    out = []
    for l in range(qn[p].shape[0]):
        for kp in range(4):
            for kq in range(4):
                want = qn[p][l] + QK[kp] + QK[kq]
                for r in range(qn[p + 2].shape[0]):
                    if qn[p + 2][r][0] == want[0] and qn[p + 2][r][1] == want[1]:
                        out.append((l, kp, kq, r))
    return out


def onehot_state(sites, p, m):
    """Sites of the one-hot state: T replaced by e_m = [l, k_p, k_{p+1}, r]."""
    l, kp, kq, r = m
    s = list(sites)
    a = np.zeros((sites[p].shape[0], 4, 1))
    a[l, kp, 0] = 1.0
    b = np.zeros((1, 4, sites[p + 1].shape[2]))
    b[0, kq, r] = 1.0
    s[p], s[p + 1] = a, b
    return s


def onehot_pencil(prob, i, p, chi_cap=None, tau_w=1e-13):
    """(index, Hd, Sd, Hc, Sc, t): the blocks of the pencil expanded over the
    one-hot states of state i at sites (p, p+1); index[m] = (l, k_p, k_{p+1},
    r), Hd, Sd [n][n], Hc, Sc [n][M] (column k: state k), t[m] = <varphi_m|phi_i>."""
    chi_cap = prob.chi if chi_cap is None else chi_cap
    bi = prob.mps[i]
    sites, qn = canonical_at(bi.sites, bi.bond_qn, p)
    index = onehot_index(qn, p)
    f = SectorFCI(prob.N, prob.n_alpha, prob.n_beta)
    hi, Li = rotate_integrals(prob.h, prob.L, bi.U)
    g = np.einsum("kpq,krs->pqrs", Li, Li)
    hp = hi - 0.5 * np.einsum("prrq->pq", g)

    def apply_h(V):
        W = f.apply_one_body(hp, V) + prob.e_core * V
        for k in range(Li.shape[0]):
            W = W + 0.5 * f.apply_one_body(Li[k], f.apply_one_body(Li[k], V))
        return W

    V = [f.from_mps(onehot_state(sites, p, m)) for m in index]
    HV = [apply_h(v) for v in V]
    n = len(index)
    Hd = np.array([[np.sum(V[a] * HV[b]) for b in range(n)] for a in range(n)])
    Sd = np.array([[np.sum(V[a] * V[b]) for b in range(n)] for a in range(n)])
    Hc = np.zeros((n, prob.M))
    Sc = np.zeros((n, prob.M))
    for k in range(prob.M):
        if k == i:
            ket = bi.sites
        else:
            bk = prob.mps[k]
            ket, _, _ = rotate_ket(bk.sites, bk.bond_qn, bi.U.T @ bk.U, chi_cap, tau_w)
        vk = f.from_mps(ket)
        Hvk = apply_h(vk)
        for a in range(n):
            Hc[a, k] = np.sum(V[a] * Hvk)
            Sc[a, k] = np.sum(V[a] * vk)
    t = Sc[:, i].copy()
    return index, Hd, Sd, Hc, Sc, t


def expanded_gep(H, S, Hd, Sd, Hc, Sc, i, eps_rel=1e-12):
    """Lowest root of the pencil with state i replaced by its one-hot states
    (eq. exp_gen_eig), and the updated two-site parameters of state i
    (eq. param_upd): t'_m = C'[im] / |C'[i.]|."""
    from .gep import solve_projection
    M = H.shape[0]
    keep = [k for k in range(M) if k != i]
    n = Hd.shape[0]
    Hx = np.zeros((n + M - 1, n + M - 1))
    Sx = np.zeros_like(Hx)
    Hx[:n, :n], Sx[:n, :n] = Hd, Sd
    Hx[:n, n:], Sx[:n, n:] = Hc[:, keep], Sc[:, keep]
    Hx[n:, :n], Sx[n:, :n] = Hc[:, keep].T, Sc[:, keep].T
    Hx[n:, n:] = H[np.ix_(keep, keep)]
    Sx[n:, n:] = S[np.ix_(keep, keep)]
    sol = solve_projection(Hx, Sx, eps_rel)
    c = sol["c"][:n]
    return sol["E"], c / np.linalg.norm(c)
