"""Matrix-product operator of the Hamiltonian and the left-environment sweep.

The paper evaluates MPS expectation values by contracting an MPO of H with the
bra and ket (Sec. II.A, "matrix product operator"; App. A1 "classical tensor
network contraction" of the diagonal blocks) but builds its MPO with ITensor
and does not describe it.  This module builds one from the operator terms:

H = sum_{ij} t_ij a+_i a_j + sum_{i<j, k<l} V_ijkl a+_i a+_j a_l a_k
(spin-orbitals i = 2p + s, t_ij = h_pq d_st, and V_ijkl = w_ijkl - w_ijlk with
w_ijkl = g_{p_i p_k p_j p_l} d(s_i, s_k) d(s_j, s_l), g in chemists' notation).

Every term is written as a product of single-mode operators sorted by mode
(stable, with the fermionic sign), so a term with ops o_1 .. o_m at sites
x_1 <= .. <= x_m is an operator string.  At bond b (sites < b on the left)
the string's left part selects a channel:

  no op on the left ............ I
  all ops on the left .......... H
  one op (o_1) ................. N1(o_1)        (coefficient not yet applied)
  two ops, b <= N - b .......... N2(o_1, o_2)   (coefficient not yet applied)
  two ops, b >  N - b .......... C2(o_3, o_4)   (coefficient applied: sum over
                                                 all left pairs)
  three ops .................... C3(o_4)        (coefficient applied)

so the two-operator channels count O(min(b, N-b)^2) and the MPO bond
dimension is O(N^2).  The coefficient is applied on the first transition
into C2, C3 or H; every other transition is a fixed operator.  On a site the
local operator of a transition is (product of the ops placed there, in sorted
order) times F^(number of ops placed so far, mod 2), F = diag(1,-1,-1,1): the
Jordan-Wigner string of the ops still to come.

The channel I is kept to the last bond, so the same sweep yields S = <bra|ket>
and H = <bra|H|ket>.
"""
from collections import defaultdict

import numpy as np
import scipy.sparse as sps

# local single-mode operators on the site basis k = n_up + 2 n_dn
_CD_UP = np.zeros((4, 4))
_CD_UP[1, 0] = 1.0       # |0>  -> |up>
_CD_UP[3, 2] = 1.0       # |dn> -> a+_up a+_dn|vac> = |up dn>
_CD_DN = np.zeros((4, 4))
_CD_DN[2, 0] = 1.0       # |0>  -> |dn>
_CD_DN[3, 1] = -1.0      # |up> -> a+_dn a+_up|vac> = -|up dn>
_F = np.diag([1.0, -1.0, -1.0, 1.0])
_LOCAL = {(0, 1): _CD_UP, (1, 1): _CD_DN, (0, 0): _CD_UP.T, (1, 0): _CD_DN.T}   # (spin, dagger)

QK = np.array([[0, 0], [1, 0], [0, 1], [1, 1]])


def _op_qn(op):
    i, dag = op
    d = 1 if dag else -1
    return (d, 0) if i % 2 == 0 else (0, d)


def _sorted_ops(ops):
    """Stable sort by mode index; returns (sign, ops)."""
    ops = list(ops)
    sign = 1.0
    n = len(ops)
    for a in range(n):
        for b in range(n - 1 - a):
            if ops[b][0] > ops[b + 1][0]:
                ops[b], ops[b + 1] = ops[b + 1], ops[b]
                sign = -sign
    return sign, tuple(ops)


def hamiltonian_terms(h, g, tol=0.0):
    """List of (coefficient, ops) with ops in their written order."""
    N = h.shape[0]
    terms = []
    for i in range(2 * N):
        for j in range(2 * N):
            if i % 2 != j % 2:
                continue
            c = h[i // 2, j // 2]
            if abs(c) > tol:
                terms.append((c, ((i, 1), (j, 0))))
    sp = lambda i: i % 2
    site = lambda i: i // 2
    for i in range(2 * N):
        for j in range(i + 1, 2 * N):
            for k in range(2 * N):
                for l in range(k + 1, 2 * N):
                    v = 0.0
                    if sp(i) == sp(k) and sp(j) == sp(l):
                        v += g[site(i), site(k), site(j), site(l)]
                    if sp(i) == sp(l) and sp(j) == sp(k):
                        v -= g[site(i), site(l), site(j), site(k)]
                    if abs(v) > tol:
                        terms.append((v, ((i, 1), (j, 1), (l, 0), (k, 0))))
    return terms


class MPO:
    """Sparse MPO: W[x][(w_in, w_out)] = 4x4 local matrix (bra index first)."""

    def __init__(self, N, terms):
        self.N = N
        half = lambda b: b <= N - b
        chans = [set() for _ in range(N + 1)]
        W = [dict() for _ in range(N)]
        coef_W = [defaultdict(lambda: np.zeros((4, 4))) for _ in range(N)]

        for b in range(N + 1):
            chans[b].add(("I",))
        for b in range(1, N + 1):
            chans[b].add(("H",))

        def channel(ops, j, b):
            m = len(ops)
            if j == 0:
                return ("I",)
            if j == m:
                return ("H",)
            if j == 1:
                return ("N1", ops[0])
            if j == 2:
                return ("N2", ops[0], ops[1]) if half(b) else ("C2", ops[2], ops[3])
            return ("C3", ops[3])

        for c, raw in terms:
            sign, ops = _sorted_ops(raw)
            # a repeated creation or annihilation on one mode is zero
            if any(ops[a] == ops[a + 1] for a in range(len(ops) - 1)):
                continue
            c = c * sign
            sites = [o[0] // 2 for o in ops]
            first, last = sites[0], sites[-1]
            applied = False
            for x in range(first, last + 1):
                j_in = sum(1 for s in sites if s < x)
                j_out = sum(1 for s in sites if s <= x)
                w_in, w_out = channel(ops, j_in, x), channel(ops, j_out, x + 1)
                placed = [o for o in ops if o[0] // 2 == x]
                if not placed and w_in == w_out:
                    continue
                chans[x].add(w_in)
                chans[x + 1].add(w_out)
                loc = np.eye(4)
                for o in placed:
                    loc = loc @ _LOCAL[(o[0] % 2, o[1])]
                if j_out % 2:
                    loc = loc @ _F
                if not applied and w_in[0] in ("I", "N1", "N2") and w_out[0] in ("C2", "C3", "H"):
                    coef_W[x][(w_in, w_out)] += c * loc
                    applied = True
                else:
                    W[x][(w_in, w_out)] = loc
        # pass-through of every channel present on both sides of a site
        for x in range(N):
            for w in chans[x] & chans[x + 1]:
                if w[0] in ("I", "H", "N2", "C2"):
                    W[x][(w, w)] = np.eye(4)
                else:
                    W[x][(w, w)] = _F.copy()
        for x in range(N):
            for key, m in coef_W[x].items():
                assert key not in W[x]
                W[x][key] = m
        self.chans = [sorted(c) for c in chans]
        self.W = W

    def qn(self, w):
        """Particle-number shift (d_alpha, d_beta) = bra sector - ket sector of channel w."""
        if w[0] in ("I", "H"):
            return (0, 0)
        if w[0] in ("N1", "N2"):
            ops = w[1:]
            return tuple(int(v) for v in np.sum([_op_qn(o) for o in ops], axis=0))
        # complementary channels: total of a term is zero, so left = -(right ops)
        ops = w[1:]
        return tuple(int(-v) for v in np.sum([_op_qn(o) for o in ops], axis=0))

    def bond_dims(self):
        return [len(c) for c in self.chans]

    def to_dense(self):
        """Contract to a dense 4^N x 4^N matrix (tiny N only)."""
        N = self.N
        idx = [{w: i for i, w in enumerate(c)} for c in self.chans]
        # T[w, bra, ket] accumulated left to right
        T = np.zeros((len(self.chans[0]), 1, 1))
        T[idx[0][("I",)], 0, 0] = 1.0
        for x in range(N):
            D1 = len(self.chans[x + 1])
            nb = T.shape[1]
            nT = np.zeros((D1, nb * 4, nb * 4))
            for (wi, wo), m in self.W[x].items():
                a, b = idx[x][wi], idx[x + 1][wo]
                nT[b] += np.kron(T[a], m)
            T = nT
        return T[idx[N][("H",)]], T[idx[N][("I",)]]


def build_mpo(h, g):
    return MPO(h.shape[0], hamiltonian_terms(h, g))


# --------------------------------------------------------------- environment sweep
def _sector_index(q):
    """dict sector -> index array, for a [n, 2] label array."""
    out = defaultdict(list)
    for i, s in enumerate(map(tuple, q.tolist())):
        out[s].append(i)
    return {s: np.array(v) for s, v in out.items()}


def expectation(mpo, bra, bra_qn, ket, ket_qn):
    """(H, S) = (<bra|H|ket>, <bra|ket>) by the block-sparse left sweep.

    The environment at bond b is kept per channel class (shift delta = bra
    sector - ket sector) and per ket sector s as an array
    [channels of the class, dim bra(s + delta), dim ket(s)].
    """
    N = mpo.N
    cls = []
    for b in range(N + 1):
        d = defaultdict(list)
        for w in mpo.chans[b]:
            d[mpo.qn(w)].append(w)
        cls.append({k: (v, {w: i for i, w in enumerate(v)}) for k, v in d.items()})
    assert cls[0][(0, 0)][0] == [("I",)]
    env = {(0, 0): {(0, 0): np.ones((1, 1, 1))}}
    for x in range(N):
        A, B = bra[x], ket[x]
        bl, br = _sector_index(bra_qn[x]), _sector_index(bra_qn[x + 1])
        kl, kr = _sector_index(ket_qn[x]), _sector_index(ket_qn[x + 1])
        # 1) X = L . ket site, per (class, ket sector s, k)
        X = defaultdict(list)
        for dl, blocks in env.items():
            for s, Lb in blocks.items():
                for k in range(4):
                    sk = (s[0] + QK[k, 0], s[1] + QK[k, 1])
                    if sk not in kr:
                        continue
                    X[(dl, k)].append((sk, Lb @ B[np.ix_(kl[s], [k], kr[sk])][:, 0, :]))
        # 2) channel mix with the MPO, grouped by (class in, class out, k', k)
        groups = defaultdict(list)
        for (wi, wo), m in mpo.W[x].items():
            di, do = mpo.qn(wi), mpo.qn(wo)
            ii = cls[x][di][1][wi]
            oo = cls[x + 1][do][1][wo]
            for kp in range(4):
                for k in range(4):
                    if m[kp, k] != 0.0:
                        groups[(di, do, kp, k)].append((oo, ii, m[kp, k]))
        Y = {}
        for (di, do, kp, k), ent in groups.items():
            if (di, k) not in X:
                continue
            shape = (len(cls[x + 1][do][0]), len(cls[x][di][0]))
            ent = np.array(ent)
            C = sps.csr_matrix((ent[:, 2], (ent[:, 0].astype(int), ent[:, 1].astype(int))), shape=shape)
            if C.nnz > 0.1 * shape[0] * shape[1]:
                C = C.toarray()
            for sk, Xb in X[(di, k)]:
                key = (do, sk, kp)
                nw, da, db = Xb.shape
                contrib = np.asarray(C @ Xb.reshape(nw, da * db)).reshape(shape[0], da, db)
                Y[key] = Y[key] + contrib if key in Y else contrib
        # 3) contract the bra site: new env[class out][ket sector sk]
        new = defaultdict(dict)
        for (do, sk, kp), Yb in Y.items():
            sa = (sk[0] + do[0] - QK[kp, 0], sk[1] + do[1] - QK[kp, 1])    # bra sector at bond x
            sb = (sk[0] + do[0], sk[1] + do[1])                           # bra sector at bond x+1
            if sa not in bl or sb not in br:
                continue
            Ab = A[np.ix_(bl[sa], [kp], br[sb])][:, 0, :]
            t = np.einsum("wab,ac->wcb", Yb, Ab)
            if sk in new[do]:
                new[do][sk] = new[do][sk] + t
            else:
                new[do][sk] = t
        env = new
    ch, chi = cls[N][(0, 0)]
    (sN,) = map(tuple, np.unique(ket_qn[N], axis=0).tolist())
    blk = env[(0, 0)][sN]
    return float(blk[chi[("H",)], 0, 0]), float(blk[chi[("I",)], 0, 0])


# ------------------------------------------------------ plain contraction (cross-check)
def expectation_plain(mpo, bra, ket):
    """(H, S) by the plainest left sweep: one dense environment E[a', w, a]
    over the full bond and channel ranges, no quantum-number or channel-class
    grouping.  Per site x, with the MPO read as one matrix C[k', k] over
    (output channel, input channel) for each pair of local states:

        T[a', w, k, b]  = sum_a E[a', w, a] ket[a, k, b]
        Y[a', w', k', b] = sum_{w, k} C[k', k][w', w] T[a', w, k, b]
        E'[b', w', b]   = sum_{a', k'} bra[a', k', b'] Y[a', w', k', b]

    It touches every zero the block-sparse sweep skips, so it is slow (minutes
    at N = 24, chi = 256); it exists to cross-check `expectation` on the full-
    size workload, where no sector FCI is possible.
    """
    N = mpo.N
    idx = [{w: i for i, w in enumerate(c)} for c in mpo.chans]
    E = np.zeros((1, len(mpo.chans[0]), 1))
    E[0, idx[0][("I",)], 0] = 1.0
    for x in range(N):
        A, B = bra[x], ket[x]
        dbl, dkl = A.shape[0], B.shape[0]
        dbr, dkr = A.shape[2], B.shape[2]
        Din, Dout = len(mpo.chans[x]), len(mpo.chans[x + 1])
        C = np.zeros((4, 4, Dout, Din))
        for (wi, wo), m in mpo.W[x].items():
            C[:, :, idx[x + 1][wo], idx[x][wi]] += m
        # T[k][w, a', b]
        T = np.tensordot(E, B, axes=([2], [0]))               # [a', w, k, b]
        T = np.ascontiguousarray(T.transpose(2, 1, 0, 3))     # [k, w, a', b]
        Y = np.zeros((4, Dout, dbl * dkr))
        for kp in range(4):
            for k in range(4):
                if np.any(C[kp, k]):
                    Y[kp] += C[kp, k] @ T[k].reshape(Din, dbl * dkr)
        del T
        Y = Y.reshape(4, Dout, dbl, dkr)                       # [k', w', a', b]
        En = np.zeros((dbr, Dout, dkr))
        for kp in range(4):
            En += np.tensordot(A[:, kp, :], Y[kp], axes=([0], [1]))   # [b', w', b]
        E = En
    return float(E[0, idx[N][("H",)], 0]), float(E[0, idx[N][("I",)], 0])
