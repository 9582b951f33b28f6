"""Seeded synthetic inputs for the subspace-matrix problem.

This module only draws random inputs of the shape of the paper's workloads
(H2O / octahedral H6 in STO-3G, Sec. III "Numerical benchmarking"); it holds
none of the method's arithmetic.  Both the FP64 CPU oracle and the GPU library
consume what it returns, and nothing else is shared between them.

Recipe (the paper's molecular integrals are not available; these stand in):

* one-electron integrals: h_pp linearly spaced on [-2, 0.5], off-diagonal
  h_pq = x / (1 + |p - q|), x ~ N(0, 0.01) (variance);
* two-electron integrals in Cholesky form g_pqrs = sum_k L^k_pq L^k_rs with K
  symmetric L^k whose upper triangles are N(0, 0.05) (variance);
* orbital rotations U = expm(A), A antisymmetric with A_pq ~ N(0, 0.3^2);
* MPS in the (N_alpha, N_beta) sector with U(1)xU(1) block structure, bond
  slots spread over quantum-number sectors in proportion to the exact sector
  dimension, N(0, 1) entries on the allowed blocks, then brought to
  left-orthonormal form and normalised so every tensor has O(1) entries.

Sub-seeds: integrals rng([base, 0]); rotation j rng([base, 1, j]);
MPS j rng([base, 2, j]); batched-subspace shape list rng([base, 3]);
subspace s of a batch uses base (base, 4, s).
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field
from math import comb

import numpy as np
import scipy.linalg

# local state k = n_up + 2 n_dn  ->  (n_up, n_dn)
QK = ((0, 0), (1, 0), (0, 1), (1, 1))


@dataclass
class MPS:
    """Real MPS in its own orbital basis.

    sites[p] has shape [bond_dim[p], 4, bond_dim[p+1]]; bond_qn[b] is an int
    array [bond_dim[b], 2] holding (n_alpha, n_beta) of sites 1..b for every
    index of bond b, sorted by sector.  U[:, p] is orbital p of this MPS in the
    reference basis.
    """
    sites: list
    bond_qn: list
    U: np.ndarray

    @property
    def bond_dim(self):
        return [q.shape[0] for q in self.bond_qn]


@dataclass
class Problem:
    N: int
    n_alpha: int
    n_beta: int
    h: np.ndarray            # [N, N]
    L: np.ndarray            # [K, N, N]
    e_core: float
    chi: int
    mps: list = field(default_factory=list)
    name: str = ""

    @property
    def M(self):
        return len(self.mps)

    def g(self):
        """Dense chemists'-notation two-electron tensor (pq|rs)."""
        return np.einsum("kpq,krs->pqrs", self.L, self.L)


def _rng(*key):
    return np.random.default_rng(list(key))


def make_integrals(N, K, base):
    r = _rng(*base, 0)
    h = np.zeros((N, N))
    h[np.arange(N), np.arange(N)] = np.linspace(-2.0, 0.5, N)
    for p in range(N):
        for q in range(p + 1, N):
            x = r.normal(0.0, 0.1)
            h[p, q] = h[q, p] = x / (1.0 + (q - p))
    L = np.zeros((K, N, N))
    iu = np.triu_indices(N)
    for k in range(K):
        v = r.normal(0.0, np.sqrt(0.05), size=len(iu[0]))
        L[k][iu] = v
        L[k] = L[k] + np.triu(L[k], 1).T
    return h, L


def make_rotation(N, base, j):
    r = _rng(*base, 1, j)
    A = np.zeros((N, N))
    for p in range(N):
        for q in range(p + 1, N):
            a = r.normal(0.0, 0.3)
            A[p, q] = a
            A[q, p] = -a
    U = scipy.linalg.expm(A)
    U = U @ (1.5 * np.eye(N) - 0.5 * (U.T @ U))   # one Newton-Schulz polish
    return U


def sector_slots(N, na, nb, chi):
    """Per-bond list of (sector (a, b), slot count), sectors sorted."""
    bonds = []
    for b in range(N + 1):
        secs = []
        for a in range(max(0, na - (N - b)), min(b, na) + 1):
            for be in range(max(0, nb - (N - b)), min(b, nb) + 1):
                left = comb(b, a) * comb(b, be)
                right = comb(N - b, na - a) * comb(N - b, nb - be)
                secs.append(((a, be), min(left, right)))
        tot = sum(D for _, D in secs)
        chat = min(chi, tot)
        m = {s: min(D, (chat * D) // tot) for s, D in secs}
        rem = chat - sum(m.values())
        order = sorted(secs, key=lambda t: (-t[1], t[0]))
        while rem > 0:
            moved = False
            for s, D in order:
                if rem == 0:
                    break
                if m[s] < D:
                    m[s] += 1
                    rem -= 1
                    moved = True
            if not moved:
                break
        bonds.append({s: m[s] for s, _ in secs})
    # nested feasibility: a sector cannot hold more slots than its neighbours feed
    for b in range(1, N + 1):
        for s in bonds[b]:
            feed = sum(bonds[b - 1].get((s[0] - qa, s[1] - qb), 0) for qa, qb in QK)
            bonds[b][s] = min(bonds[b][s], feed)
    for b in range(N - 1, -1, -1):
        for s in bonds[b]:
            feed = sum(bonds[b + 1].get((s[0] + qa, s[1] + qb), 0) for qa, qb in QK)
            bonds[b][s] = min(bonds[b][s], feed)
    return [[(s, d) for s, d in sorted(bd.items()) if d > 0] for bd in bonds]


def _bond_labels(slots):
    lab = []
    for (a, b), d in slots:
        lab += [(a, b)] * d
    return np.array(lab, dtype=np.int64).reshape(-1, 2)


def make_mps(N, na, nb, chi, base, j):
    """Random sector-conserving MPS, left-orthonormal and normalised."""
    r = _rng(*base, 2, j)
    slots = sector_slots(N, na, nb, chi)
    qn = [_bond_labels(s) for s in slots]
    sites = []
    for p in range(N):
        ql, qr = qn[p], qn[p + 1]
        A = np.zeros((len(ql), 4, len(qr)))
        for k, (ua, ub) in enumerate(QK):
            mask = (ql[:, None, 0] + ua == qr[None, :, 0]) & (ql[:, None, 1] + ub == qr[None, :, 1])
            A[:, k, :] = np.where(mask, r.normal(0.0, 1.0, size=mask.shape), 0.0)
        sites.append(A)
    # left-orthonormal form, one right-sector block at a time
    for p in range(N - 1):
        A = sites[p]
        dl, _, dr = A.shape
        ql, qr = qn[p], qn[p + 1]
        M = A.reshape(dl * 4, dr)
        rowq = (ql[:, None, :] + np.array(QK)[None, :, :]).reshape(-1, 2)
        Q = np.zeros_like(M)
        R = np.zeros((dr, dr))
        for s in sorted(set(map(tuple, qr))):
            cols = np.where((qr[:, 0] == s[0]) & (qr[:, 1] == s[1]))[0]
            rows = np.where((rowq[:, 0] == s[0]) & (rowq[:, 1] == s[1]))[0]
            q, rr = np.linalg.qr(M[np.ix_(rows, cols)])
            Q[np.ix_(rows, cols)] = q
            R[np.ix_(cols, cols)] = rr
        sites[p] = Q.reshape(dl, 4, dr)
        sites[p + 1] = np.einsum("ab,bkc->akc", R, sites[p + 1])
    sites[-1] /= np.linalg.norm(sites[-1])
    return sites, qn


# (N, n_alpha, n_beta, chi, M, K, seed base)
CONFIGS = {
    1: dict(N=4, na=2, nb=2, chi=4, M=2, K=8, base=1001),
    2: dict(N=7, na=5, nb=5, chi=16, M=4, K=12, base=1002),
    3: dict(N=12, na=6, nb=6, chi=64, M=8, K=12, base=1003),
    5: dict(N=24, na=12, nb=12, chi=256, M=16, K=24, base=1005),
}


def make_permutation(N, base, j):
    """An orbital permutation matrix U[p, perm[p]] = 1 (a network of fermionic
    swaps only: the TNQE-F variant)."""
    perm = _rng(*base, 5, j).permutation(N)
    U = np.zeros((N, N))
    U[np.arange(N), perm] = 1.0
    return U


ROTATIONS = ("expm", "perm", "identity")


def make_problem(N, na, nb, chi, M, K, base, name="", rotations="expm"):
    """rotations: "expm" (random orbital rotations, TNQE), "perm" (orbital
    permutations: fermionic-swap networks, TNQE-F) or "identity" (no
    rotations: a linear combination of MPS, LC-MPS)."""
    assert rotations in ROTATIONS
    base = tuple(base) if isinstance(base, (tuple, list)) else (base,)
    h, L = make_integrals(N, K, base)
    mps = []
    for j in range(M):
        if rotations == "expm":
            U = make_rotation(N, base, j)
        elif rotations == "perm":
            U = make_permutation(N, base, j)
        else:
            U = np.eye(N)
        sites, qn = make_mps(N, na, nb, chi, base, j)
        mps.append(MPS(sites=sites, bond_qn=qn, U=U))
    return Problem(N=N, n_alpha=na, n_beta=nb, h=h, L=L, e_core=0.0, chi=chi, mps=mps, name=name)


def make_config(k, rotations="expm"):
    """Workload k: 1 (N=4), 2 (N=7), 3 (N=12), 5 (N=24); rotations as in
    make_problem (the integrals and MPS do not depend on it)."""
    c = CONFIGS[k]
    name = f"config{k}" if rotations == "expm" else f"config{k}_{rotations}"
    return make_problem(c["N"], c["na"], c["nb"], c["chi"], c["M"], c["K"], c["base"], name=name,
                        rotations=rotations)


def batch_shapes(base=1004, n_sub=64):
    """Shapes of the batched workload: N ~ U{8..16}, chi ~ U{16,32,64,128}, M ~ U{2..8}."""
    r = _rng(base, 3)
    out = []
    for _ in range(n_sub):
        N = int(r.integers(8, 17))
        chi = int(r.choice([16, 32, 64, 128]))
        M = int(r.integers(2, 9))
        out.append((N, chi, M))
    return out


def make_batch(base=1004, n_sub=64):
    probs = []
    for s, (N, chi, M) in enumerate(batch_shapes(base, n_sub)):
        na, nb = (N + 1) // 2, N // 2
        probs.append(make_problem(N, na, nb, chi, M, N, (base, 4, s), name=f"batch{s}"))
    return probs


def problem_digest(p: Problem) -> str:
    """SHA-256 over every array of a problem (NumPy stream stability guard)."""
    hsh = hashlib.sha256()
    for a in [p.h, p.L] + [x for m in p.mps for x in (m.U, *m.sites, *m.bond_qn)]:
        hsh.update(np.ascontiguousarray(a).tobytes())
    return hsh.hexdigest()
