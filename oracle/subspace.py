"""The subspace pencil for M MPS in rotated orbital bases (arXiv 2404.10223).

MPS j with rotation U_j represents |phi_j> = G(U_j)|Phi_j>, where |Phi_j> is
the MPS read in reference-basis labels and column p of U_j is orbital p of
basis j (eq. tnqe with each MPS in its own basis, Sec. II.B).  Then

  S_ij = <Phi_i| G(U_i^T U_j) |Phi_j>,
  H_ij = <Phi_i| H[h^(i), g^(i)] G(U_i^T U_j) |Phi_j> + e_core S_ij,

with h^(i) = U_i^T h U_i and L^k(i) = U_i^T L^k U_i: rotating the basis is the
same as transforming the Hamiltonian coefficients (Sec. II.F), and the
off-diagonal elements need the rotation network between the two bases
(eq. givens_decomp, Fig. mat_el b).  The method replaces G(U_i^T U_j)|Phi_j>
by the Givens network applied gate by gate to the MPS with SVD truncation to
chi after every gate (the "severe truncations" of Sec. II.B); the ket j is
taken into bra i's basis for i <= j and the result mirrored, since the adjoint
blocks are copies (App. A1).  The generalized eigenproblem (eq. GEE) closes
the step.
"""
import numpy as np

from . import gates, givens, mps as mpsops
from .fock import SectorFCI
from .gep import solve_projection
from .mpo import build_mpo, expectation


def rotate_integrals(h, L, U):
    hi = U.T @ h @ U
    Li = np.einsum("pa,kpq,qb->kab", U, L, U)
    return hi, Li


def rotate_ket(sites, qn, W, chi_cap, tau_w=1e-13, renormalize=False):
    """Givens network for W applied to an MPS with truncation after each gate."""
    sites, qn = mpsops.copy_mps(sites, qn)
    centre = mpsops.left_canonicalize(sites, qn)
    gl, det_sign = givens.plan(W)
    if det_sign < 0:
        mpsops.apply_site_op(sites, len(sites) - 1, gates.parity_gate())
    stats = []
    for a, theta in gl:
        centre = mpsops.move_centre(sites, qn, centre, a)
        stats.append(mpsops.gate_and_truncate(sites, qn, a, gates.g4(theta), chi_cap, tau_w, renormalize))
        centre = a + 1
    return sites, qn, stats


def pair_element(prob, i, j, chi_cap=None, tau_w=1e-13, h_method="auto", mpo_cache=None, return_ket=False,
                 renormalize=False):
    """(H_ij, S_ij, truncation stats[, rotated ket sites]) for one pair i <= j."""
    chi_cap = prob.chi if chi_cap is None else chi_cap
    bi, bj = prob.mps[i], prob.mps[j]
    if i == j:
        ket, kqn, stats = bi.sites, bi.bond_qn, []
    else:
        W = bi.U.T @ bj.U
        ket, kqn, stats = rotate_ket(bj.sites, bj.bond_qn, W, chi_cap, tau_w, renormalize)
    S = mpsops.overlap(bi.sites, ket)
    hi, Li = rotate_integrals(prob.h, prob.L, bi.U)
    if h_method == "auto":
        h_method = "fci" if prob.N <= 12 else "mpo"
    if h_method == "fci":
        f = SectorFCI(prob.N, prob.n_alpha, prob.n_beta)
        H = f.expectation(hi, Li, prob.e_core, f.from_mps(bi.sites), f.from_mps(ket))
    else:
        key = i
        if mpo_cache is not None and key in mpo_cache:
            W_ = mpo_cache[key]
        else:
            W_ = build_mpo(hi, np.einsum("kpq,krs->pqrs", Li, Li))
            if mpo_cache is not None:
                mpo_cache[key] = W_
        H, S2 = expectation(W_, bi.sites, bi.bond_qn, ket, kqn)
        H += prob.e_core * S
    if return_ket:
        return H, S, stats, ket
    return H, S, stats


def subspace(prob, chi_cap=None, tau_w=1e-13, h_method="auto", eps_S=1e-12, renormalize=False):
    """Full pencil, lowest eigenvalue and a report (FP64, CPU)."""
    M = prob.M
    H = np.zeros((M, M))
    S = np.zeros((M, M))
    disc, gaps = np.zeros((M, M)), []
    cache = {}
    for i in range(M):
        for j in range(i, M):
            h, s, st = pair_element(prob, i, j, chi_cap, tau_w, h_method, cache, renormalize=renormalize)
            H[i, j] = H[j, i] = h
            S[i, j] = S[j, i] = s
            disc[i, j] = sum(x["discarded"] for x in st)
            gaps += [x["gap"] for x in st if x["gap"] is not None]
    sol = solve_projection(H, S, eps_S)
    rep = dict(max_discarded_weight_sum=float(disc.max()),
               min_rel_gap=float(min(gaps)) if gaps else None,
               cond_S=sol["cond_S"], kappa1=sol["kappa1"], n_dropped=sol["n_dropped"],
               lam_min=sol["lam_min"])
    return H, S, sol["E"], sol["c"], rep
