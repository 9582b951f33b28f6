"""One step of the generalized sweep (Alg. A.1 of arXiv 2404.10223) at the
two-site position (p, p+1) for one expanded state i -- test infrastructure
only, like the whole package.

The step, in the algorithm's order, with jset = {i} (App. A1: expanding a
chosen reference state) and no single-site mitigation repetitions (App. A4):

1. State i in canonical form centred on (p, p+1), its one-hot states and the
   blocks of the expanded pencil (oracle.onehot, eq. oht_exp, eq. subs_exp).
   The other states enter unexpanded, each with its own row of the current
   pencil (H, S).
2. Discard of linearly dependent columns (Sec. V, regulating the subspace
   condition number; App. A2).  Columns are taken in the combined order of
   eq. subs_exp (states k < i, the one-hot states of i, states k > i).
   Column c is dropped when its squared distance from the span of the kept
   earlier columns, S'_cc - s^T (S_kept)^+ s, falls below tol_ld S'_cc
   (pseudo-inverse cut at sqrt(eps) ||S_kept||_2, as the paper uses).
3. The projection-thresholded eigenproblem of the kept columns
   (eq. exp_gen_eig): lowest root E1' and its vector C'.
4. Parameter update (eq. param_upd): t'_m = C'[i m] / ||C'[i .]||, with the
   sign for which sum_m t'_m t_m >= 0 (t_m: the current parameters).
5. Orbital rotation of the bond (App. A3): none; the FSWAP f4, accepted when
   it lowers the truncation error xi = 1 - sum_{l <= chi} sigma_l^2; or the
   Givens gate g4(theta) at theta_opt = argmin xi(theta), found on a grid of
   n_grid angles over [-pi/2, pi/2) (xi has period pi) refined by n_golden
   golden-section steps around the best grid point.  "Lowers" means by more
   than xi_tol (1e-12): xi is a difference of order-one sums, and below that
   a rotation would be chosen by rounding alone.
6. Truncation of the rotated two-site tensor with the rule of the gates
   (App. A1): A_p = U (left-orthonormal), A_{p+1} = Sigma V; centre at p+1.
7. Merge of the rotation into the orbital basis of state i: applying g4(theta)
   = G(R_p(theta)) to the sites is compensated by U_i <- U_i R_p(theta)^T
   (FSWAP: f4 = G(P_swap), columns p and p+1 of U_i exchanged), so that the
   state is the same before the truncation.
8. Acceptance (Alg. A.1): E1' < E_old + e_tol, E_old being the lowest root of
   the current pencil.
"""
import numpy as np

from . import gates
from . import mps as mpsops
from .gep import solve_projection
from .givens import rot
from .onehot import canonical_at, onehot_pencil

QK = mpsops.QK
ROTATIONS = ("none", "fswap", "givens")


def combined_order(M, i, n):
    """Positions of the rows of the expanded pencil: ('state', k) for k != i
    and ('onehot', m) for the n one-hot states of i, in the order of
    eq. subs_exp."""
    return [("state", k) for k in range(i)] + [("onehot", m) for m in range(n)] + \
           [("state", k) for k in range(i + 1, M)]


def expanded_pencil(H, S, Hd, Sd, Hc, Sc, i):
    """(H', S') in the combined order, and the positions of the one-hot rows."""
    M, n = H.shape[0], Hd.shape[0]
    order = combined_order(M, i, n)
    D = len(order)
    Hx, Sx = np.zeros((D, D)), np.zeros((D, D))
    for a, (ta, xa) in enumerate(order):
        for b, (tb, xb) in enumerate(order):
            if ta == "state" and tb == "state":
                Hx[a, b], Sx[a, b] = H[xa, xb], S[xa, xb]
            elif ta == "onehot" and tb == "onehot":
                Hx[a, b], Sx[a, b] = Hd[xa, xb], Sd[xa, xb]
            elif ta == "onehot":
                Hx[a, b], Sx[a, b] = Hc[xa, xb], Sc[xa, xb]
            else:
                Hx[a, b], Sx[a, b] = Hc[xb, xa], Sc[xb, xa]
    pos = np.array([a for a, (t, _) in enumerate(order) if t == "onehot"])
    return Hx, Sx, pos


def discard_dependent(S, tol_ld):
    """Keep mask of the columns of S, taken in order: column c is dropped when
    S_cc - s^T pinv(S_kept) s < tol_ld S_cc, s = S[kept, c]."""
    D = S.shape[0]
    keep = np.zeros(D, dtype=bool)
    kept = []
    for c in range(D):
        if kept:
            Sk = S[np.ix_(kept, kept)]
            s = S[kept, c]
            rc = np.sqrt(np.finfo(float).eps) * np.linalg.norm(Sk, 2)
            proj = s @ np.linalg.pinv(Sk, rcond=rc / np.linalg.norm(Sk, 2), hermitian=True) @ s
        else:
            proj = 0.0
        if S[c, c] - proj >= tol_ld * S[c, c]:
            keep[c] = True
            kept.append(c)
    return keep


def two_site_blocks(T4, qn_p, qn_p2):
    """The quantum-number blocks of T4 [dl, 4, 4, dr] as a matrix over
    (l, k_p) x (k_{p+1}, r): list of (sector, rows, cols)."""
    dl, dr = T4.shape[0], T4.shape[3]
    rowq = (qn_p[:, None, :] + QK[None, :, :]).reshape(-1, 2)
    colq = (qn_p2[None, :, :] - QK[:, None, :]).reshape(-1, 2)
    out = []
    for s in mpsops._sectors(rowq):
        rows = mpsops._where(rowq, s)
        cols = mpsops._where(colq, s)
        if len(cols):
            out.append((s, rows, cols))
    return out


def xi(T4, qn_p, qn_p2, chi):
    """Truncation error 1 - sum of the chi largest squared singular values of
    the two-site matrix (App. A3), from the singular values of its blocks."""
    Tm = T4.reshape(T4.shape[0] * 4, 4 * T4.shape[3])
    sv = [np.linalg.svd(Tm[np.ix_(r, c)], compute_uv=False) for _, r, c in two_site_blocks(T4, qn_p, qn_p2)]
    allsv = np.sort(np.concatenate(sv))[::-1] if sv else np.zeros(0)
    return 1.0 - float(np.sum(allsv[:chi] ** 2))


def apply_gate(T4, G16):
    """T4 with a 16 x 16 gate on (k_p, k_{p+1})."""
    dl, dr = T4.shape[0], T4.shape[3]
    return np.einsum("xy,ayb->axb", G16, T4.reshape(dl, 16, dr)).reshape(dl, 4, 4, dr)


def theta_grid(n_grid):
    return [(q - n_grid // 2) * (np.pi / n_grid) for q in range(n_grid)]


def optimise_theta(T4, qn_p, qn_p2, chi, n_grid=36, n_golden=40, xi_tol=1e-12):
    """theta_opt = argmin xi(theta) (eq. theta_opt): the best of n_grid angles
    over [-pi/2, pi/2), then n_golden golden-section steps on the bracket of
    one grid spacing either side of it.  Returns (theta_opt, xi(theta_opt),
    xi(0)); theta_opt is 0 unless it lowers xi below xi(0) - xi_tol."""
    f = lambda th: xi(apply_gate(T4, gates.g4(th)), qn_p, qn_p2, chi)
    grid = theta_grid(n_grid)
    vals = [f(th) for th in grid]
    qb = int(np.argmin(vals))
    xi0 = vals[n_grid // 2]
    h = np.pi / n_grid
    a, b = grid[qb] - h, grid[qb] + h
    g = (np.sqrt(5.0) - 1.0) / 2.0
    x1, x2 = b - g * (b - a), a + g * (b - a)
    f1, f2 = f(x1), f(x2)
    for _ in range(n_golden):
        if f1 <= f2:
            b, x2, f2 = x2, x1, f1
            x1 = b - g * (b - a)
            f1 = f(x1)
        else:
            a, x1, f1 = x1, x2, f2
            x2 = a + g * (b - a)
            f2 = f(x2)
    th, fv = (x1, f1) if f1 <= f2 else (x2, f2)
    if vals[qb] < fv:
        th, fv = grid[qb], vals[qb]
    if not fv < xi0 - xi_tol:
        th, fv = 0.0, xi0
    return float(th), float(fv), float(xi0)


def truncate_two_site(T4, qn_p, qn_p2, chi_cap, tau_w):
    """Split T4 by truncated SVD per block with the rule of the gates
    (mps.select_kept): (A_p, A_{p+1}, labels of the new bond, stats).  The new
    bond is sorted by sector, and inside a sector by decreasing value."""
    dl, dr = T4.shape[0], T4.shape[3]
    Tm = T4.reshape(dl * 4, 4 * dr)
    blocks = []
    for s, rows, cols in two_site_blocks(T4, qn_p, qn_p2):
        u, sv, _ = np.linalg.svd(Tm[np.ix_(rows, cols)], full_matrices=False)
        blocks.append((s, rows, u, sv))
    allsv = np.concatenate([b[3] for b in blocks]) if blocks else np.zeros(0)
    kept_mask, keep, nnz, gap, discarded, total = mpsops.select_kept(allsv, chi_cap, tau_w)
    newq, cols_u = [], []
    o = 0
    for s, rows, u, sv in blocks:
        k = int(kept_mask[o:o + len(sv)].sum())
        assert kept_mask[o:o + k].all()
        o += len(sv)
        if k:
            newq += [s] * k
            cols_u.append((rows, u[:, :k]))
    U = np.zeros((dl * 4, len(newq)))
    c = 0
    for rows, uk in cols_u:
        U[rows, c:c + uk.shape[1]] = uk
        c += uk.shape[1]
    Ap = U.reshape(dl, 4, len(newq))
    Aq = (U.T @ Tm).reshape(len(newq), 4, dr)
    return Ap, Aq, np.array(newq, dtype=np.int64).reshape(-1, 2), dict(
        kept=keep, nonzero=nnz, gap=gap, discarded=discarded, total=total)


def finish(T4, sites, qn, U, p, rotation, theta, chi_cap, tau_w):
    """Steps 5 (with a given decision) to 7: the rotated, truncated two-site
    tensor put into the canonical MPS centred on (p, p+1), and the merged
    orbital basis.  rotation 'fswap' with theta != 0 means accepted."""
    U = U.copy()
    if rotation == "givens" and theta != 0.0:
        T4 = apply_gate(T4, gates.g4(theta))
        U = U @ rot(U.shape[0], p, theta).T
    elif rotation == "fswap" and theta != 0.0:
        T4 = apply_gate(T4, gates.f4())
        U[:, [p, p + 1]] = U[:, [p + 1, p]]
    Ap, Aq, newq, st = truncate_two_site(T4, qn[p], qn[p + 2], chi_cap, tau_w)
    s2, q2 = list(sites), list(qn)
    s2[p], s2[p + 1] = Ap, Aq
    q2[p + 1] = newq
    return s2, q2, U, T4, st


def solve_expanded(H, S, Hd, Sd, Hc, Sc, i, t_cur, tol_ld, eps_S):
    """Steps 2-4 on an expanded pencil whose state-i block is spanned by an
    orthonormal set (Hd, Sd, Hc, Sc as in oracle.onehot): the discard, the
    lowest root and the normalised, signed coefficients of that set."""
    Hx, Sx, pos = expanded_pencil(H, S, Hd, Sd, Hc, Sc, i)
    keep = discard_dependent(Sx, tol_ld)
    kidx = np.nonzero(keep)[0]
    sol = solve_projection(Hx[np.ix_(kidx, kidx)], Sx[np.ix_(kidx, kidx)], eps_S)
    c = np.zeros(len(keep))
    c[kidx] = sol["c"]
    tn = c[pos]
    nrm = np.linalg.norm(tn)
    tn = tn / nrm if nrm > 0.0 else tn
    ov = float(tn @ t_cur)
    if ov < 0.0 or (ov == 0.0 and tn[np.argmax(np.abs(tn))] < 0.0):
        tn = -tn
    return sol, keep, pos, tn


def onehot_gate_matrix(index, G16):
    """[G]_{m'm}: the new one-hot state m (after the gate G16 on the sites was
    merged into the orbital basis) in the old one-hot basis, i.e. the
    coefficient G16[(k_p, k_{p+1})_m, (k_p, k_{p+1})_m'] for equal (l, r)
    (App. A4: the rotation represented in the one-hot basis)."""
    n = len(index)
    at = {e: m for m, e in enumerate(index)}
    G = np.zeros((n, n))
    for m, (l, kp, kq, r) in enumerate(index):
        for x in range(16):
            m2 = at.get((l, x >> 2, x & 3, r))
            if m2 is not None:
                G[m2, m] = G16[kp * 4 + kq, x]
    return G


def single_site_index(qn_l, qn_r):
    """One-hot entries (a, k, b) of a single-site tensor [dl, 4, dr] that
    conserve the particle numbers, row-major."""
    out = []
    for a in range(qn_l.shape[0]):
        for k in range(4):
            want = qn_l[a] + QK[k]
            for b in range(qn_r.shape[0]):
                if qn_r[b][0] == want[0] and qn_r[b][1] == want[1]:
                    out.append((a, k, b))
    return out


def _positive_split(A, qn_l, qn_r, left):
    """Exact QR (left=True: A[(a,k), b] = Q R with Q over rows (a, k)) or LQ
    (A[a, (k,b)] = L Q) of a single-site tensor per sector, non-negative
    triangular diagonal, bond kept as is.  Returns (orthonormal factor as a
    site tensor, triangle)."""
    dl, _, dr = A.shape
    if left:
        rowq = (qn_l[:, None, :] + QK[None, :, :]).reshape(-1, 2)
        M = A.reshape(dl * 4, dr)
        Q = np.zeros_like(M)
        R = np.zeros((dr, dr))
        for s in mpsops._sectors(qn_r):
            cols = mpsops._where(qn_r, s)
            rows = mpsops._where(rowq, s)
            q, r = mpsops._positive_qr(M[np.ix_(rows, cols)])
            Q[np.ix_(rows, cols)] = q
            R[np.ix_(cols, cols)] = r
        return Q.reshape(dl, 4, dr), R
    colq = (qn_r[None, :, :] - QK[:, None, :]).reshape(-1, 2)
    M = A.reshape(dl, 4 * dr)
    Q = np.zeros_like(M)
    L = np.zeros((dl, dl))
    for s in mpsops._sectors(qn_l):
        rows = mpsops._where(qn_l, s)
        cols = mpsops._where(colq, s)
        q, r = mpsops._positive_qr(M[np.ix_(rows, cols)].T)
        Q[np.ix_(rows, cols)] = q.T
        L[np.ix_(rows, rows)] = r.T
    return Q.reshape(dl, 4, dr), L


def mitigate(prob, H, S, i, p, index, Hd, Sd, Hc, Sc, G16, Ap, Aq, qn, newq, nreps, tol_ld, eps_S):
    """App. A4: the two-site pencil moved to the rotated basis
    (H^[ii] -> G^T H^[ii] G, H^[ik] -> G^T H^[ik]), then nreps rounds of
    single-site expansions at p and p+1.  For site p the two-site state is
    (U Sigma) V with V right-orthonormal; the single-site one-hot states times
    V map to the two-site one-hot states by the isometry T[m1, n] =
    V[b, k_{p+1}, r] where (l, k_p) agree, and the pencil becomes T H T^T
    (and T H^[ik] for the columns); the root updates U Sigma.  For site p+1
    the left site is made orthonormal by an exact QR and the isometry is
    T[m2, n] = Q[l, k_p, b] where (k_{p+1}, r) agree.  Returns the final
    (A_p, A_{p+1}) (centre at p+1), the last root and the discard counts."""
    Gm = onehot_gate_matrix(index, G16)
    Hd2, Sd2 = Gm.T @ Hd @ Gm, Gm.T @ Sd @ Gm
    Hc2, Sc2 = Gm.T @ Hc, Gm.T @ Sc
    at = {e: m for m, e in enumerate(index)}
    n = len(index)
    qp, qq = qn[p], qn[p + 2]
    last = None
    for _ in range(nreps):
        for site in (p, p + 1):
            if site == p:
                # site p+1 right-orthonormal: A_{p+1} = L Q
                V, Lm = _positive_split(Aq, newq, qq, left=False)
                T1 = np.einsum("akb,bc->akc", Ap, Lm)
                sidx = single_site_index(qp, newq)
                Tiso = np.zeros((len(sidx), n))
                for m1, (l, kp, b) in enumerate(sidx):
                    for kq in range(4):
                        for r in range(qq.shape[0]):
                            m2 = at.get((l, kp, kq, r))
                            if m2 is not None:
                                Tiso[m1, m2] = V[b, kq, r]
            else:
                # site p left-orthonormal: A_p = Q R
                Q, Rm = _positive_split(Ap, qp, newq, left=True)
                T1 = np.einsum("ab,bkc->akc", Rm, Aq)
                sidx = single_site_index(newq, qq)
                Tiso = np.zeros((len(sidx), n))
                for m1, (b, kq, r) in enumerate(sidx):
                    for l in range(qp.shape[0]):
                        for kp in range(4):
                            m2 = at.get((l, kp, kq, r))
                            if m2 is not None:
                                Tiso[m1, m2] = Q[l, kp, b]
            t_cur = np.array([T1[e] for e in sidx])
            sol, keep, pos, tn = solve_expanded(H, S, Tiso @ Hd2 @ Tiso.T, Tiso @ Sd2 @ Tiso.T, Tiso @ Hc2,
                                                 Tiso @ Sc2, i, t_cur, tol_ld, eps_S)
            T1n = np.zeros_like(T1)
            for m1, e in enumerate(sidx):
                T1n[e] = tn[m1]
            if site == p:
                Ap, Aq = T1n, V
            else:
                Ap, Aq = Q, T1n
            last = (sol, keep)
    return Ap, Aq, last


def sweep_step(prob, H, S, i, p, rotation="none", tol_ld=1e-3, eps_S=1e-12, e_tol=0.0, chi_cap=None,
               tau_w=1e-13, n_grid=36, n_golden=40, xi_tol=1e-12, nreps=0, theta_given=None):
    """Steps 1-8 above (with nreps > 0, the single-site mitigation of App. A4
    after step 7; E_new is then its last root).  H, S: the current pencil.
    theta_given: a Givens angle to use instead of the search (checks of what
    follows the search, at another implementation's angle).  Returns a dict."""
    assert rotation in ROTATIONS
    chi_cap = prob.chi if chi_cap is None else chi_cap
    M = prob.M
    bi = prob.mps[i]
    sites, qn = canonical_at(bi.sites, bi.bond_qn, p)
    index, Hd, Sd, Hc, Sc, t = onehot_pencil(prob, i, p, chi_cap, tau_w)
    n = len(index)
    sol, keep, pos, tn = solve_expanded(H, S, Hd, Sd, Hc, Sc, i, t, tol_ld, eps_S)
    dl, dr = sites[p].shape[0], sites[p + 1].shape[2]
    T4 = np.zeros((dl, 4, 4, dr))
    for m, (l, kp, kq, r) in enumerate(index):
        T4[l, kp, kq, r] = tn[m]
    xi_none = xi(T4, qn[p], qn[p + 2], chi_cap)
    theta, xi_rot = 0.0, xi_none
    if rotation == "fswap":
        xs = xi(apply_gate(T4, gates.f4()), qn[p], qn[p + 2], chi_cap)
        if xs < xi_none - xi_tol:
            theta, xi_rot = np.pi / 2, xs
    elif rotation == "givens" and theta_given is not None:
        theta = float(theta_given)
        xi_rot = xi(apply_gate(T4, gates.g4(theta)), qn[p], qn[p + 2], chi_cap) if theta != 0.0 else xi_none
    elif rotation == "givens":
        theta, xi_rot, _ = optimise_theta(T4, qn[p], qn[p + 2], chi_cap, n_grid, n_golden, xi_tol)
    new_sites, new_qn, U_new, T4r, st = finish(T4, sites, qn, bi.U, p, rotation, theta, chi_cap, tau_w)
    E_old = solve_projection(H, S, eps_S)["E"]
    E_new, mit = sol["E"], None
    if nreps > 0:
        G16 = np.eye(16)
        if theta != 0.0:
            G16 = gates.g4(theta) if rotation == "givens" else gates.f4()
        Ap, Aq, (msol, mkeep) = mitigate(prob, H, S, i, p, index, Hd, Sd, Hc, Sc, G16, new_sites[p],
                                         new_sites[p + 1], qn, new_qn[p + 1], nreps, tol_ld, eps_S)
        new_sites[p], new_sites[p + 1] = Ap, Aq
        E_new = msol["E"]
        mit = dict(E=msol["E"], n_kept=int(mkeep.sum()), n_columns=len(mkeep), n_dropped_S=msol["n_dropped"])
    return dict(E_old=E_old, E1=sol["E"], E_new=E_new, mitigation=mit,
                accepted=bool(E_new < E_old + e_tol), keep=keep, pos=pos,
                n_onehot=n, index=index, t_old=t, t_new=tn, T4=T4, T4_rotated=T4r, theta=theta,
                xi_none=xi_none, xi=xi_rot, canon_sites=sites, canon_qn=qn, sites=new_sites, qn=new_qn,
                U=U_new, trunc=st, n_dropped_S=sol["n_dropped"], onehot=(Hd, Sd, Hc, Sc))
