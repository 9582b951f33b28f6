"""MPS operations in FP64 (Sec. II.A and App. A1, A3 of arXiv 2404.10223).

An MPS is a pair (sites, qn): sites[p] has shape [d_p, 4, d_{p+1}] and
qn[b] is an int array [d_b, 2] giving (n_alpha, n_beta) of sites 0..b-1 for
each index of bond b.  Site tensors conserve particle number and S_z: entry
[l, k, r] may be nonzero only if qn[p+1][r] = qn[p][l] + q(k) with
q(k) = (k & 1, k >> 1).  This is the block-sparse (U(1) x U(1)) structure the
paper's numerics enforce (Sec. V "Numerical details"); here it only decides
which blocks the factorisations work on, the storage is dense.

Canonical form (App. A1, eq. orth_l / orth_r): sites left of the centre are
left-orthonormal, sites right of it right-orthonormal.  Moving the centre is an
exact QR/LQ factorisation.  A two-site gate is applied to the centre pair and
the result split by SVD (eq. svd_longform), keeping the chi largest singular
values over all quantum-number blocks; the singular values are absorbed to the
right, so the centre moves one site to the right (the "Sigma contracted into V"
step after eq. svd_longform).  No renormalisation after truncation by default: the kept
state is the orthogonal projection of the gated state.
"""
import numpy as np

QK = np.array([[0, 0], [1, 0], [0, 1], [1, 1]])


def copy_mps(sites, qn):
    return [a.copy() for a in sites], [q.copy() for q in qn]


def _sectors(q):
    """Sorted list of distinct sectors in a [n, 2] label array."""
    if len(q) == 0:
        return []
    return sorted(set(map(tuple, q.tolist())))


def _where(q, s):
    return np.nonzero((q[:, 0] == s[0]) & (q[:, 1] == s[1]))[0]


def _positive_qr(a):
    """Reduced QR with a non-negative diagonal of R: for a block of full rank
    this fixes the factors uniquely, so the canonical form (and with it the
    one-hot states of App. A1) does not depend on the QR routine's signs."""
    q, r = np.linalg.qr(a)
    d = np.where(np.diag(r) < 0.0, -1.0, 1.0)
    return q * d[None, :], r * d[:, None]


def _qr_right(sites, qn, p):
    """Exact move of the centre from site p to p+1 (A_p = Q R, R into A_{p+1})."""
    A = sites[p]
    dl, _, dr = A.shape
    rowq = (qn[p][:, None, :] + QK[None, :, :]).reshape(-1, 2)
    M = A.reshape(dl * 4, dr)
    qblocks, rblocks, newq = [], [], []
    for s in _sectors(qn[p + 1]):
        cols = _where(qn[p + 1], s)
        rows = _where(rowq, s)
        if len(rows) == 0:
            continue
        q, r = _positive_qr(M[np.ix_(rows, cols)])
        qblocks.append((rows, q))
        rblocks.append((cols, r))
        newq += [s] * q.shape[1]
    dn = len(newq)
    Qm = np.zeros((dl * 4, dn))
    R = np.zeros((dn, dr))
    o = 0
    for (rows, q), (cols, r) in zip(qblocks, rblocks):
        Qm[rows, o:o + q.shape[1]] = q
        R[o:o + q.shape[1], cols] = r
        o += q.shape[1]
    sites[p] = Qm.reshape(dl, 4, dn)
    sites[p + 1] = np.einsum("ab,bkc->akc", R, sites[p + 1])
    qn[p + 1] = np.array(newq, dtype=np.int64).reshape(-1, 2)


def _lq_left(sites, qn, p):
    """Exact move of the centre from site p to p-1 (A_p = L Q, L into A_{p-1})."""
    A = sites[p]
    dl, _, dr = A.shape
    colq = (qn[p + 1][None, :, :] - QK[:, None, :]).reshape(-1, 2)   # index (k, r)
    M = A.reshape(dl, 4 * dr)
    lblocks, qblocks, newq = [], [], []
    for s in _sectors(qn[p]):
        rows = _where(qn[p], s)
        cols = _where(colq, s)
        if len(cols) == 0:
            continue
        q, r = _positive_qr(M[np.ix_(rows, cols)].T)     # M_b = r^T q^T
        lblocks.append((rows, r.T))
        qblocks.append((cols, q.T))
        newq += [s] * q.shape[1]
    dn = len(newq)
    Lm = np.zeros((dl, dn))
    Qm = np.zeros((dn, 4 * dr))
    o = 0
    for (rows, l), (cols, q) in zip(lblocks, qblocks):
        Lm[rows, o:o + l.shape[1]] = l
        Qm[o:o + q.shape[0], cols] = q
        o += q.shape[0]
    sites[p] = Qm.reshape(dn, 4, dr)
    sites[p - 1] = np.einsum("akb,bc->akc", sites[p - 1], Lm)
    qn[p] = np.array(newq, dtype=np.int64).reshape(-1, 2)


def left_canonicalize(sites, qn):
    """QR sweep left to right; the centre (and the norm) ends on the last site."""
    for p in range(len(sites) - 1):
        _qr_right(sites, qn, p)
    return len(sites) - 1


def move_centre(sites, qn, centre, target):
    while centre > target:
        _lq_left(sites, qn, centre)
        centre -= 1
    while centre < target:
        _qr_right(sites, qn, centre)
        centre += 1
    return centre


def select_kept(allsv, chi_cap, tau_w):
    """Truncation rule of App. A1 over the singular values of all blocks of a
    two-site matrix (concatenated in block order): the keep = min(chi_cap,
    #{s^2 > tau_w sum s^2}) largest are kept, equal values taken in the order
    of allsv.

    Returns (kept mask, keep, number above the threshold, relative gap at the
    cut or None, discarded weight, total weight).
    """
    w2 = allsv ** 2
    total = w2.sum()
    nnz = int((w2 > tau_w * total).sum())
    keep = min(chi_cap, nnz)
    order = np.argsort(-allsv, kind="stable")
    kept_mask = np.zeros(len(allsv), dtype=bool)
    kept_mask[order[:keep]] = True
    gap = None
    if keep < len(allsv) and keep > 0:
        s_in, s_out = allsv[order[keep - 1]], allsv[order[keep]]
        gap = (s_in - s_out) / s_in
    discarded = float(w2[~kept_mask].sum())
    return kept_mask, keep, nnz, gap, discarded, float(total)


def gate_and_truncate(sites, qn, p, G16, chi_cap, tau_w, renormalize=False):
    """Apply a 16x16 gate to sites (p, p+1) (centre at p), split by truncated SVD.

    With renormalize, the kept part is rescaled to the weight the gated state
    had before the cut (App. A1 renormalises after truncating in its DMRG
    setting; here it is optional, off by default).

    Returns a dict with the discarded weight, the number kept, the number of
    nonzero singular values and the relative gap at the cut (None if nothing
    was cut).
    """
    A, B = sites[p], sites[p + 1]
    dl, dr = A.shape[0], B.shape[2]
    T = np.einsum("akm,mlb->aklb", A, B)                            # [dl, kp, kq, dr]
    T = np.einsum("xy,ayb->axb", G16, T.reshape(dl, 16, dr))         # gate on (kp, kq)
    Tm = T.reshape(dl * 4, 4 * dr)
    rowq = (qn[p][:, None, :] + QK[None, :, :]).reshape(-1, 2)
    colq = (qn[p + 2][None, :, :] - QK[:, None, :]).reshape(-1, 2)
    blocks = []
    for s in _sectors(rowq):
        rows = _where(rowq, s)
        cols = _where(colq, s)
        if len(cols) == 0:
            continue
        u, sv, vt = np.linalg.svd(Tm[np.ix_(rows, cols)], full_matrices=False)
        blocks.append((s, rows, cols, u, sv))
    allsv = np.concatenate([b[4] for b in blocks]) if blocks else np.zeros(0)
    kept_mask, keep, nnz, gap, discarded, total = select_kept(allsv, chi_cap, tau_w)
    # new bond, sorted by sector; inside a sector, singular vectors by decreasing value
    newq, cols_u = [], []
    o = 0
    for s, rows, cols, u, sv in blocks:
        n = len(sv)
        k = int(kept_mask[o:o + n].sum())
        # numpy's SVD returns values in decreasing order inside a block, and the
        # global selection keeps a prefix of each block's list
        assert kept_mask[o:o + k].all()
        o += n
        if k == 0:
            continue
        newq += [s] * k
        cols_u.append((rows, u[:, :k]))
    dn = len(newq)
    U = np.zeros((dl * 4, dn))
    c = 0
    for rows, uk in cols_u:
        U[rows, c:c + uk.shape[1]] = uk
        c += uk.shape[1]
    sites[p] = U.reshape(dl, 4, dn)
    sites[p + 1] = (U.T @ Tm).reshape(dn, 4, dr)
    if renormalize and discarded > 0.0 and total > discarded:
        sites[p + 1] = sites[p + 1] * np.sqrt(total / (total - discarded))
    qn[p + 1] = np.array(newq, dtype=np.int64).reshape(-1, 2)
    return dict(discarded=discarded, kept=dn, nonzero=nnz, gap=gap, total=total)


def apply_site_op(sites, p, G4):
    sites[p] = np.einsum("xk,akb->axb", G4, sites[p])


def overlap(bra, ket):
    """<bra|ket> by the left transfer sweep."""
    E = np.ones((1, 1))
    for A, B in zip(bra, ket):
        X = np.einsum("ab,bkc->akc", E, B)
        E = np.einsum("akd,akc->dc", A, X)
    return float(E[0, 0])


def check_qn(sites, qn, tol=0.0):
    """Largest magnitude of an entry that violates particle-number conservation."""
    worst = 0.0
    for p, A in enumerate(sites):
        for k in range(4):
            allowed = ((qn[p][:, None, 0] + QK[k, 0] == qn[p + 1][None, :, 0])
                       & (qn[p][:, None, 1] + QK[k, 1] == qn[p + 1][None, :, 1]))
            bad = np.abs(A[:, k, :][~allowed])
            if bad.size:
                worst = max(worst, float(bad.max()))
    return worst
