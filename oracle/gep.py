"""Generalized eigenproblem H c = E S c with S thresholding.

Sec. V "Regulating the subspace condition number" and App. A2 of arXiv
2404.10223: diagonalise S = U Lambda U^T, keep eigenvalues above a tolerance,
then either

* projection: solve [U_e^T H U_e] C' = [U_e^T S U_e] C' E' and map back with
  U_e (here written with the whitened basis X = U_e Lambda_e^(-1/2), which is
  the same reduced problem since U_e^T S U_e = Lambda_e), or
* inversion: diagonalise U Lambda_e^(-1) U^T H, then normalise c / sqrt(c^T S c).

The ground-state eigenvalue condition number is kappa_1 = |c_1|^2 / sqrt(E_1^2 + 1)
(App. A2, following Epperly et al.).
"""
import numpy as np


def solve_projection(H, S, eps_rel=1e-12):
    lam, U = np.linalg.eigh(S)
    lmax = lam.max()
    keep = lam > eps_rel * lmax
    X = U[:, keep] / np.sqrt(lam[keep])[None, :]
    Ht = X.T @ H @ X
    Ht = 0.5 * (Ht + Ht.T)
    e, y = np.linalg.eigh(Ht)
    c = X @ y[:, 0]
    E = float(e[0])
    return dict(E=E, c=c, n_dropped=int((~keep).sum()),
                cond_S=float(lmax / lam[keep].min()), lam_min=float(lam.min()),
                kappa1=float(c @ c / np.sqrt(E * E + 1.0)))


def solve_inversion(H, S, eps_rel=1e-12):
    lam, U = np.linalg.eigh(S)
    keep = lam > eps_rel * lam.max()
    Sinv = (U[:, keep] / lam[keep][None, :]) @ U[:, keep].T
    e, C = np.linalg.eig(Sinv @ H)
    e = np.real(e)
    C = np.real(C)
    order = np.argsort(np.where(np.abs(e) > 0, e, np.inf))
    # eigenvalues of the projected pencil; zero modes of the pseudo-inverse are excluded
    nz = [i for i in order if np.linalg.norm(S @ C[:, i]) > 1e-10]
    i0 = nz[0]
    c = C[:, i0] / np.sqrt(C[:, i0] @ S @ C[:, i0])
    return dict(E=float(e[i0]), c=c)
