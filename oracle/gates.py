"""Two-site gates (App. A3 of arXiv 2404.10223).

Spin-orbital (d = 2) gates are the 4x4 matrices printed in App. A3 in the basis
|00>, |01>, |10>, |11> of two adjacent fermionic modes (first mode = most
significant bit):

* FSWAP f2 (eq. fswap): swaps the modes and puts -1 on |11>;
* Givens g2(theta): |01> -> cos|01> + sin|10>, |10> -> cos|10> - sin|01>.

The spatial-orbital (d = 4) gates are the composites given at the end of
App. A3, f4 = (1 x f2 x 1)(f2 x f2)(1 x f2 x 1) and
g4 = (1 x f2 x 1)(g2 x g2)(1 x f2 x 1), acting on the four modes
(p up, p down, p+1 up, p+1 down) in that Jordan-Wigner order.

Site basis used everywhere in this project: k = n_up + 2 n_dn, i.e.
0 = vac, 1 = up, 2 = down, 3 = up+down (the label order of Sec. II.A), with
|up, down> = a+_{p,up} a+_{p,down} |vac>.  The 16x16 two-site matrices
returned here act on the pair index k_p * 4 + k_{p+1}.
"""
import numpy as np

F2 = np.array([[1, 0, 0, 0],
               [0, 0, 1, 0],
               [0, 1, 0, 0],
               [0, 0, 0, -1]], dtype=float)


def g2(theta):
    c, s = np.cos(theta), np.sin(theta)
    return np.array([[1, 0, 0, 0],
                     [0, c, -s, 0],
                     [0, s, c, 0],
                     [0, 0, 0, 1]], dtype=float)


# mode-bit index (n_up, n_dn) with n_up most significant  ->  site index k
def _site_perm():
    P = np.zeros((4, 4))
    for nu in (0, 1):
        for nd in (0, 1):
            P[nu + 2 * nd, 2 * nu + nd] = 1.0
    return P


_P1 = _site_perm()
_P2 = np.kron(_P1, _P1)     # (kron basis of 4 modes) -> (k_p, k_{p+1})


def _to_site_basis(M16):
    return _P2 @ M16 @ _P2.T


def g4(theta):
    """Spatial-orbital Givens gate on (k_p, k_{p+1}), 16x16."""
    I2 = np.eye(2)
    mid = np.kron(np.kron(I2, F2), I2)
    return _to_site_basis(mid @ np.kron(g2(theta), g2(theta)) @ mid)


def f4():
    """Spatial-orbital FSWAP on (k_p, k_{p+1}), 16x16."""
    I2 = np.eye(2)
    mid = np.kron(np.kron(I2, F2), I2)
    return _to_site_basis(mid @ np.kron(F2, F2) @ mid)


def parity_gate():
    """Single-site diag(1, -1, -1, 1): the rotation diag(1, .., 1, -1) on the last orbital."""
    return np.diag([1.0, -1.0, -1.0, 1.0])
