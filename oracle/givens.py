"""Givens decomposition of an orbital rotation (Sec. II.B, eq. givens_decomp).

The paper factors an orbital rotation G_ij into N(N-1)/2 nearest-neighbour
Givens gates g_{p,p+1}(theta), following from a QR factorisation of the N x N
rotation matrix.  The paper fixes neither the elimination order nor the angle
convention; any valid factorisation gives the same exact operator but a
different truncated state, so this project fixes one (both the oracle and the
library follow this text, not shared code):

  R_a(theta) = identity except [[c, s], [-s, c]] on rows/cols (a, a+1), which
  is the single-particle matrix of g_{a,a+1}(theta) = exp[theta (a+_a a_{a+1}
  - a+_{a+1} a_a)] (summed over spin).

  Q <- W.  For column c = 0..N-2 and row r = N-1 down to c+1: a = r-1,
  theta = atan2(-Q[r, c], Q[a, c]), Q <- R_a(theta)^T Q, record (a, theta).
  An entry already zero to rounding (|Q[r, c]| <= 1e-14) is not rotated
  away: theta = 0, except pi at the pivot row (a = c) when Q[a, c] < 0, so
  that the pivot ends non-negative.  Without this, rounding noise in a W close
  to a permutation or the identity would pick arbitrary angles.  Then
  Q = diag(1, .., 1, det W) and W = R_(1) R_(2) ... R_(K) D.

  Gates are applied to a ket in the reverse of the recorded order, after the
  parity gate D (only needed when det W = -1).
"""
import numpy as np

ZERO = 1e-14   # entries of an orthogonal matrix at or below this are rounding noise


def rot(N, a, theta):
    R = np.eye(N)
    c, s = np.cos(theta), np.sin(theta)
    R[a, a] = c
    R[a, a + 1] = s
    R[a + 1, a] = -s
    R[a + 1, a + 1] = c
    return R


def plan(W):
    """Return (gates, det_sign): gates = [(a, theta)] in APPLICATION order."""
    W = np.asarray(W, dtype=float)
    N = W.shape[0]
    Q = W.copy()
    elim = []
    for c in range(N - 1):
        for r in range(N - 1, c, -1):
            a = r - 1
            if abs(Q[r, c]) <= ZERO:
                theta = float(np.pi) if (a == c and Q[a, c] < 0.0) else 0.0
            else:
                theta = float(np.arctan2(-Q[r, c], Q[a, c]))
            Q = rot(N, a, theta).T @ Q
            elim.append((a, theta))
    det_sign = 1 if Q[N - 1, N - 1] > 0 else -1
    return list(reversed(elim)), det_sign


def compose(N, gates, det_sign):
    """Single-particle matrix of the planned network (for the P3 pin)."""
    W = np.eye(N)
    if det_sign < 0:
        W[N - 1, N - 1] = -1.0
    for a, theta in gates:          # application order: later gates multiply on the left
        W = rot(N, a, theta) @ W
    return W
