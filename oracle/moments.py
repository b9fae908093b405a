"""Galerkin projection and moment matching (test infrastructure only).

Projection onto the columns of V (eq. (1.4)): M_hat = V^T M V,
D_hat = V^T D V, K_hat = V^T K V, F_hat = V^T F, C_hat = C_p V, and the
reduced transfer function H_hat(s) = C_hat (s^2 M_hat + s D_hat + K_hat)^{-1}
F_hat (Section 2).  When the range of V contains the solves X(s_i) at the
expansion points, the reduced model interpolates the full one there,
H_hat(s_i) = H(s_i): the goal of the moment-matching construction
(Section 2).  This pins the solves as a whole.

The block steps of Algorithm 1 around the solves are here too: the
right-hand sides (a M + b K) X, the orthogonalisation of a block against
the earlier ones in the trace inner product (global Arnoldi), and the thin
QR of the collected blocks.
"""
from __future__ import annotations

import numpy as np


def project(m, k, alpha, beta, f, cp, v):
    """Reduced matrices of eq. (1.4) for dense or sparse M, K."""
    mh = v.T @ (m @ v)
    kh = v.T @ (k @ v)
    dh = alpha * mh + beta * kh
    return mh, dh, kh, v.T @ f, cp @ v


def reduced_transfer(mh, dh, kh, fh, ch, s):
    return ch @ np.linalg.solve(s * s * mh + s * dh + kh, fh)


def orth_basis(blocks):
    """Orthonormal basis of the span of the given n x m blocks (QR)."""
    q, _ = np.linalg.qr(np.hstack(blocks))
    return q


def pencil_apply(m, k, a, b, x):
    """(a M + b K) x: with a = 1, b = 0 the right-hand side M V_j of the
    moment solves of Algorithm 1 (Section 2)."""
    return a * (m @ x) + b * (k @ x)


def global_orth(v_blocks, x):
    """Algorithm 1's loop over t for one n x m block X: in order t = 1..j,
    gamma_t = trace(V_t^T X), then X <- X - gamma_t V_t (each product sees
    the X left by the previous step).  Returns (X, gammas, ||X||_F)."""
    x = np.array(x, dtype=float, copy=True)
    gam = []
    for vt in v_blocks:
        g = float(np.trace(vt.T @ x))
        x = x - g * vt
        gam.append(g)
    return x, np.array(gam, dtype=float), float(np.linalg.norm(x))


def thin_qr(w):
    """Thin QR W = Q R with the diagonal of R positive (the factorisation is
    then unique for full column rank): the library QR, column signs fixed."""
    q, r = np.linalg.qr(w)
    sgn = np.where(np.diag(r) < 0, -1.0, 1.0)
    return q * sgn, r * sgn[:, None]
