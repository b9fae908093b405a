"""Galerkin projection and moment matching (test infrastructure only).

Projection onto the columns of V (eq. (1.4)): M_hat = V^T M V,
D_hat = V^T D V, K_hat = V^T K V, F_hat = V^T F, C_hat = C_p V, and the
reduced transfer function H_hat(s) = C_hat (s^2 M_hat + s D_hat + K_hat)^{-1}
F_hat (Section 2).  When the range of V contains the solves X(s_i) at the
expansion points, the reduced model interpolates the full one there,
H_hat(s_i) = H(s_i): the goal of the moment-matching construction
(Section 2).  This pins the solves as a whole.
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
