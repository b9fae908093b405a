"""The shifted operator of the second-order system (test infrastructure only).

K(s) = s^2 M + s D + K with proportional damping D = alpha M + beta K
(eq. (1.1) and the transfer function H(s) = (C_p + s C_v)(s^2 M + s D + K)^{-1} F
of Section 2; the same matrix is the coefficient matrix of every solve in the
AIRGA algorithms).  The result keeps the shared structural pattern of M and K
(explicit zeros stay), because the SPAI pattern is the pattern of K(s).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def csr(n, row_ptr, col_idx, val) -> sp.csr_matrix:
    """CSR matrix on the given structural pattern; explicit zeros are kept."""
    a = sp.csr_matrix((np.asarray(val, dtype=np.float64), np.asarray(col_idx),
                       np.asarray(row_ptr)), shape=(n, n))
    a.has_sorted_indices = True
    return a


def damping_values(m_val, k_val, alpha, beta):
    """Entries of D = alpha M + beta K on the shared pattern (eq. (1.1))."""
    return alpha * np.asarray(m_val) + beta * np.asarray(k_val)


def shifted_values(m_val, k_val, alpha, beta, s):
    """Entries of s^2 M + s D + K on the shared pattern, written as the formula reads."""
    m_val = np.asarray(m_val, dtype=np.float64)
    k_val = np.asarray(k_val, dtype=np.float64)
    return (s * s) * m_val + s * damping_values(m_val, k_val, alpha, beta) + k_val


def shifted_values_complex(m_val, k_val, alpha, beta, s: complex):
    """Entries of s^2 M + s D + K for a complex expansion point s, in complex
    binary64, written as the formula reads."""
    s = complex(s)
    m_val = np.asarray(m_val, dtype=np.float64)
    k_val = np.asarray(k_val, dtype=np.float64)
    return (s * s) * m_val + s * damping_values(m_val, k_val, alpha, beta) + k_val


def shifted_operator_complex(pen, s: complex) -> sp.csr_matrix:
    """K(s) for complex s as a complex CSR matrix on the shared pattern (complex
    symmetric: K(s)^T = K(s))."""
    a = sp.csr_matrix((shifted_values_complex(pen.m_val, pen.k_val, pen.alpha, pen.beta, s),
                       np.asarray(pen.col_idx), np.asarray(pen.row_ptr)), shape=(pen.n, pen.n))
    a.has_sorted_indices = True
    return a


def shifted_operator(pen, s) -> sp.csr_matrix:
    """K(s) for a ``synthetic.beam.Pencil``-like object (n, row_ptr, col_idx,
    m_val, k_val, alpha, beta) as a CSR matrix on the shared pattern."""
    return csr(pen.n, pen.row_ptr, pen.col_idx,
               shifted_values(pen.m_val, pen.k_val, pen.alpha, pen.beta, s))


def frobenius_diagnostics(pen, s_old, s_new):
    """The two quantities the paper tabulates per expansion point:
    ||I - K(s_new)||_F and ||K(s_old) - K(s_new)||_F, computed directly."""
    a_new = shifted_operator(pen, s_new)
    a_old = shifted_operator(pen, s_old)
    eye = sp.identity(pen.n, format="csr")
    d1 = (eye - a_new)
    d2 = (a_old - a_new)
    return float(np.sqrt((d1.multiply(d1)).sum())), float(np.sqrt((d2.multiply(d2)).sum()))
