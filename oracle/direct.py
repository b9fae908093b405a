"""Reference solve X(s) = K(s)^{-1} F by banded Cholesky (test infrastructure only).

This is the plain definition of what every shifted solve of the paper
computes (the state X(s) of Section 2; the shifted systems of Algorithm 1),
written out as a direct factorisation of the symmetric
positive definite band matrix.  Two precisions are provided (binary64 and
double-double); the double-double path can also assemble K(s) itself in
double-double from the exact binary64 M and K, so its result is the solution
of the pencil as specified rather than of a rounded K(s).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import _native
from .pencil import shifted_operator


def bandwidth(a: sp.csr_matrix) -> int:
    a = a.tocoo()
    if a.nnz == 0:
        return 0
    return int(np.max(np.abs(a.row.astype(np.int64) - a.col.astype(np.int64))))


def lower_band(a: sp.csr_matrix, w: int | None = None) -> tuple[np.ndarray, int]:
    """Lower band storage ab[i, k] = A[i, i-k], k = 0..w (C-contiguous)."""
    if w is None:
        w = bandwidth(a)
    n = a.shape[0]
    c = a.tocoo()
    keep = (c.row >= c.col) & (c.row - c.col <= w)
    ab = np.zeros((n, w + 1))
    np.add.at(ab, (c.row[keep], c.row[keep] - c.col[keep]), c.data[keep])
    return ab, w


def band_solve(ab: np.ndarray, w: int, b: np.ndarray, precision: str = "f64",
               ab_lo: np.ndarray | None = None):
    """Solve with an SPD band matrix; b has shape (nrhs, n) or (n,).

    precision "f64" returns x; "dd" returns (x_hi, x_lo).
    Raises ``np.linalg.LinAlgError`` when a pivot is not positive.
    """
    ab = np.ascontiguousarray(ab, dtype=np.float64)
    n = ab.shape[0]
    squeeze = b.ndim == 1
    bb = np.ascontiguousarray(np.atleast_2d(b), dtype=np.float64)
    nrhs = bb.shape[0]
    xh = np.empty_like(bb)
    xl = np.empty_like(bb)
    lo = None if ab_lo is None else np.ascontiguousarray(ab_lo, dtype=np.float64)
    st = _native.lib().oracle_band_solve(n, w, _native.dptr(ab), _native.dptr(lo), nrhs,
                                         _native.dptr(bb), _native.dptr(xh), _native.dptr(xl),
                                         0 if precision == "f64" else 1)
    if st != 0:
        raise np.linalg.LinAlgError(f"band Cholesky: non-positive pivot (code {st})")
    if precision == "f64":
        return xh[0] if squeeze else xh
    return (xh[0], xl[0]) if squeeze else (xh, xl)


def residual_dd(ab, w, b, x_hi, x_lo=None, ab_lo=None) -> np.ndarray:
    """b - A x evaluated in double-double (x = x_hi + x_lo exactly)."""
    ab = np.ascontiguousarray(ab, dtype=np.float64)
    n = ab.shape[0]
    bb = np.ascontiguousarray(np.atleast_2d(b), dtype=np.float64)
    xh = np.ascontiguousarray(np.atleast_2d(x_hi), dtype=np.float64)
    xl = None if x_lo is None else np.ascontiguousarray(np.atleast_2d(x_lo), dtype=np.float64)
    lo = None if ab_lo is None else np.ascontiguousarray(ab_lo, dtype=np.float64)
    r = np.empty_like(bb)
    _native.lib().oracle_band_residual_dd(n, w, _native.dptr(ab), _native.dptr(lo), bb.shape[0],
                                          _native.dptr(bb), _native.dptr(xh),
                                          _native.dptr(xl), _native.dptr(r))
    return r[0] if np.ndim(b) == 1 else r


def shifted_band_dd(pen, s, w: int | None = None):
    """Lower band of K(s) = s^2 M + s D + K assembled entrywise in double-double."""
    m_band, w = lower_band(_pattern_matrix(pen, pen.m_val), w)
    k_band, _ = lower_band(_pattern_matrix(pen, pen.k_val), w)
    hi = np.empty_like(m_band)
    lo = np.empty_like(m_band)
    _native.lib().oracle_shift_dd(m_band.size, _native.dptr(m_band), _native.dptr(k_band),
                                  float(s), float(pen.alpha), float(pen.beta),
                                  _native.dptr(hi), _native.dptr(lo))
    return hi, lo, w


def _pattern_matrix(pen, val):
    from .pencil import csr
    return csr(pen.n, pen.row_ptr, pen.col_idx, val)


def reference_solve(pen, s, f: np.ndarray, precision: str = "dd") -> np.ndarray:
    """X(s) = K(s)^{-1} F for F of shape (m, n).

    "dd": K(s) assembled and factorised in double-double (the trusted
    reference); "f64": K(s) from the binary64 formula, factorised in binary64.
    """
    if precision == "dd":
        hi, lo, w = shifted_band_dd(pen, s)
        xh, xl = band_solve(hi, w, f, "dd", ab_lo=lo)
        return xh + xl
    a = shifted_operator(pen, s)
    ab, w = lower_band(a)
    return band_solve(ab, w, f, "f64")


def reference_solves(pen, shifts, f: np.ndarray, precision: str = "dd",
                     workers: int = 1, each=None) -> list | None:
    """reference_solve for every shift in ``shifts`` (a list of (m, n) arrays,
    or, when ``each`` is given, each(i, x) called in shift order as the
    results arrive, which are then not kept).

    The lower bands of M and K are extracted once and K(s) is formed on the
    band for each shift by the same entrywise formula as reference_solve
    ("f64": s^2 M + s (alpha M + beta K) + K in binary64; "dd": the
    double-double assembly), so each result equals reference_solve's.
    Shifts run on ``workers`` threads (the factorisations release the
    interpreter lock).
    """
    from concurrent.futures import ThreadPoolExecutor
    from .pencil import shifted_values
    m_band, w = lower_band(_pattern_matrix(pen, pen.m_val))
    k_band, _ = lower_band(_pattern_matrix(pen, pen.k_val), w)
    _native.lib()

    def one(s):
        if precision == "dd":
            hi = np.empty_like(m_band)
            lo = np.empty_like(m_band)
            _native.lib().oracle_shift_dd(m_band.size, _native.dptr(m_band), _native.dptr(k_band),
                                          float(s), float(pen.alpha), float(pen.beta),
                                          _native.dptr(hi), _native.dptr(lo))
            xh, xl = band_solve(hi, w, f, "dd", ab_lo=lo)
            return xh + xl
        ab = shifted_values(m_band, k_band, pen.alpha, pen.beta, s)
        return band_solve(ab, w, f, "f64")

    if each is None:
        if workers <= 1:
            return [one(s) for s in shifts]
        with ThreadPoolExecutor(workers) as ex:
            return list(ex.map(one, shifts))
    if workers <= 1:
        for i, s in enumerate(shifts):
            each(i, one(s))
        return None
    with ThreadPoolExecutor(workers) as ex:
        for i, x in enumerate(ex.map(one, shifts)):
            each(i, x)
    return None


# ------------------------------------------------------------ complex shifts
#
# For a complex expansion point s, K(s) = s^2 M + s D + K is complex
# symmetric, not Hermitian.  The reference solve factorises it as
# L Dg L^T (transposes without conjugation) on the band, in binary64 complex
# or in double-double complex with K(s) assembled entrywise in double-double
# from the exact binary64 M and K.


def cband_solve(re, im, w, b, precision="f64", re_lo=None, im_lo=None):
    """Solve with a complex symmetric band matrix (lower band re + i im);
    b (nrhs, n) or (n,), real or complex.  Returns the complex solution
    (rounded to binary64 in double-double mode)."""
    n = re.shape[0]
    squeeze = np.ndim(b) == 1
    bb = np.atleast_2d(np.asarray(b))
    br = np.ascontiguousarray(bb.real, dtype=np.float64)
    bi = np.ascontiguousarray(bb.imag, dtype=np.float64) if np.iscomplexobj(bb) else None
    xr = np.empty_like(br)
    xi = np.empty_like(br)
    arrs = [np.ascontiguousarray(a, dtype=np.float64) if a is not None else None
            for a in (re, re_lo, im, im_lo)]
    st = _native.lib().oracle_cband_solve(n, w, *(_native.dptr(a) for a in arrs), bb.shape[0],
                                          _native.dptr(br), _native.dptr(bi), _native.dptr(xr),
                                          _native.dptr(xi), None, None,
                                          0 if precision == "f64" else 1)
    if st != 0:
        raise np.linalg.LinAlgError(f"complex band LDL^T: zero pivot (code {st})")
    x = xr + 1j * xi
    return x[0] if squeeze else x


def shifted_band_cdd(pen, s: complex, w: int | None = None):
    """Lower band of K(s) for complex s, entrywise in double-double:
    (re_hi, re_lo, im_hi, im_lo, w)."""
    m_band, w = lower_band(_pattern_matrix(pen, pen.m_val), w)
    k_band, _ = lower_band(_pattern_matrix(pen, pen.k_val), w)
    out = [np.empty_like(m_band) for _ in range(4)]
    _native.lib().oracle_shift_cdd(m_band.size, _native.dptr(m_band), _native.dptr(k_band),
                                   float(np.real(s)), float(np.imag(s)), float(pen.alpha),
                                   float(pen.beta), *(_native.dptr(o) for o in out))
    return (*out, w)


def reference_solve_complex(pen, s: complex, f: np.ndarray, precision: str = "dd") -> np.ndarray:
    """X(s) = K(s)^{-1} F for complex s and F of shape (m, n) (complex result).

    "dd": K(s) assembled and factorised in double-double complex (the trusted
    reference); "f64": K(s) from the binary64 complex formula, factorised in
    binary64 complex."""
    if precision == "dd":
        rh, rl, ih, il, w = shifted_band_cdd(pen, s)
        return cband_solve(rh, ih, w, f, "dd", re_lo=rl, im_lo=il)
    from .pencil import shifted_values_complex
    m_band, w = lower_band(_pattern_matrix(pen, pen.m_val))
    k_band, _ = lower_band(_pattern_matrix(pen, pen.k_val), w)
    ab = shifted_values_complex(m_band, k_band, pen.alpha, pen.beta, s)
    return cband_solve(ab.real, ab.imag, w, f, "f64")
