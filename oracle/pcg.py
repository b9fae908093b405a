"""Preconditioned conjugate gradients (test infrastructure only).

CG is the solver the paper uses for its symmetric positive definite shifted
systems (Section 3 and Section 5): a Ritz-Galerkin method whose residual is
orthogonal to the Krylov space, the property its stability result requires
(Theorem 4.2).  Preconditioning is applied as z = C r with C the SPAI (or the
chain Q_z ... Q_2 P_1 of the update algorithm); right preconditioning
K C y = f, x = C y, produces the same iterates x.

A fixed-pattern right SPAI, and every update chain, is not a symmetric
operator, so the direction update must not rely on the symmetry of C.  The
default ("flexible") keeps each new direction K-conjugate to the previous one:
    beta = -(z_new, K p) / (p, K p),
which equals the classical ratio (r_new, z_new) / (r_old, z_old) (and the
Polak-Ribiere one) whenever C is symmetric.  The Polak-Ribiere
(r_new, z_new - z_old) / (r_old, z_old) and Fletcher-Reeves forms are
available for comparison.  The step length alpha = (r, z) / (p, K p) is the
exact line search of the K-norm error along p; it stays meaningful when
(r, z) < 0 (possible for a non-symmetric C), so only (p, K p) <= 0 stops the
iteration as a breakdown.

Iteration, from x_0 (zero unless given):
    r = f - K x;  z = C r;  p = z
    repeat:  w = K p;  alpha = (r, z) / (p, w);  x += alpha p;  r -= alpha w
             stop when ||r|| <= tol ||f||
             z_new = C r;  beta as above;  p = z_new + beta p
Per-system status: CONVERGED, MAXIT (iteration cap), BREAKDOWN ((p, w) <= 0),
NONFINITE (a NaN or infinity appeared).
"""
from __future__ import annotations

import dataclasses

import numpy as np

CONVERGED, MAXIT, BREAKDOWN, NONFINITE = 0, 1, 2, 3


@dataclasses.dataclass
class PcgResult:
    x: np.ndarray
    status: int
    iters: int
    relres: float            # recurrence residual ||r|| / ||f|| at exit
    history: list            # recurrence residual norms, one per iteration
    directions: list         # search directions (only when keep=True)
    residuals: list          # residuals (only when keep=True)


def pcg(matvec, precond, f, *, tol=1e-10, max_iter=10000, x0=None, beta="flexible",
        keep=False) -> PcgResult:
    f = np.asarray(f, dtype=np.float64)
    fnorm = float(np.linalg.norm(f))
    x = np.zeros_like(f) if x0 is None else np.array(x0, dtype=np.float64)
    r = f - matvec(x) if x0 is not None else f.copy()
    hist, dirs, ress = [], [], []
    if not np.all(np.isfinite(r)):
        return PcgResult(x, NONFINITE, 0, float("nan"), hist, dirs, ress)
    rnorm = float(np.linalg.norm(r))
    if rnorm <= tol * fnorm:
        return PcgResult(x, CONVERGED, 0, rnorm / fnorm if fnorm > 0 else 0.0, hist, dirs, ress)
    z = precond(r)
    rz = float(r @ z)
    if not np.isfinite(rz):
        return PcgResult(x, NONFINITE, 0, rnorm / fnorm, hist, dirs, ress)
    p = z.copy()
    for k in range(max_iter):
        if keep:
            dirs.append(p.copy())
            ress.append(r.copy())
        w = matvec(p)
        pw = float(p @ w)
        if not np.isfinite(pw):
            return PcgResult(x, NONFINITE, k, rnorm / fnorm, hist, dirs, ress)
        if pw <= 0.0:
            return PcgResult(x, BREAKDOWN, k, rnorm / fnorm, hist, dirs, ress)
        alpha = rz / pw
        x = x + alpha * p
        r = r - alpha * w
        rnorm = float(np.linalg.norm(r))
        hist.append(rnorm)
        if not np.isfinite(rnorm):
            return PcgResult(x, NONFINITE, k + 1, rnorm, hist, dirs, ress)
        if rnorm <= tol * fnorm:
            if keep:
                ress.append(r.copy())
            return PcgResult(x, CONVERGED, k + 1, rnorm / fnorm, hist, dirs, ress)
        z_new = precond(r)
        rz_new = float(r @ z_new)
        if not np.isfinite(rz_new):
            return PcgResult(x, NONFINITE, k + 1, rnorm / fnorm, hist, dirs, ress)
        if beta == "flexible":
            b = -float(z_new @ w) / pw
        elif beta == "pr":
            b = (rz_new - float(r @ z)) / rz
        elif beta == "fr":
            b = rz_new / rz
        else:
            raise ValueError(beta)
        p = z_new + b * p
        z, rz = z_new, rz_new
    return PcgResult(x, MAXIT, max_iter, rnorm / fnorm, hist, dirs, ress)


def cocg(matvec, precond, f, *, tol=1e-10, max_iter=10000, beta="flexible", keep=False) -> PcgResult:
    """Conjugate orthogonal CG for complex symmetric systems (K(s) at a complex
    expansion point; van der Vorst and Melissen, IEEE Trans. Magn. 1990):
    CG with the bilinear form x^T y (no conjugation) in place of the inner
    product, for a complex symmetric K and a complex symmetric preconditioner
    C.  From x = 0:  r = f;  z = C r;  p = z
      repeat:  w = K p;  mu = p^T w;  alpha = (r^T z) / mu;  x += alpha p;
               r -= alpha w;  stop when ||r|| <= tol ||f|| (Euclidean norm);
               z_new = C r;  beta;  p = z_new + beta p
    with the flexible beta = -(z_new^T w) / mu (p stays conjugate orthogonal
    to the previous direction, K-wise, under any C) or ("fr") the classical
    ratio (r^T z)_new / (r^T z)_old.  Both reduce to CG for real data.  Statuses as
    for pcg: BREAKDOWN when mu = 0 (the bilinear form has no sign to test),
    NONFINITE on a NaN or infinity."""
    f = np.asarray(f, dtype=complex)
    fnorm = float(np.linalg.norm(f))
    x = np.zeros_like(f)
    r = f.copy()
    hist, dirs, ress = [], [], []
    rnorm = fnorm
    if rnorm <= tol * fnorm:
        return PcgResult(x, CONVERGED, 0, 0.0, hist, dirs, ress)
    z = precond(r)
    rz = complex(r @ z)
    p = z.copy()
    for k in range(max_iter):
        if keep:
            dirs.append(p.copy())
            ress.append(r.copy())
        w = matvec(p)
        mu = complex(p @ w)
        if not np.isfinite(mu):
            return PcgResult(x, NONFINITE, k, rnorm / fnorm, hist, dirs, ress)
        if mu == 0:
            return PcgResult(x, BREAKDOWN, k, rnorm / fnorm, hist, dirs, ress)
        alpha = rz / mu
        x = x + alpha * p
        r = r - alpha * w
        rnorm = float(np.linalg.norm(r))
        hist.append(rnorm / fnorm)
        if not np.isfinite(rnorm):
            return PcgResult(x, NONFINITE, k + 1, rnorm / fnorm, hist, dirs, ress)
        if rnorm <= tol * fnorm:
            return PcgResult(x, CONVERGED, k + 1, rnorm / fnorm, hist, dirs, ress)
        zn = precond(r)
        rzn = complex(r @ zn)
        if beta == "flexible":
            b = -complex(zn @ w) / mu
        elif beta == "fr":
            b = rzn / rz
        else:
            raise ValueError(f"unknown beta form {beta!r}")
        p = zn + b * p
        rz = rzn
    return PcgResult(x, MAXIT, max_iter, rnorm / fnorm, hist, dirs, ress)
