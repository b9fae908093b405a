"""AIRGA's iteration (Algorithm 1) on the CPU (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU baseline use this
module; the library never calls it.

Algorithm 1 repeats, until the reduced model stops changing in the H2 norm:
solves X(s_i) = K(s_i)^{-1} F at the l expansion points and their thin QR;
a moment loop that picks an expansion point sigma_j, appends
V_j = X(sigma_j) / ||X(sigma_j)||_F to the basis, replaces X(sigma_j) by the
next moment -K(sigma_j)^{-1} M V_j, orthogonalises every X(s_i) against
V_1..V_j in the trace inner product, and forms an intermediate reduced model
from the thin QR of the normalised blocks; then the final basis
[V_1 .. V_J], its reduced model (eq. (1.4)), and new expansion points from
the eigenvalues of the reduced quadratic pencil, taking their real parts
(Section 5 explains why the real parts are used).  Both loops stop on an
H2 change below 1e-6 (Section 5).

The paper leaves these to Bonin et al. and does not fix them; the readings
taken here (also listed with the design notes) are:
  A1  the moment error at s_i is the fraction of the newest moment block
      X^{(j)}(s_i) that the orthogonalisation against V_1..V_j leaves,
      ||X after||_F / ||X before||_F (the part the basis does not hold
      yet, independent of the block's scale, which falls like s^-2);
      sigma_{j+1} is the s_i with the largest one.  sigma_1 = s_1, since
      before the first V there is nothing to compare.
  A2  "s_i == sigma_j" compares indices, not values.
  A3  the moment loop runs while j < floor(r_max / m), so the final basis
      [V_1..V_J] has J <= floor(r_max / m) blocks.
  A4  the new expansion points: each conjugate pair of reduced poles gives
      one candidate -Re(lambda), each real pole its own -lambda; candidates
      are ranked by |lambda| (smallest first) and the first l, in
      ascending order, are the new s_i.  The i-th new point's
      preconditioner is the update of the i-th old one (both ascending).
  A5  both H2 tests are relative: ||H_new - H_old||_H2 / ||H_new||_H2.
  A6  the H2 norm of a reduced model with output (C_p + s C_v) is that of
      its first-order realisation x' = A x + B u, y = C x with
      A = [[0, I], [-M^-1 K, -M^-1 D]], B = [0; M^-1 F], C = [C_p, C_v],
      from the controllability Gramian.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from . import moments


def qep_poles(mh, dh, kh):
    """The 2r eigenvalues of lambda^2 Mh + lambda Dh + Kh: the companion
    linearisation [[0, I], [-Mh^-1 Kh, -Mh^-1 Dh]] and the library
    eigenvalue routine."""
    r = mh.shape[0]
    a = np.block([[np.zeros((r, r)), np.eye(r)],
                  [-np.linalg.solve(mh, kh), -np.linalg.solve(mh, dh)]])
    return np.linalg.eigvals(a)


def next_shifts(poles, l):
    """Reading A4: one candidate per conjugate pair (-Re lambda), one per
    real pole (-lambda), ranked by |lambda|; the first l, ascending."""
    cands = []
    for lam in poles:
        if abs(lam.imag) <= 1e-12 * abs(lam):
            cands.append((abs(lam), -lam.real))
        elif lam.imag > 0:
            cands.append((abs(lam), -lam.real))
    cands.sort(key=lambda t: t[0])
    if len(cands) < l:
        raise ValueError("fewer candidate expansion points than l")
    return np.sort(np.array([c[1] for c in cands[:l]]))


class Model:
    """Reduced second-order model: (Mh, Dh, Kh, Fh, Cph, Cvh)."""

    def __init__(self, mh, dh, kh, fh, cph, cvh=None):
        self.mh, self.dh, self.kh, self.fh, self.cph = mh, dh, kh, fh, cph
        self.cvh = cvh if cvh is not None else np.zeros_like(cph)

    def transfer(self, s):
        return (self.cph + s * self.cvh) @ np.linalg.solve(
            s * s * self.mh + s * self.dh + self.kh, self.fh)

    def first_order(self):
        """Reading A6: (A, B, C) of the first-order realisation."""
        r = self.mh.shape[0]
        a = np.block([[np.zeros((r, r)), np.eye(r)],
                      [-np.linalg.solve(self.mh, self.kh), -np.linalg.solve(self.mh, self.dh)]])
        b = np.vstack([np.zeros_like(self.fh), np.linalg.solve(self.mh, self.fh)])
        c = np.hstack([self.cph, self.cvh])
        return a, b, c


def h2_norm_first_order(a, b, c):
    """||C (sI - A)^{-1} B||_H2 from the controllability Gramian P,
    A P + P A^T + B B^T = 0: the norm is sqrt(trace(C P C^T))."""
    p = sla.solve_continuous_lyapunov(a, -b @ b.T)
    return float(np.sqrt(max(np.trace(c @ p @ c.T), 0.0)))


def h2_distance(ma, mb=None):
    """||H_a - H_b||_H2 (mb None: ||H_a||_H2), from the realisation of the
    difference: block-diagonal A, stacked B, C = [C_a, -C_b]."""
    aa, ba, ca = ma.first_order()
    if mb is None:
        return h2_norm_first_order(aa, ba, ca)
    ab, bb, cb = mb.first_order()
    a = sla.block_diag(aa, ab)
    b = np.vstack([ba, bb])
    c = np.hstack([ca, -cb])
    return h2_norm_first_order(a, b, c)


def reduce(mv, kv, alpha, beta, f, cp, cv, v):
    """The reduced model of eq. (1.4) on the basis v (n x r)."""
    mh, dh, kh, fh, cph = moments.project(mv, kv, alpha, beta, f, cp, v)
    cvh = cv @ v if cv is not None else None
    return Model(mh, dh, kh, fh, cph, cvh)


def airga(mv, kv, alpha, beta, f, cp, cv, shifts0, rmax, tol_outer=1e-6, tol_inner=1e-6,
          max_outer=10, solve=None):
    """Algorithm 1 with readings A1-A6.

    mv, kv: sparse n x n M and K (D = alpha M + beta K); f: n x m; cp, cv:
    p x n (cv may be None); shifts0: the l initial expansion points.
    solve(s, rhs) returns K(s)^{-1} rhs (default: sparse LU).
    Returns (V, model, history): history holds one dict per outer
    iteration with its expansion points, sigma sequence, J, moment errors,
    intermediate H2 changes, final model and relative H2 change.
    """
    if solve is None:
        def solve(s, rhs):
            ks = (s * s + alpha * s) * mv + (1.0 + beta * s) * kv
            return spla.splu(ks.tocsc()).solve(rhs)
    n, m = f.shape
    shifts = np.asarray(shifts0, dtype=float)
    l = len(shifts)
    jmax = rmax // m
    if jmax < 1:
        raise ValueError("r_max below the input count")
    history = []
    prev_final = None
    v = None
    for _z in range(max_outer):
        # solves at every expansion point, then the thin QR of each
        xs = [moments.thin_qr(solve(s, f))[0] for s in shifts]
        vs = []
        errors = None
        sigmas = []
        step_errors = []
        inner_changes = []
        prev_int = None
        j = 1
        while j < jmax:
            q = 0 if errors is None else int(np.argmax(errors))          # A1
            sigmas.append(q)
            vs.append(xs[q] / np.linalg.norm(xs[q]))
            xs[q] = -solve(shifts[q], mv @ vs[-1])                       # A2
            errors, norms = [], []
            for i in range(l):
                before = np.linalg.norm(xs[i])
                xs[i], _, fro = moments.global_orth(vs, xs[i])
                errors.append(fro / before)
                norms.append(fro)
            errors = np.array(errors)
            step_errors.append(errors.copy())
            w, _ = moments.thin_qr(np.hstack([xs[i] / norms[i] for i in range(l)]))
            model_int = reduce(mv, kv, alpha, beta, f, cp, cv, w)
            if prev_int is not None:
                change = h2_distance(model_int, prev_int) / h2_distance(model_int)  # A5
                inner_changes.append(change)
                if change < tol_inner:
                    j += 1
                    break
            prev_int = model_int
            j += 1
        # J = j: the last block from the largest moment error
        q = 0 if errors is None else int(np.argmax(errors))
        sigmas.append(q)
        vs.append(xs[q] / np.linalg.norm(xs[q]))
        v, _ = moments.thin_qr(np.hstack(vs))
        final = reduce(mv, kv, alpha, beta, f, cp, cv, v)
        change = None
        if prev_final is not None:
            change = h2_distance(final, prev_final) / h2_distance(final)
        history.append(dict(shifts=shifts.copy(), sigmas=sigmas, J=len(vs),
                            errors=None if errors is None else errors.copy(),
                            step_errors=step_errors,
                            inner_changes=inner_changes, model=final, change=change))
        prev_final = final
        if change is not None and change < tol_outer:
            break
        shifts = next_shifts(qep_poles(final.mh, final.dh, final.kh), l)   # A4
    return v, prev_final, history
