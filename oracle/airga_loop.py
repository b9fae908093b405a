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
taken here are:
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


def moment_error(vs, x_before, x_after):
    """Reading A1: the part of the newest moment block that the basis
    V_1..V_j does not hold yet, as a fraction of the block:
    ||x_after||_F / ||x_before||_F (x_after = x_before orthogonalised against
    the trace-orthonormal blocks vs)."""
    return float(np.linalg.norm(x_after) / np.linalg.norm(x_before))


def next_point(errors):
    """Reading A1: the expansion point whose moment error is largest (the
    first such index on a tie); before any error exists, the first point."""
    if errors is None:
        return 0
    errors = np.asarray(errors, dtype=float)
    return int(np.flatnonzero(errors == errors.max())[0])


def relative_change(new, old):
    """Reading A5: ||H_new - H_old||_H2 / ||H_new||_H2."""
    return h2_distance(new, old) / h2_distance(new)


def airga(mv, kv, alpha, beta, f, cp, cv, shifts0, rmax, tol_outer=1e-6, tol_inner=1e-6,
          max_outer=10, solve=None):
    """AIRGA's outer iteration (Algorithm 1) under readings A1-A6.

    mv, kv: sparse n x n M and K (D = alpha M + beta K); f: n x m; cp, cv:
    p x n (cv may be None); shifts0: the l initial expansion points.
    solve(s, rhs) returns K(s)^{-1} rhs (default: sparse LU).

    One outer iteration: the state X(s_i) = K(s_i)^{-1} F at every point,
    each replaced by its thin QR factor; then the moment loop, which grows
    the basis one n x m block at a time.  A step takes the point sigma with
    the largest moment error (A1), appends its current block, normalised in
    the Frobenius norm, as V_j, replaces that point's block by its next
    moment -K(sigma)^{-1} M V_j, and orthogonalises every point's block
    against V_1..V_j in the trace inner product, which gives the new moment
    errors.  The normalised blocks span an intermediate reduced model; the
    loop ends when that model's relative H2 change drops below tol_inner (A5)
    or the basis reaches floor(rmax / m) blocks (A3), the last block being
    taken, again by the largest moment error, after the loop.  The final
    basis is the thin QR of [V_1 .. V_J], the reduced model is its Galerkin
    projection (eq. (1.4)), and the next expansion points come from the
    reduced model's poles (A4).  The outer loop ends when the final model's
    relative H2 change drops below tol_outer, or after max_outer iterations.

    Returns (V, model, history): history holds one dict per outer
    iteration with its expansion points, sigma sequence (indices), J,
    moment errors after each step, the intermediate models and their
    relative H2 changes, the final model and its relative H2 change.
    """
    if solve is None:
        def solve(s, rhs):
            ks = (s * s + alpha * s) * mv + (1.0 + beta * s) * kv
            return spla.splu(ks.tocsc()).solve(rhs)
    n, m = f.shape
    shifts = np.asarray(shifts0, dtype=float)
    l = len(shifts)
    blocks_max = rmax // m
    if blocks_max < 1:
        raise ValueError("r_max below the input count")
    history = []
    final_prev = None
    basis = None
    for _ in range(max_outer):
        state = [moments.thin_qr(solve(s, f))[0] for s in shifts]
        vs, sigmas, step_errors, inner_models, inner_changes = [], [], [], [], []
        errors = None

        def take_block():
            q = next_point(errors)
            sigmas.append(q)
            vs.append(state[q] / np.linalg.norm(state[q]))
            return q

        while len(vs) + 1 < blocks_max:
            q = take_block()
            state[q] = -solve(shifts[q], mv @ vs[-1])
            before = [x.copy() for x in state]
            fro = []
            for i in range(l):
                state[i], _, nrm = moments.global_orth(vs, state[i])
                fro.append(nrm)
            errors = np.array([moment_error(vs, b, x) for b, x in zip(before, state)])
            step_errors.append(errors.copy())
            w, _ = moments.thin_qr(np.hstack([state[i] / fro[i] for i in range(l)]))
            inner_models.append(reduce(mv, kv, alpha, beta, f, cp, cv, w))
            if len(inner_models) > 1:
                change = relative_change(inner_models[-1], inner_models[-2])
                inner_changes.append(change)
                if change < tol_inner:
                    break
        take_block()
        basis, _ = moments.thin_qr(np.hstack(vs))
        final = reduce(mv, kv, alpha, beta, f, cp, cv, basis)
        change = None if final_prev is None else relative_change(final, final_prev)
        history.append(dict(shifts=shifts.copy(), sigmas=sigmas, J=len(vs),
                            errors=None if errors is None else errors.copy(),
                            step_errors=step_errors, inner_models=inner_models,
                            inner_changes=inner_changes, model=final, change=change))
        final_prev = final
        if change is not None and change < tol_outer:
            break
        shifts = next_shifts(qep_poles(final.mh, final.dh, final.kh), l)   # A4
    return basis, final_prev, history
