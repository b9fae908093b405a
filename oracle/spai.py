"""SPAI preconditioner and its cheap update (test infrastructure only).

Build (Section 3.1, eq. (3.1)): the right approximate inverse minimises
||I - K P||_F over matrices P with a prescribed sparsity pattern; the square
of the Frobenius norm splits into n independent least-squares problems, one
per column, min ||e_j - K p_j||_2.  The paper reaches each column's minimum
iteratively (a minimal-residual loop stopped at a tolerance); here each column
problem is solved exactly, which is the limit that loop approaches, with the
pattern fixed to the structural pattern of K(s):
    J = pattern of column j (allowed nonzeros of p_j),
    I = rows where K(:, J) has nonzeros,
    p_J = argmin || e_j(I) - K(I, J) p ||_2   (a library least-squares solve).
Rows outside I are zero on both sides, so this is the full column problem.

Readings fixed here (each listed in the design notes):
  * equilibrate: the column problems are posed for Khat = S K S with
    S = diag(K)^{-1/2}; the result is mapped back as P = S Phat S.
  * symmetrize (on by default): Phat is replaced by (Phat + Phat^T) / 2
    before mapping back, so the preconditioner handed to CG is symmetric.
    The average can be indefinite (on the cantilever, at the free tip), so CG
    uses a step and direction update that stay defined then; without the
    average the fixed-pattern right SPAI stalls CG on the stiff literal beam.

Update (Section 3.2): instead of a new SPAI for K_new, find Q minimising
||K_old - K_new Q||_F column by column, starting from Q = alpha I with alpha
the minimiser of ||K_old - alpha K_new||_F, i.e.
    alpha = (1/2) trace(K_old^T K_new + K_new^T K_old) / trace(K_new^T K_new).
A column whose residual at the start, k_old_j - alpha K_new e_j, is already
within the tolerance keeps q_j = alpha e_j (the update algorithm never enters
its inner loop for it); every other column is solved exactly on the pattern.
The tolerance is read relative to ||k_old_j||.  With equilibration both
matrices are scaled by the *new* diagonal, Khat_x = S_new K_x S_new, and the
factor is mapped back as Q = S_new Qhat S_new^{-1}, so that K_new Q ~ K_old.
The preconditioner after updates is the chain Q_z ... Q_2 P_1, applied factor
by factor and never multiplied out (Section 3.2, last paragraph).

Minimal-residual mode (mr_iters > 0): each column is reached the way the
paper's iterative algorithms reach it (Algorithms 2 and 4) instead of by the
exact solve: starting from p_j = alpha e_j (q_j = alpha e_j), a sequence of
minimal-residual steps on the column objective ||t - K p_j|| with t = e_j
(k_old_j), each an exact line search along the current residual, until the
residual is within tol ||t||.  In the paper P (Q) stays alpha I inside the
column loop (its write-back is not part of the algorithm), so the direction
is alpha times the residual; it is restricted to the pattern J of column j,
which keeps p_j on the pattern of K(s) (the structural reading above), and
the residual then lives on the rows I, so the iteration runs on the column's
local block exactly.  It is capped at mr_iters steps, because on a fixed
pattern the residual may never reach tol.  The build's alpha is
trace(Khat) / trace(Khat Khat^T) of the matrix whose inverse is sought.

Pattern control (lfil > 0, minimal-residual mode only): the sparsity-pattern
step that the paper leaves out of Algorithms 2 and 4 (and says can be added)
is the one of Chow and Saad's minimal-residual iteration: the direction takes
the entries of t = alpha r on the current pattern of p_j, and while that
pattern holds fewer than lfil entries it also admits the largest remaining
entry of t in absolute value.  Readings: the pattern starts as {j} (the start
alpha e_j); the remaining entries are those of J outside the current pattern,
so p_j stays on the structural pattern of K(s) and the factor keeps its
layout; entries within a relative PICK_TIE (1e-8) of the largest count as
equal and the lowest row wins, so that rounding (two correct evaluations of
a small entry of r can differ by far more than eps relative) never decides
the pattern; an entry that is exactly zero is never admitted.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class Factor:
    """One preconditioner factor on the structural pattern of K(s)."""

    values: np.ndarray        # CSR-ordered values of the mapped-back factor
    hat: np.ndarray           # CSR-ordered values before symmetrisation / mapping
    objective: np.ndarray     # per column: least-squares residual norm (nan = not computed)
    skipped: np.ndarray       # per column: True when kept at alpha e_j (update only)
    alpha: float              # initial scaling (build: trace formula of Alg. 2; update: Alg. 4)
    cols: np.ndarray          # columns actually computed
    pattern: tuple            # (n, row_ptr, col_idx)
    iters: np.ndarray = None  # minimal-residual mode: steps per column
    margin: np.ndarray = None  # closest approach of ||r|| / (tol ||t||) to 1 over
                               # the column's tolerance tests (update: the skip
                               # test; minimal-residual mode: every test)
    pick_margin: np.ndarray = None  # pattern control: per column, the smallest
                                    # distance of a pattern decision from its
                                    # tie threshold

    def matrix(self) -> sp.csr_matrix:
        n, rp, ci = self.pattern
        m = sp.csr_matrix((self.values, ci, rp), shape=(n, n))
        return m

    @property
    def scalar_only(self) -> bool:
        return bool(np.all(self.skipped))


def _csc_positions(n, row_ptr, col_idx):
    """For the CSC ordering of the pattern: (indptr, row indices, CSR position)."""
    nnz = len(col_idx)
    pos = sp.csr_matrix((np.arange(1, nnz + 1, dtype=np.int64), col_idx, row_ptr),
                        shape=(n, n)).tocsc()
    pos.sort_indices()
    return pos.indptr, pos.indices, pos.data - 1


def mirror_positions(n, row_ptr, col_idx):
    """CSR position of entry (c, r) for every CSR entry (r, c); requires a
    structurally symmetric pattern."""
    nnz = len(col_idx)
    t = sp.csr_matrix((np.arange(1, nnz + 1, dtype=np.int64), col_idx, row_ptr),
                      shape=(n, n)).T.tocsr()
    t.sort_indices()
    if not (np.array_equal(t.indptr, np.asarray(row_ptr)) and
            np.array_equal(t.indices, np.asarray(col_idx))):
        raise ValueError("pattern is not structurally symmetric")
    return t.data - 1


def _rows_of(row_ptr, n):
    return np.repeat(np.arange(n), np.diff(row_ptr))


def _column_problem(indptr, rows, vals, j):
    """I, J and the dense block Khat(I, J) for column j (CSC arrays)."""
    jj = rows[indptr[j]:indptr[j + 1]]
    parts = [rows[indptr[k]:indptr[k + 1]] for k in jj]
    ii = np.unique(np.concatenate(parts))
    blk = np.zeros((len(ii), len(jj)), dtype=vals.dtype)
    for t, k in enumerate(jj):
        r = rows[indptr[k]:indptr[k + 1]]
        blk[np.searchsorted(ii, r), t] = vals[indptr[k]:indptr[k + 1]]
    return ii, jj, blk


def _scaled_values(a_val, rows, cols, s_row, s_col):
    return a_val * s_row[rows] * s_col[cols]


PICK_TIE = 1e-8


def _pick_entry(tv, inside, tie=PICK_TIE):
    """Pattern control: the position of the largest |tv| outside the
    current pattern (`inside`), ties within a relative `tie` going to the
    lowest position; None when every remaining entry is zero.  Also returns
    how far the decision is from flipping: the smallest distance of any
    remaining |tv_u| / max from the tie threshold 1 - tie (1.0 when there
    is nothing to compare)."""
    cand = np.flatnonzero(~inside)
    if len(cand) == 0:
        return None, 1.0
    mag = np.abs(tv[cand])
    top = mag.max()
    if not top > 0:
        return None, 1.0
    ratio = mag / top
    pick = cand[np.flatnonzero(ratio >= 1.0 - tie)[0]]
    return int(pick), float(np.min(np.abs(ratio - (1.0 - tie))))


def _mr_column(blk, rhs, jpos, p, alpha, tol, mr_iters, lfil=0, jself=None):
    """The paper's iterative column solve (Algorithms 2 and 4) on one
    column's local problem, minimise f(p) = ||t - B p||^2 with
    B = blk = Khat(I, J) and t = rhs = t(I), from the start p on J.

    Each step is an exact line search of f: the direction is the current
    residual t - B p scaled by alpha and restricted to the pattern J
    (jpos = positions of J in I), d = alpha (t - B p)|_J, and
    f(p + a d) = f(p) - 2 a <t - B p, B d> + a^2 ||B d||^2 is smallest at
    a = <t - B p, B d> / ||B d||^2.  The residual is formed from its
    definition at every step.  The loop stops once ||t - B p|| <= tol ||t||,
    after mr_iters steps, or when B d = 0 (no descent left along d).
    With lfil > 0 the direction is confined to the current pattern of p,
    which starts as {jself} (the position of j in J) and admits the largest
    remaining entry of alpha r|_J at each step while it holds fewer than
    lfil entries (pattern control, see the module notes).
    Returns (p, ||t - B p||, steps, margin, pick_margin), margin = the
    closest approach of ||t - B p|| / (tol ||t||) to 1 over the stopping
    tests taken, pick_margin = the smallest distance of a pattern decision
    from its tie threshold (inf without pattern control)."""
    thr = tol * np.linalg.norm(rhs)
    margin = np.inf
    pick_margin = np.inf
    steps = 0
    inside = None
    if lfil > 0:
        inside = np.zeros(len(jpos), bool)
        inside[jself] = True
    while True:
        res = rhs - blk @ p
        nres = np.linalg.norm(res)
        if thr > 0:
            margin = min(margin, abs(nres / thr - 1.0))
        if nres <= thr or steps >= mr_iters:
            break
        d = alpha * res[jpos]
        if inside is not None:
            if inside.sum() < lfil:
                u, pm = _pick_entry(d, inside)
                pick_margin = min(pick_margin, pm)
                if u is not None:
                    inside[u] = True
            d = np.where(inside, d, 0.0)
        bd = blk @ d
        curv = bd @ bd
        if not curv > 0:
            break
        p = p + ((res @ bd) / curv) * d
        steps += 1
    return p, float(np.linalg.norm(rhs - blk @ p)), steps, margin, pick_margin


def spai_build(a: sp.csr_matrix, *, equilibrate=True, symmetrize=True, cols=None,
               mr_iters=0, tol=0.01, lfil=0) -> Factor:
    """SPAI of K(s) on its own structural pattern (eq. (3.1)).

    K(s) may be complex (a complex expansion point): the column problems are
    then complex least-squares problems, S = diag(K)^{-1/2} takes the
    principal square root, and the symmetric average is (Phat + Phat^T) / 2
    with the plain transpose, so that the factor stays complex symmetric like
    K(s) (conjugate orthogonal CG needs that).  The minimal-residual mode is
    real only.

    ``cols`` restricts the computation to a subset of columns (sampled checks
    at large n); the returned values are then only meaningful for those.
    ``mr_iters`` > 0 selects the minimal-residual loop of Algorithm 2 with
    stopping tolerance ``tol`` instead of the exact column solves, and
    ``lfil`` > 0 adds its pattern control (at most lfil entries per column).
    """
    if lfil < 0 or (lfil > 0 and mr_iters <= 0):
        raise ValueError("lfil applies to the minimal-residual mode")
    n = a.shape[0]
    rp, ci = a.indptr, a.indices
    rows = _rows_of(rp, n)
    d = a.diagonal()
    s = 1.0 / np.sqrt(d) if equilibrate else np.ones(n)
    khat = _scaled_values(a.data, rows, ci, s, s)
    indptr, crow, cpos = _csc_positions(n, rp, ci)
    cval = khat[cpos]
    hat = np.full(len(ci), np.nan)
    obj = np.full(n, np.nan)
    iters = np.zeros(n, np.int64)
    margin = np.full(n, np.inf)
    pick = np.full(n, np.inf)
    todo = np.arange(n) if cols is None else np.asarray(cols)
    cplx = np.iscomplexobj(khat)
    if cplx:
        if mr_iters > 0:
            raise ValueError("the minimal-residual mode is for real shifts only")
        hat = np.full(len(ci), np.nan, dtype=complex)
    if mr_iters > 0:
        kh = sp.csr_matrix((khat, ci, rp), shape=(n, n))
        alpha_hat = float(kh.diagonal().sum() / (kh @ kh.T).diagonal().sum())
    for j in todo:
        ii, jj, blk = _column_problem(indptr, crow, cval, j)
        rhs = (ii == j).astype(np.float64)
        if mr_iters > 0:
            p0 = alpha_hat * (jj == j).astype(np.float64)
            p, obj[j], iters[j], margin[j], pick[j] = _mr_column(
                blk, rhs, np.searchsorted(ii, jj), p0, alpha_hat, tol, mr_iters, lfil,
                int(np.flatnonzero(jj == j)[0]))
        else:
            p, *_ = np.linalg.lstsq(blk, rhs, rcond=None)
            obj[j] = np.linalg.norm(rhs - blk @ p)
        hat[cpos[indptr[j]:indptr[j + 1]]] = p
    if symmetrize:
        mir = mirror_positions(n, rp, ci)
        sym = 0.5 * (hat + hat[mir])
    else:
        sym = hat
    values = _scaled_values(sym, rows, ci, s, s)
    # Alg. 2's initial scaling: trace(K) / trace(K K^T) (reported, not used by
    # the exact column solves; the minimal-residual loop uses it for Khat).
    if cplx:
        # complex: the minimiser of ||I - alpha K||_F is trace(K^H) / ||K||_F^2
        alpha = complex(np.conj(a.diagonal()).sum() / np.vdot(a.data, a.data).real)
    else:
        alpha = alpha_hat if mr_iters > 0 else float(a.diagonal().sum() /
                                                     (a @ a.T).diagonal().sum())
    return Factor(values=values, hat=hat, objective=obj, skipped=np.zeros(n, bool),
                  alpha=alpha, cols=todo, pattern=(n, rp, ci),
                  iters=iters if mr_iters > 0 else None, margin=margin if mr_iters > 0 else None,
                  pick_margin=pick if lfil > 0 else None)


def update_alpha(k_old: sp.csr_matrix, k_new: sp.csr_matrix):
    """Minimiser of ||K_old - alpha K_new||_F as derived in Section 3.2.

    For complex matrices (complex expansion points) alpha ranges over the
    complex numbers and the minimiser is <K_new, K_old> / <K_new, K_new>
    with the Hermitian inner product <A, B> = trace(A^H B); for real
    matrices this is the formula of Section 3.2."""
    if np.iscomplexobj(k_old.data) or np.iscomplexobj(k_new.data):
        num = (k_new.conj().T @ k_old).diagonal().sum()
        den = (k_new.conj().T @ k_new).diagonal().sum().real
        return complex(num / den)
    num = 0.5 * ((k_old.T @ k_new).diagonal().sum() + (k_new.T @ k_old).diagonal().sum())
    return float(num / (k_new.T @ k_new).diagonal().sum())


def spai_update(a_old: sp.csr_matrix, a_new: sp.csr_matrix, *, tol=0.01, equilibrate=True,
                cols=None, mr_iters=0, lfil=0) -> Factor:
    """Q with K_new Q ~ K_old (Section 3.2), on the structural pattern;
    ``mr_iters`` > 0 selects the minimal-residual loop of Algorithm 4, and
    ``lfil`` > 0 its pattern control.  Complex K_old, K_new (complex
    expansion points): complex alpha (update_alpha), S_new from the principal
    square root, complex column least squares; the minimal-residual mode is
    real only."""
    if lfil < 0 or (lfil > 0 and mr_iters <= 0):
        raise ValueError("lfil applies to the minimal-residual mode")
    n = a_new.shape[0]
    rp, ci = a_new.indptr, a_new.indices
    if not (np.array_equal(a_old.indptr, rp) and np.array_equal(a_old.indices, ci)):
        raise ValueError("K_old and K_new must share one pattern")
    rows = _rows_of(rp, n)
    cplx = np.iscomplexobj(a_new.data) or np.iscomplexobj(a_old.data)
    if cplx and mr_iters > 0:
        raise ValueError("the minimal-residual mode is for real shifts only")
    dt = complex if cplx else np.float64
    d = a_new.diagonal().astype(dt)
    s = 1.0 / np.sqrt(d) if equilibrate else np.ones(n, dtype=dt)
    new_hat = _scaled_values(a_new.data.astype(dt), rows, ci, s, s)
    old_hat = _scaled_values(a_old.data.astype(dt), rows, ci, s, s)
    k_new_hat = sp.csr_matrix((new_hat, ci, rp), shape=(n, n))
    k_old_hat = sp.csr_matrix((old_hat, ci, rp), shape=(n, n))
    alpha = update_alpha(k_old_hat, k_new_hat)
    indptr, crow, cpos = _csc_positions(n, rp, ci)
    cnew = new_hat[cpos]
    cold = old_hat[cpos]
    hat = np.full(len(ci), np.nan, dtype=dt)
    obj = np.full(n, np.nan)
    skipped = np.zeros(n, bool)
    iters = np.zeros(n, np.int64)
    margin = np.full(n, np.inf)
    pick = np.full(n, np.inf)
    todo = np.arange(n) if cols is None else np.asarray(cols)
    for j in todo:
        sl = slice(indptr[j], indptr[j + 1])
        jj = crow[sl]
        kold_j = cold[sl]
        r0 = kold_j - alpha * cnew[sl]
        thr = tol * np.linalg.norm(kold_j)
        if thr > 0:
            margin[j] = abs(np.linalg.norm(r0) / thr - 1.0)
        if np.linalg.norm(r0) <= thr:
            skipped[j] = True
            q = alpha * (jj == j).astype(dt)
            obj[j] = np.linalg.norm(r0)
        else:
            ii, jj2, blk = _column_problem(indptr, crow, cnew, j)
            rhs = np.zeros(len(ii), dtype=dt)
            jpos = np.searchsorted(ii, jj)
            rhs[jpos] = kold_j
            if mr_iters > 0:
                q0 = alpha * (jj == j).astype(np.float64)
                q, obj[j], iters[j], m2, pick[j] = _mr_column(
                    blk, rhs, jpos, q0, alpha, tol, mr_iters, lfil,
                    int(np.flatnonzero(jj == j)[0]))
                margin[j] = min(margin[j], m2)
            else:
                q, *_ = np.linalg.lstsq(blk, rhs, rcond=None)
                obj[j] = np.linalg.norm(rhs - blk @ q)
        hat[cpos[sl]] = q
    # Q = S Qhat S^{-1}
    values = hat * s[rows] / s[ci]
    return Factor(values=values, hat=hat, objective=obj, skipped=skipped, alpha=alpha,
                  cols=todo, pattern=(n, rp, ci),
                  iters=iters if mr_iters > 0 else None, margin=margin,
                  pick_margin=pick if lfil > 0 else None)


def chain_apply(factors, r: np.ndarray) -> np.ndarray:
    """z = Q_z ( ... Q_2 ( P_1 r ) ): ``factors`` lists P_1 first, then each
    update factor in the order it was computed; only products with vectors
    are formed."""
    z = np.asarray(r)
    if not np.iscomplexobj(z):
        z = z.astype(np.float64)
    for fac in factors:
        z = fac.matrix() @ z
    return z
