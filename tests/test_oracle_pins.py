"""Pins of the CPU oracle against facts the paper and the mathematics fix.

None of these re-types an oracle formula: each checks the oracle against a
closed form, an invariant, a special case that reduces to a textbook or
library routine, or brute force on tiny inputs.
"""
import fractions
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import direct, moments, pcg, pencil, spai
from synthetic import beam

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "cantilever.json")


def golden():
    with open(GOLDEN) as fh:
        return json.load(fh)


def small_pencil(n_el=20, surrogate=True, lu=(0.5, 2.0), seed=3):
    return beam.make_beam(n_el, ei_loguniform=lu, surrogate=surrogate, seed=seed)


# ----------------------------------------------------------------- generator

def test_beam_pattern_shape_and_symmetry():
    p = beam.make_beam(37)
    n = p.n
    assert n == 74 and p.nnz == 6 * n - 8
    m, k = beam.pencil_dense(p)
    assert np.array_equal(m, m.T) and np.array_equal(k, k.T)
    for r in range(n):
        c = p.col_idx[p.row_ptr[r]:p.row_ptr[r + 1]]
        assert np.all(np.diff(c) > 0)
    assert np.all(np.linalg.eigvalsh(m) > 0) and np.all(np.linalg.eigvalsh(k) > 0)


def test_beam_eigenvalues_converge_to_euler_bernoulli():
    g = golden()["free_vibration"]
    p = beam.make_beam(40)
    m, k = beam.pencil_dense(p)
    w = sla.eigh(k, m, eigvals_only=True)[:3]
    exact = np.array(g["beta_L"]) ** 4
    # Hermite cubics converge as h^4; at 40 elements the first three modes agree to:
    assert abs(w[0] / exact[0] - 1) < 1e-8
    assert abs(w[1] / exact[1] - 1) < 1e-6
    assert abs(w[2] / exact[2] - 1) < 1e-5


def test_beam_heterogeneous_ei_is_seeded():
    a = beam.make_beam(50, ei_loguniform=(0.5, 2.0), seed=7)
    b = beam.make_beam(50, ei_loguniform=(0.5, 2.0), seed=7)
    c = beam.make_beam(50, ei_loguniform=(0.5, 2.0), seed=8)
    assert np.array_equal(a.k_val, b.k_val) and not np.array_equal(a.k_val, c.k_val)
    assert a.ei.min() >= 0.5 and a.ei.max() <= 2.0


# ------------------------------------------------------------ shifted operator

def test_shifted_operator_matches_expanded_form():
    p = small_pencil()
    m, k = beam.pencil_dense(p)
    for s in (0.5, 3.0, 1e3):
        a = pencil.shifted_operator(p, s).toarray()
        other = (s * s + p.alpha * s) * m + (1 + p.beta * s) * k
        assert np.allclose(a, other, rtol=1e-14, atol=1e-14 * np.abs(other).max())


def test_shifted_operator_spd_for_positive_shift():
    p = small_pencil(surrogate=False)
    for s in (1e-3, 1.0, 1e4):
        a = pencil.shifted_operator(p, s).toarray()
        assert np.all(np.linalg.eigvalsh(a) > 0)
        np.linalg.cholesky(a)


def test_shift_dd_is_exactly_rounded():
    """Double-double K(s) entries equal the exact rational value to ~2^-100."""
    p = small_pencil(n_el=4)
    s = 37.0 / 3.0
    hi, lo, w = direct.shifted_band_dd(p, s)
    mb, _ = direct.lower_band(pencil.csr(p.n, p.row_ptr, p.col_idx, p.m_val), w)
    kb, _ = direct.lower_band(pencil.csr(p.n, p.row_ptr, p.col_idx, p.k_val), w)
    F = fractions.Fraction
    fs, fa, fb = F(s), F(p.alpha), F(p.beta)
    for idx in np.ndindex(mb.shape):
        exact = fs * fs * F(mb[idx]) + fs * (fa * F(mb[idx]) + fb * F(kb[idx])) + F(kb[idx])
        got = F(hi[idx]) + F(lo[idx])
        if exact == 0:
            assert got == 0
        else:
            assert abs((got - exact) / exact) < F(1, 2 ** 100)


def test_frobenius_diagnostics_dense():
    p = small_pencil()
    d1, d2 = pencil.frobenius_diagnostics(p, 2.0, 2.5)
    a1 = pencil.shifted_operator(p, 2.0).toarray()
    a2 = pencil.shifted_operator(p, 2.5).toarray()
    assert np.isclose(d1, np.linalg.norm(np.eye(p.n) - a2, "fro"), rtol=1e-13)
    assert np.isclose(d2, np.linalg.norm(a1 - a2, "fro"), rtol=1e-13)


# ------------------------------------------------------------ reference solve

def _random_band_spd(n, w, rng):
    a = np.zeros((n, n))
    for k in range(1, w + 1):
        v = rng.uniform(-1, 1, n - k)
        a += np.diag(v, k) + np.diag(v, -k)
    a += np.diag(np.abs(a).sum(1) + rng.uniform(0.1, 1.0, n))
    return a


@pytest.mark.parametrize("n,w", [(1, 0), (7, 1), (50, 3), (200, 4)])
def test_band_solve_matches_dense(n, w):
    rng = np.random.default_rng(n + w)
    a = _random_band_spd(n, w, rng)
    ab, ww = direct.lower_band(sp.csr_matrix(a), w)
    b = rng.standard_normal((3, n))
    x = direct.band_solve(ab, ww, b, "f64")
    xh, xl = direct.band_solve(ab, ww, b, "dd")
    ref = np.linalg.solve(a, b.T).T
    assert np.allclose(x, ref, rtol=1e-12, atol=1e-12)
    assert np.allclose(xh + xl, ref, rtol=1e-12, atol=1e-12)


def test_band_solve_dd_recovers_integer_solution_of_ill_conditioned_matrix():
    """Clamped biharmonic band [1 -4 6 -4 1]: kappa ~ n^4 (1e16 here); with an
    integer solution the right-hand side is exact in binary64, so the
    double-double solve must return it far below binary64's error."""
    n = 10_000
    a = sp.diags([np.ones(n - 2), -4 * np.ones(n - 1), 6 * np.ones(n), -4 * np.ones(n - 1),
                  np.ones(n - 2)], [-2, -1, 0, 1, 2], format="csr")
    a = a.tolil()
    a[0, 0] = 7  # clamped-end modification keeps it SPD
    a = a.tocsr()
    rng = np.random.default_rng(0)
    x = rng.integers(-1000, 1000, n).astype(np.float64)
    b = a @ x
    assert np.all(np.abs(b) < 2 ** 53)
    ab, w = direct.lower_band(a)
    xh, xl = direct.band_solve(ab, w, b, "dd")
    err_dd = np.abs(xh + xl - x).max() / np.abs(x).max()
    x64 = direct.band_solve(ab, w, b, "f64")
    err_64 = np.abs(x64 - x).max() / np.abs(x).max()
    assert err_dd < 1e-14
    assert err_64 > 1e3 * err_dd  # the binary64 solve is visibly worse here


@pytest.mark.parametrize("n_el", [64, 4096])
def test_static_cantilever_closed_form(n_el):
    """K w = e_tip gives w(x) = x^2 (3 - x) / 6, theta = x (2 - x) / 2 at every
    node (L = EI = 1; h = 2^-k so M, K are exact in binary64)."""
    g = golden()["static_tip_load"]
    p = beam.make_beam(n_el)
    f = beam.tip_load(p.n)
    x = direct.reference_solve(p, 0.0, f, "dd")[0]
    xs = np.arange(1, n_el + 1) / n_el
    assert abs(x[-2] - g["tip_deflection"]) < 1e-15
    assert abs(x[-1] - g["tip_rotation"]) < 1e-15
    assert np.allclose(x[0::2], xs * xs * (3 - xs) / 6, rtol=0, atol=1e-15)
    assert np.allclose(x[1::2], xs * (2 - xs) / 2, rtol=0, atol=1e-15)


def test_reference_solve_residual_and_precisions_agree_when_well_conditioned():
    p = beam.make_beam(2000, ei_loguniform=(0.5, 2.0), surrogate=True, seed=1)
    rng = np.random.default_rng(0)
    f, _ = beam.node_loads(p.n, 3, rng)
    for s in (1.0, 100.0):
        xd = direct.reference_solve(p, s, f, "dd")
        x64 = direct.reference_solve(p, s, f, "f64")
        assert np.linalg.norm(xd - x64) / np.linalg.norm(xd) < 1e-13
        hi, lo, w = direct.shifted_band_dd(p, s)
        r = direct.residual_dd(hi, w, f, xd, ab_lo=lo)
        anorm = np.abs(hi).sum(1).max() * 2
        assert np.linalg.norm(r) <= 1e-14 * anorm * np.linalg.norm(xd)


def test_reference_solve_rejects_indefinite():
    a = sp.csr_matrix(np.array([[1.0, 2.0], [2.0, 1.0]]))
    ab, w = direct.lower_band(a)
    with pytest.raises(np.linalg.LinAlgError):
        direct.band_solve(ab, w, np.ones(2), "f64")
    with pytest.raises(np.linalg.LinAlgError):
        direct.band_solve(ab, w, np.ones(2), "dd")


# ----------------------------------------------------------------------- SPAI

def _normal_eq_residual(a_hat, fac, j, rhs_col):
    """|| Khat(:,J)^T (rhs - Khat(:,J) p_J) || for column j (dense, small n)."""
    n = a_hat.shape[0]
    rp, ci = fac.pattern[1], fac.pattern[2]
    csc = sp.csr_matrix((fac.hat, ci, rp), shape=(n, n)).tocsc()
    jj = csc.indices[csc.indptr[j]:csc.indptr[j + 1]]
    pj = csc.data[csc.indptr[j]:csc.indptr[j + 1]]
    sub = a_hat[:, jj]
    res = rhs_col - sub @ pj
    return np.linalg.norm(sub.T @ res), np.linalg.norm(sub) * np.linalg.norm(res)


def _equilibrated(a):
    d = a.diagonal()
    s = 1 / np.sqrt(d)
    return (sp.diags(s) @ a @ sp.diags(s)).toarray(), s


@pytest.mark.parametrize("sur,s", [(True, 1.0), (True, 1e3), (False, 100.0)])
def test_spai_columns_are_least_squares_optimal(sur, s):
    p = small_pencil(surrogate=sur)
    a = pencil.shifted_operator(p, s)
    fac = spai.spai_build(a)
    ah, _ = _equilibrated(a)
    for j in range(p.n):
        g, scale = _normal_eq_residual(ah, fac, j, np.eye(p.n)[:, j])
        assert g <= 1e-12 * max(scale, 1e-300)


def test_spai_matches_full_column_lstsq():
    """Restricting column j's problem to the rows I loses nothing: it equals
    the least-squares fit over all n rows (rows outside I are zero)."""
    p = small_pencil(n_el=12)
    a = pencil.shifted_operator(p, 7.0)
    fac = spai.spai_build(a)
    ah, _ = _equilibrated(a)
    csc = sp.csr_matrix((fac.hat, a.indices, a.indptr), shape=a.shape).tocsc()
    for j in range(p.n):
        jj = csc.indices[csc.indptr[j]:csc.indptr[j + 1]]
        ref, *_ = np.linalg.lstsq(ah[:, jj], np.eye(p.n)[:, j], rcond=None)
        assert np.allclose(csc.data[csc.indptr[j]:csc.indptr[j + 1]], ref, rtol=1e-10, atol=1e-12)
        assert np.isclose(fac.objective[j], np.linalg.norm(np.eye(p.n)[:, j] - ah[:, jj] @ ref),
                          rtol=1e-10, atol=1e-14)


def test_spai_column_split_identity():
    """eq. (3.1): ||I - Khat Phat||_F^2 = sum_j ||e_j - Khat p_j||^2."""
    p = small_pencil(n_el=15)
    a = pencil.shifted_operator(p, 3.0)
    fac = spai.spai_build(a)
    ah, _ = _equilibrated(a)
    phat = sp.csr_matrix((fac.hat, a.indices, a.indptr), shape=a.shape).toarray()
    lhs = np.linalg.norm(np.eye(p.n) - ah @ phat, "fro") ** 2
    assert np.isclose(lhs, np.sum(fac.objective ** 2), rtol=1e-12)


def test_spai_full_pattern_is_exact_inverse():
    rng = np.random.default_rng(5)
    a = _random_band_spd(9, 8, rng)  # dense SPD
    fac = spai.spai_build(sp.csr_matrix(a), equilibrate=True)
    assert np.allclose(fac.matrix().toarray(), np.linalg.inv(a), rtol=1e-10, atol=1e-12)
    fac2 = spai.spai_build(sp.csr_matrix(a), equilibrate=False)
    assert np.allclose(fac2.matrix().toarray(), np.linalg.inv(a), rtol=1e-10, atol=1e-12)
    assert np.all(fac.objective < 1e-12)


def test_spai_block_diagonal_pattern_gives_block_inverse():
    rng = np.random.default_rng(6)
    blocks = [_random_band_spd(k, k - 1, rng) for k in (1, 2, 3, 4)]
    a = sla.block_diag(*blocks)
    fac = spai.spai_build(sp.csr_matrix(a))
    assert np.allclose(fac.matrix().toarray(), np.linalg.inv(a), rtol=1e-10, atol=1e-12)


def test_spai_one_by_one():
    fac = spai.spai_build(sp.csr_matrix(np.array([[4.0]])), equilibrate=False)
    assert fac.values[0] == 0.25
    assert fac.alpha == 0.25


def test_spai_initial_alpha_is_frobenius_minimiser():
    """Alg. 2's alpha = trace(K)/trace(K K^T) minimises ||I - alpha K||_F
    (checked by brute force over alpha)."""
    p = small_pencil(n_el=10)
    a = pencil.shifted_operator(p, 2.0)
    fac = spai.spai_build(a)
    ad = a.toarray()
    grid = fac.alpha * np.linspace(0.9, 1.1, 2001)
    vals = [np.linalg.norm(np.eye(p.n) - g * ad, "fro") for g in grid]
    assert abs(grid[int(np.argmin(vals))] / fac.alpha - 1) < 2e-4


def test_spai_symmetrize_is_symmetric():
    p = small_pencil()
    a = pencil.shifted_operator(p, 10.0)
    pm = spai.spai_build(a, symmetrize=True).matrix().toarray()
    assert np.allclose(pm, pm.T, rtol=0, atol=1e-14 * np.abs(pm).max())


def test_spai_sampled_columns_match_full():
    p = small_pencil(n_el=30)
    a = pencil.shifted_operator(p, 5.0)
    full = spai.spai_build(a)
    cols = np.array([0, 1, 17, 58, 59])
    part = spai.spai_build(a, cols=cols)
    assert np.allclose(part.objective[cols], full.objective[cols], rtol=0, atol=0)


# --------------------------------------------------------------- SPAI update

def test_update_same_shift_is_identity():
    p = small_pencil()
    a = pencil.shifted_operator(p, 4.0)
    q = spai.spai_update(a, a, tol=0.01)
    assert q.alpha == pytest.approx(1.0, abs=1e-15)
    assert q.scalar_only
    assert np.allclose(q.matrix().toarray(), np.eye(p.n), rtol=0, atol=1e-15)


def test_update_alpha_is_frobenius_minimiser():
    p = small_pencil(n_el=10)
    a_old = pencil.shifted_operator(p, 2.0)
    a_new = pencil.shifted_operator(p, 3.0)
    al = spai.update_alpha(a_old, a_new)
    o, nw = a_old.toarray(), a_new.toarray()
    grid = al * np.linspace(0.9, 1.1, 2001)
    vals = [np.linalg.norm(o - g * nw, "fro") for g in grid]
    assert abs(grid[int(np.argmin(vals))] / al - 1) < 2e-4


def test_update_columns_optimal_and_no_worse_than_start():
    p = small_pencil()
    a_old = pencil.shifted_operator(p, 2.0)
    a_new = pencil.shifted_operator(p, 6.0)
    q = spai.spai_update(a_old, a_new, tol=0.01)
    assert not q.scalar_only
    s = 1 / np.sqrt(a_new.diagonal())
    nh = (sp.diags(s) @ a_new @ sp.diags(s)).toarray()
    oh = (sp.diags(s) @ a_old @ sp.diags(s)).toarray()
    for j in range(p.n):
        start = np.linalg.norm(oh[:, j] - q.alpha * nh[:, j])
        assert q.objective[j] <= start * (1 + 1e-12)
        if not q.skipped[j]:
            g, scale = _normal_eq_residual(nh, q, j, oh[:, j])
            assert g <= 1e-12 * scale
    # K_new Q ~ K_old, with the column objectives splitting the Frobenius norm
    qh = sp.csr_matrix((q.hat, a_new.indices, a_new.indptr), shape=a_new.shape).toarray()
    assert np.isclose(np.linalg.norm(oh - nh @ qh, "fro") ** 2, np.sum(q.objective ** 2), rtol=1e-12)
    qm = q.matrix().toarray()
    assert np.allclose(a_new.toarray() @ qm, np.diag(1 / s) @ nh @ qh @ np.diag(1 / s), rtol=1e-12,
                       atol=1e-12 * np.abs(a_new.toarray() @ qm).max())


def test_update_tolerance_limits():
    p = small_pencil()
    a_old = pencil.shifted_operator(p, 2.0)
    a_new = pencil.shifted_operator(p, 2.2)
    assert spai.spai_update(a_old, a_new, tol=np.inf).scalar_only
    assert not np.any(spai.spai_update(a_old, a_new, tol=0.0).skipped)


def test_chain_apply_equals_explicit_product():
    p = small_pencil()
    a1 = pencil.shifted_operator(p, 2.0)
    a2 = pencil.shifted_operator(p, 3.0)
    a3 = pencil.shifted_operator(p, 5.0)
    p1 = spai.spai_build(a1)
    q2 = spai.spai_update(a1, a2, tol=0.0)
    q3 = spai.spai_update(a2, a3, tol=0.0)
    r = np.random.default_rng(0).standard_normal(p.n)
    explicit = q3.matrix().toarray() @ q2.matrix().toarray() @ p1.matrix().toarray() @ r
    assert np.allclose(spai.chain_apply([p1, q2, q3], r), explicit, rtol=1e-13, atol=1e-13)


# ------------------------------------------------------------------------ PCG

def _spd(n, rng):
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return q @ np.diag(rng.uniform(0.5, 4.0, n)) @ q.T


def test_pcg_matches_direct_solve():
    p = beam.make_beam(300, ei_loguniform=(0.5, 2.0), surrogate=True, seed=2)
    f = beam.tip_load(p.n)[0]
    for s in (1.0, 30.0, 1e4):
        a = pencil.shifted_operator(p, s)
        pm = spai.spai_build(a).matrix()
        res = pcg.pcg(lambda v: a @ v, lambda v: pm @ v, f, tol=1e-12, max_iter=2000)
        ref = direct.reference_solve(p, s, f[None], "dd")[0]
        assert res.status == pcg.CONVERGED
        assert np.linalg.norm(res.x - ref) / np.linalg.norm(ref) < 1e-9


def test_pcg_finite_termination_and_galerkin_orthogonality():
    rng = np.random.default_rng(1)
    n = 16
    a = _spd(n, rng)
    c = _spd(n, rng)  # symmetric positive definite preconditioner
    f = rng.standard_normal(n)
    res = pcg.pcg(lambda v: a @ v, lambda v: c @ v, f, tol=1e-13, max_iter=200, keep=True)
    assert res.status == pcg.CONVERGED and res.iters <= n + 3
    # residuals are orthogonal to earlier search directions (Ritz-Galerkin)
    for k in range(1, min(len(res.residuals), 8)):
        for i in range(k):
            pi, rk = res.directions[i], res.residuals[k]
            assert abs(pi @ rk) <= 1e-9 * np.linalg.norm(pi) * np.linalg.norm(rk)
    assert np.allclose(res.x, np.linalg.solve(a, f), rtol=1e-10)


def test_pcg_beta_forms_agree_for_symmetric_preconditioner():
    rng = np.random.default_rng(2)
    n = 40
    a = _spd(n, rng)
    c = _spd(n, rng)
    f = rng.standard_normal(n)
    hs = [pcg.pcg(lambda v: a @ v, lambda v: c @ v, f, tol=1e-30, max_iter=6, beta=b).history
          for b in ("flexible", "pr", "fr")]
    assert np.allclose(hs[0], hs[1], rtol=1e-9) and np.allclose(hs[0], hs[2], rtol=1e-9)


def test_pcg_statuses():
    rng = np.random.default_rng(3)
    n = 10
    a = _spd(n, rng)
    f = rng.standard_normal(n)
    eye = lambda v: v  # noqa: E731
    assert pcg.pcg(lambda v: a @ v, eye, f, tol=1e-14, max_iter=1).status == pcg.MAXIT
    bad = f.copy()
    bad[3] = np.nan
    assert pcg.pcg(lambda v: a @ v, eye, bad).status == pcg.NONFINITE
    assert pcg.pcg(lambda v: a @ v, lambda v: 0 * v, f).status == pcg.BREAKDOWN
    assert pcg.pcg(lambda v: -(a @ v), eye, f).status == pcg.BREAKDOWN
    z = pcg.pcg(lambda v: a @ v, eye, np.zeros(n))
    assert z.status == pcg.CONVERGED and z.iters == 0 and not np.any(z.x)


def test_pcg_warm_start_resumes():
    rng = np.random.default_rng(4)
    n = 30
    a = _spd(n, rng)
    f = rng.standard_normal(n)
    first = pcg.pcg(lambda v: a @ v, lambda v: v, f, tol=1e-3, max_iter=100)
    second = pcg.pcg(lambda v: a @ v, lambda v: v, f, tol=1e-12, max_iter=100, x0=first.x)
    assert second.status == pcg.CONVERGED
    assert np.allclose(second.x, np.linalg.solve(a, f), rtol=1e-9)


# -------------------------------------------------------------- moment matching

def test_galerkin_projection_interpolates_at_expansion_points():
    """V spanning X(s_i) and dX/ds(s_i) makes the reduced transfer function and
    its derivative match the full one there (Section 2 moment matching);
    H is evaluated by an independent dense solve."""
    p = beam.make_beam(60, ei_loguniform=(0.5, 2.0), surrogate=True, seed=4)
    m, k = beam.pencil_dense(p)
    f = beam.tip_load(p.n).T
    cp = f.T
    shifts = [1.5, 40.0, 900.0]
    xs = []
    for s in shifts:
        x0 = direct.reference_solve(p, s, f.T, "dd").T
        d = p.alpha * m + p.beta * k
        rhs = -((2 * s) * m + d) @ x0  # first moment, eq. (2.2) second line
        x1 = direct.reference_solve(p, s, rhs.T, "dd").T
        xs += [x0, x1]
    v = moments.orth_basis(xs)
    red = moments.project(m, k, p.alpha, p.beta, f, cp, v)

    def h_full(s):
        return cp @ np.linalg.solve(s * s * m + s * (p.alpha * m + p.beta * k) + k, f)

    for s in shifts:
        hs = h_full(s)
        assert np.allclose(moments.reduced_transfer(*red, s), hs, rtol=1e-9)
        e = 1e-4 * s
        dfull = (h_full(s + e) - h_full(s - e)) / (2 * e)
        dred = (moments.reduced_transfer(*red, s + e) - moments.reduced_transfer(*red, s - e)) / (2 * e)
        assert np.allclose(dred, dfull, rtol=1e-5)
    # away from the expansion points the reduced model is only approximate
    assert not np.allclose(moments.reduced_transfer(*red, 7.0), h_full(7.0), rtol=1e-9)


# ------------------------------------------------ moment sequence blocks

def test_pencil_apply_special_cases_match_dense_operators():
    p = small_pencil(15)
    m, k = beam.pencil_dense(p)
    ms = pencil.csr(p.n, p.row_ptr, p.col_idx, p.m_val)
    ks = pencil.csr(p.n, p.row_ptr, p.col_idx, p.k_val)
    x = np.random.default_rng(0).standard_normal((p.n, 3))
    # a = 1, b = 0 is M X (the moment right-hand side); the shift
    # coefficients give K(s) X, the pinned operator
    assert np.allclose(moments.pencil_apply(ms, ks, 1.0, 0.0, x), m @ x, rtol=0, atol=1e-13)
    s = 7.0
    a, b = s * s + p.alpha * s, 1.0 + p.beta * s
    ref = pencil.shifted_operator(p, s).toarray() @ x
    assert np.allclose(moments.pencil_apply(ms, ks, a, b, x), ref, rtol=1e-13, atol=1e-12)


def test_global_orth_hand_example_follows_the_loop_order():
    # n = 2, m = 1: V1 = e1, V2 = (1, 1)/sqrt 2, X = (3, 4).  In the
    # algorithm's order gamma_1 = 3, X = (0, 4), gamma_2 = <V2, (0, 4)> =
    # 2 sqrt 2, X = (-2, 2).  Products with the unchanged X (classical
    # Gram-Schmidt) would give gamma_2 = 7 / sqrt 2 instead.
    v1 = np.array([[1.0], [0.0]])
    v2 = np.array([[1.0], [1.0]]) / np.sqrt(2.0)
    x, g, f = moments.global_orth([v1, v2], np.array([[3.0], [4.0]]))
    assert np.allclose(g, [3.0, 2.0 * np.sqrt(2.0)], rtol=0, atol=1e-15)
    assert np.allclose(x, [[-2.0], [2.0]], rtol=0, atol=1e-15)
    assert abs(f - np.sqrt(8.0)) < 1e-15


def test_global_orth_orthonormal_basis_invariants():
    rng = np.random.default_rng(4)
    n, m, j = 50, 3, 5
    # blocks orthonormal in the trace inner product: orthonormal vec(V_t)
    q, _ = np.linalg.qr(rng.standard_normal((n * m, j)))
    vs = [q[:, t].reshape(n, m) for t in range(j)]
    for t in range(j):
        for u in range(j):
            assert abs(np.trace(vs[t].T @ vs[u]) - (t == u)) < 1e-13
    x0 = rng.standard_normal((n, m))
    x, g, f = moments.global_orth(vs, x0)
    # orthogonal to every block, coefficients are the plain projections,
    # and X0 is recovered from the result and the coefficients
    for t in range(j):
        assert abs(np.trace(vs[t].T @ x)) < 1e-12
        assert abs(g[t] - np.trace(vs[t].T @ x0)) < 1e-12
    assert np.allclose(x + sum(g[t] * vs[t] for t in range(j)), x0, rtol=0, atol=1e-13)
    assert abs(f - np.linalg.norm(x)) < 1e-13
    # Pythagoras in the trace inner product
    assert abs(f * f + np.sum(g * g) - np.linalg.norm(x0) ** 2) < 1e-10


def test_thin_qr_is_unique_factorisation_and_matches_gram_schmidt():
    rng = np.random.default_rng(5)
    w = rng.standard_normal((40, 6))
    q, r = moments.thin_qr(w)
    assert np.allclose(q.T @ q, np.eye(6), atol=1e-14)
    assert np.allclose(np.tril(r, -1), 0.0) and np.all(np.diag(r) > 0)
    assert np.allclose(q @ r, w, atol=1e-13)
    # brute force: classical Gram-Schmidt, column by column
    qg = np.zeros_like(w)
    rg = np.zeros((6, 6))
    for j in range(6):
        v = w[:, j].copy()
        for i in range(j):
            rg[i, j] = qg[:, i] @ w[:, j]
            v -= rg[i, j] * qg[:, i]
        rg[j, j] = np.linalg.norm(v)
        qg[:, j] = v / rg[j, j]
    assert np.allclose(q, qg, atol=1e-12) and np.allclose(r, rg, atol=1e-12)


# ------------------------------------------- SPAI minimal-residual mode

def test_spai_mr_one_step_closed_form():
    # one step of Algorithm 2 from p = alpha e_j, computed densely by hand:
    # r0 = e_j - alpha K e_j, d = alpha r0 on the pattern J, w = K d,
    # a = (r0, w) / (w, w), p = alpha e_j + a d
    p = small_pencil(8)
    a = pencil.shifted_operator(p, 3.0)
    k = a.toarray()
    f = spai.spai_build(a, equilibrate=False, symmetrize=False, mr_iters=1, tol=0.0)
    alpha = np.trace(k) / np.trace(k @ k.T)
    assert abs(f.alpha - alpha) < 1e-15 * abs(alpha)
    got = f.matrix().toarray()
    for j in (0, 5, p.n - 1):
        e = np.zeros(p.n)
        e[j] = 1.0
        r0 = e - alpha * k[:, j]
        mask = k[:, j] != 0
        mask |= np.arange(p.n) == j
        d = np.where(mask, alpha * r0, 0.0)
        w = k @ d
        step = (r0 @ w) / (w @ w)
        ref = alpha * e + step * d
        assert np.allclose(got[:, j], ref, rtol=0, atol=1e-14 * np.abs(ref).max())


def test_spai_mr_steps_decrease_residual_and_stop_at_tol():
    p = small_pencil(30)
    a = pencil.shifted_operator(p, 12.0)
    prev = None
    for it in (1, 2, 4, 8, 16):
        f = spai.spai_build(a, mr_iters=it, tol=0.0)
        if prev is not None:
            # each minimal-residual step can only lower a column's residual
            assert np.all(f.objective <= prev * (1 + 1e-12))
        prev = f.objective
    # the loop stops as soon as ||r|| <= tol (||e_j|| = 1)
    f = spai.spai_build(a, mr_iters=500, tol=0.3)
    stopped = f.iters < 500
    assert np.all(f.objective[stopped] <= 0.3)
    assert np.all(f.iters >= 0)
    # tolerance above the start: no step, P = alpha I
    f0 = spai.spai_build(a, symmetrize=False, mr_iters=5, tol=10.0)
    assert np.all(f0.iters == 0)
    d = f0.matrix().diagonal()
    n = p.n
    s = 1.0 / np.sqrt(a.diagonal())
    assert np.allclose(d, f0.alpha * s * s, rtol=1e-14)
    assert abs(f0.matrix().sum() - d.sum()) < 1e-12 * abs(d.sum())


def test_spai_mr_full_pattern_converges_to_inverse():
    # on a full pattern nothing is dropped: d = alpha r is the plain
    # minimal-residual iteration for K p = e_j, which converges to the inverse
    rng = np.random.default_rng(2)
    b = rng.standard_normal((6, 6))
    k = b @ b.T + 6 * np.eye(6)
    a = sp.csr_matrix(k)
    f = spai.spai_build(a, equilibrate=False, symmetrize=False, mr_iters=4000, tol=1e-13)
    assert np.allclose(f.matrix().toarray(), np.linalg.inv(k), atol=1e-11)


def test_spai_mr_update_skips_exactly_the_exact_mode_skips():
    p = small_pencil(40)
    a_old = pencil.shifted_operator(p, 4.0)
    a_new = pencil.shifted_operator(p, 4.4)
    ex = spai.spai_update(a_old, a_new, tol=0.05)
    mr = spai.spai_update(a_old, a_new, tol=0.05, mr_iters=20)
    # the start residual and the test are the same, so the columns that take
    # no step are exactly those the exact mode keeps at alpha e_j
    assert np.array_equal(ex.skipped, mr.skipped) and 0 < ex.skipped.sum() < p.n
    assert np.all(mr.iters[mr.skipped] == 0) and np.all(mr.iters[~mr.skipped] > 0)
    # entries of the skipped columns (CSR entry (r, c) belongs to column c)
    sel = ex.skipped[p.col_idx]
    assert np.array_equal(ex.hat[sel], mr.hat[sel])
    # minimal residual never beats the exact least squares of a column
    solved = ~ex.skipped
    assert np.all(mr.objective[solved] >= ex.objective[solved] * (1 - 1e-12))


# ------------------------------- SPAI minimal-residual pattern control (lfil)

def test_spai_lfil_one_entry_is_the_one_dimensional_least_squares():
    # lfil = 1 keeps p_j = c e_j: the line search along e_j reaches the
    # minimiser of ||e_j - c k_j|| in its first step, c = k_jj / ||k_j||^2,
    # and later steps leave it there
    p = small_pencil(12)
    a = pencil.shifted_operator(p, 5.0)
    k = a.toarray()
    f = spai.spai_build(a, equilibrate=False, symmetrize=False, mr_iters=7, tol=0.0, lfil=1)
    got = f.matrix().toarray()
    c = np.diag(k) / np.sum(k * k, axis=0)
    assert np.allclose(np.diag(got), c, rtol=1e-13, atol=0)
    assert np.count_nonzero(got - np.diag(np.diag(got))) == 0


def test_spai_lfil_admits_the_largest_remaining_entry():
    # K = I + c e_j^T + e_j c^T with the entries of c of distinct sizes: from
    # p = alpha e_j, r = e_j - alpha (e_j + c + c_j e_j) is -alpha c off j,
    # so the first step with lfil = 2 must admit the row of the largest |c_i|
    # and nothing else; lfil = 3 admits the two largest after two steps
    n, j = 7, 3
    cvec = np.array([0.05, -0.31, 0.12, 0.0, 0.27, -0.08, 0.2])
    k = np.eye(n)
    k[:, j] += cvec
    k[j, :] += cvec
    a = sp.csr_matrix(k)
    f1 = spai.spai_build(a, equilibrate=False, symmetrize=False, mr_iters=1, tol=0.0, lfil=2)
    col = f1.matrix().toarray()[:, j]
    assert set(np.flatnonzero(col)) == {j, 1}
    f2 = spai.spai_build(a, equilibrate=False, symmetrize=False, mr_iters=2, tol=0.0, lfil=3)
    col = f2.matrix().toarray()[:, j]
    assert set(np.flatnonzero(col)) <= {j, 1, 4} and col[1] != 0 and col[j] != 0
    # the cap: no column ever holds more than lfil entries
    f9 = spai.spai_build(a, equilibrate=False, symmetrize=False, mr_iters=50, tol=0.0, lfil=3)
    assert np.all(np.count_nonzero(f9.matrix().toarray(), axis=0) <= 3)


def test_spai_lfil_grown_to_a_full_pattern_converges_to_the_inverse():
    # on a dense SPD matrix with lfil = n the pattern reaches every row after
    # n - 1 steps; from then on d = alpha r is the plain minimal-residual
    # iteration for K p = e_j, which converges to the inverse
    rng = np.random.default_rng(5)
    b = rng.standard_normal((6, 6))
    k = b @ b.T + 6 * np.eye(6)
    a = sp.csr_matrix(k)
    f = spai.spai_build(a, equilibrate=False, symmetrize=False, mr_iters=4000, tol=1e-13,
                        lfil=6)
    assert np.allclose(f.matrix().toarray(), np.linalg.inv(k), atol=1e-11)
    # with a smaller cap the columns stay sparser than the inverse
    g = spai.spai_build(a, equilibrate=False, symmetrize=False, mr_iters=4000, tol=1e-13,
                        lfil=4)
    assert np.all(np.count_nonzero(g.matrix().toarray(), axis=0) == 4)


def test_spai_lfil_residuals_fall_and_patterns_stay_within_the_cap():
    p = small_pencil(30)
    a = pencil.shifted_operator(p, 12.0)
    prev = None
    for it in (1, 2, 3, 5, 9):
        f = spai.spai_build(a, symmetrize=False, mr_iters=it, tol=0.0, lfil=3)
        if prev is not None:
            assert np.all(f.objective <= prev * (1 + 1e-12))
        prev = f.objective
        # after `it` steps a column holds at most min(1 + it, 3) entries
        nnz = np.count_nonzero(f.matrix().toarray(), axis=0)
        assert np.all(nnz <= min(1 + it, 3))
    # the update: Q's columns obey the same cap; the skipped ones stay alpha e_j
    a_new = pencil.shifted_operator(p, 15.0)
    q = spai.spai_update(a, a_new, tol=0.01, mr_iters=9, lfil=2)
    nnz = np.count_nonzero(q.matrix().toarray(), axis=0)
    assert np.all(nnz <= 2) and np.all(nnz[q.skipped] == 1)
    with pytest.raises(ValueError):
        spai.spai_build(a, lfil=2)


# ------------------------------------------------- AIRGA's outer iteration

from oracle import airga_loop  # noqa: E402


def one_dof(m, d, k, cv=0.0, cp=1.0):
    a = np.array([[m]])
    return airga_loop.Model(a, np.array([[d]]), np.array([[k]]), np.array([[1.0]]),
                            np.array([[cp]]), np.array([[cv]]))


@pytest.mark.parametrize("m,d,k", [(2.0, 0.3, 5.0), (1.5, 9.0, 4.0)])
def test_qep_poles_one_dof_are_the_quadratic_roots(m, d, k):
    lam = np.sort_complex(airga_loop.qep_poles(np.array([[m]]), np.array([[d]]), np.array([[k]])))
    disc = complex(d * d - 4 * m * k)
    want = np.sort_complex(np.array([(-d + np.sqrt(disc)) / (2 * m), (-d - np.sqrt(disc)) / (2 * m)]))
    assert np.allclose(lam, want, rtol=1e-12, atol=0)


def test_qep_poles_make_the_pencil_singular():
    rng = np.random.default_rng(4)
    g = rng.standard_normal((4, 4))
    mh = g @ g.T + 4 * np.eye(4)
    g = rng.standard_normal((4, 4))
    kh = g @ g.T + np.eye(4)
    dh = 0.05 * mh + 0.02 * kh
    lam = airga_loop.qep_poles(mh, dh, kh)
    assert lam.size == 8
    # closed under conjugation, and each makes lambda^2 M + lambda D + K singular
    assert np.allclose(np.sort_complex(lam), np.sort_complex(lam.conj()), atol=1e-12)
    for x in lam:
        sv = np.linalg.svd(x * x * mh + x * dh + kh, compute_uv=False)
        assert sv[-1] <= 1e-10 * sv[0]


@pytest.mark.parametrize("m,d,k", [(1.0, 0.4, 3.0), (2.5, 1.7, 0.6)])
def test_h2_one_dof_closed_forms(m, d, k):
    # (1 / 2 pi) int |1 / (k - m w^2 + i d w)|^2 dw = 1 / (2 d k); with the
    # velocity output s / (...) it is 1 / (2 m d)
    pos = airga_loop.h2_distance(one_dof(m, d, k))
    vel = airga_loop.h2_distance(one_dof(m, d, k, cv=1.0, cp=0.0))
    assert abs(pos ** 2 - 1 / (2 * d * k)) <= 1e-12 / (2 * d * k)
    assert abs(vel ** 2 - 1 / (2 * m * d)) <= 1e-12 / (2 * m * d)


def random_model(rng, r, m=2, p=1, alpha=0.05, beta=0.02):
    g = rng.standard_normal((r, r))
    mh = g @ g.T + r * np.eye(r)
    g = rng.standard_normal((r, r))
    kh = g @ g.T + 0.5 * np.eye(r)
    return airga_loop.Model(mh, alpha * mh + beta * kh, kh, rng.standard_normal((r, m)),
                            rng.standard_normal((p, r)), rng.standard_normal((p, r)))


def test_h2_distance_equals_the_frequency_integral():
    import scipy.integrate as si
    rng = np.random.default_rng(8)
    a, b = random_model(rng, 3), random_model(rng, 2)

    def dens(w):
        h = a.transfer(1j * w) - b.transfer(1j * w)
        return float(np.sum(np.abs(h) ** 2))
    # |H(-iw)| = |H(iw)| for real models: twice the half line, over 2 pi
    val = 0.0
    for lo, hi in ((0, 1), (1, 10), (10, 100), (100, np.inf)):
        val += si.quad(dens, lo, hi, epsabs=0, epsrel=1e-11, limit=400)[0]
    want = np.sqrt(val / np.pi)
    assert abs(airga_loop.h2_distance(a, b) - want) <= 1e-7 * want


def test_h2_distance_is_a_norm_of_the_difference():
    rng = np.random.default_rng(9)
    a = random_model(rng, 4)
    assert airga_loop.h2_distance(a, a) <= 1e-7 * airga_loop.h2_distance(a)
    half = airga_loop.Model(a.mh, a.dh, a.kh, 0.5 * a.fh, a.cph, a.cvh)
    assert abs(airga_loop.h2_distance(a, half) - 0.5 * airga_loop.h2_distance(a)) <= \
        1e-9 * airga_loop.h2_distance(a)


def test_next_shifts_reading_on_a_hand_example():
    # candidates by |lambda|: -0.5 +- 2i (|.| 2.06) -> 0.5, -3 -> 3,
    # -1 +- 10i (10.05) -> 1, -40 -> 40; the first three, ascending
    poles = np.array([-1 + 10j, -1 - 10j, -0.5 + 2j, -0.5 - 2j, -3.0 + 0j, -40.0 + 0j])
    assert np.array_equal(airga_loop.next_shifts(poles, 3), [0.5, 1.0, 3.0])
    assert np.array_equal(airga_loop.next_shifts(poles, 4), [0.5, 1.0, 3.0, 40.0])
    with pytest.raises(ValueError):
        airga_loop.next_shifts(poles, 5)


def beam_system(n_el=60, m=2, alpha=0.1, beta=0.02, seed=3):
    pen = beam.make_beam(n_el, ei_loguniform=(0.5, 2.0), surrogate=True, seed=seed,
                         alpha=alpha, beta=beta)
    n = pen.n
    ms = pencil.csr(n, pen.row_ptr, pen.col_idx, pen.m_val)
    ks = pencil.csr(n, pen.row_ptr, pen.col_idx, pen.k_val)
    f, _ = beam.node_loads(n, m, np.random.default_rng(1))
    cp = np.zeros((1, n))
    cp[0, n - 2] = 1.0
    return pen, ms, ks, f.T, cp


def test_airga_iteration_interpolates_at_its_first_expansion_point():
    # V_1 is the QR of X(sigma_1) = K(sigma_1)^{-1} F, and every final basis
    # holds it, so each iteration's reduced model equals the full transfer
    # function at sigma_1 (Section 2)
    pen, ms, ks, f, cp = beam_system()
    _, _, hist = airga_loop.airga(ms, ks, pen.alpha, pen.beta, f, cp, None, [1.0, 30.0, 500.0],
                                  rmax=12, max_outer=3)
    assert len(hist) == 3
    for h in hist:
        s = h["shifts"][h["sigmas"][0]]
        ksp = (s * s + pen.alpha * s) * ms + (1 + pen.beta * s) * ks
        full = cp @ np.linalg.solve(ksp.toarray(), f)
        red = h["model"].transfer(s)
        assert np.allclose(red, full, rtol=1e-8, atol=1e-14 * np.abs(full).max())
        assert h["J"] == 12 // 2 and len(h["sigmas"]) == h["J"]


def test_real_part_expansion_points_fall_below_the_low_modes():
    # after the first iteration the new points are |Re lambda| = (alpha +
    # beta w^2) / 2 of the lowest reduced modes: far below those modes'
    # frequencies on a lightly damped beam, so the solves there nearly
    # coincide (the behaviour the design notes record)
    pen, ms, ks, f, cp = beam_system(alpha=0.01, beta=0.001)
    _, _, hist = airga_loop.airga(ms, ks, pen.alpha, pen.beta, f, cp, None, [1.0, 30.0, 500.0],
                                  rmax=12, max_outer=2)
    lam = airga_loop.qep_poles(hist[0]["model"].mh, hist[0]["model"].dh, hist[0]["model"].kh)
    w_low = np.sort(np.abs(lam))[0]
    assert np.all(hist[1]["shifts"] < 0.1 * w_low)


# ---- pins of the oracle's readings A1 (choice of sigma) and A5 (the H2
# stopping test), as its airga_loop module states them

def _diag_system(k=(1.0, 30.0, 900.0), alpha=0.1):
    """M = I, K = diag(k), D = alpha I, F = (1, 1, 1): every state
    X(s) = F / ((s^2 + alpha s) + k) is known entry by entry."""
    kk = np.asarray(k, float)
    ms = sp.identity(3, format="csr")
    ks = sp.diags(kk).tocsr()
    return kk, ms, ks, np.ones((3, 1)), np.array([[1.0, 0.0, 0.0]])


def _sin_angle(u, v):
    # |sin| of the angle between two 3-vectors from their cross product
    return float(np.linalg.norm(np.cross(u, v)) / (np.linalg.norm(u) * np.linalg.norm(v)))


@pytest.mark.parametrize("s2,want", [(30.0, 1), (1.02, 0), (3.0, 1)])
def test_sigma_is_the_point_with_the_largest_moment_error(s2, want):
    """Reading A1 on a diagonal 3-DOF system, r_max = 2 (one moment step):
    sigma_1 = s_1 and V_1 = X(s_1)/|X(s_1)|; then s_1's block becomes its next
    moment, parallel to X(s_1) * X(s_1) entrywise, and s_2's block is X(s_2).
    The moment errors are the sines of their angles with V_1 (cross
    products), and sigma_2 is the point with the larger one.  s_2 = 30 and 3
    give the larger error at s_2, s_2 = 1.02 (next to s_1) at s_1, so neither
    the smaller error nor a fixed index passes all three."""
    k, ms, ks, f, cp = _diag_system()
    alpha, s1 = 0.1, 1.0
    x = lambda s: 1.0 / ((s * s + alpha * s) + k)  # noqa: E731
    e_closed = [_sin_angle(x(s1), x(s1) * x(s1)), _sin_angle(x(s1), x(s2))]
    assert (e_closed[1] > e_closed[0]) == (want == 1)
    _, _, hist = airga_loop.airga(ms, ks, alpha, 0.0, f, cp, None, [s1, s2], rmax=2, max_outer=1)
    h = hist[0]
    assert h["sigmas"] == [0, want]
    assert np.allclose(h["step_errors"][0], e_closed, rtol=1e-12, atol=0)
    # the choice on its own: largest error, first index on a tie
    assert airga_loop.next_point(None) == 0
    assert airga_loop.next_point([0.2, 0.7, 0.1]) == 1
    assert airga_loop.next_point([0.5, 0.1, 0.5]) == 0


def _quad_h2(a, b):
    """||H_a - H_b||_H2 by quadrature of the frequency response."""
    import scipy.integrate as si

    def dens(w):
        h = a.transfer(1j * w) - b.transfer(1j * w)
        return float(np.sum(np.abs(h) ** 2))
    val = 0.0
    for lo, hi in ((0, 0.1), (0.1, 1), (1, 10), (10, 100), (100, 1e3), (1e3, np.inf)):
        val += si.quad(dens, lo, hi, epsabs=0, epsrel=1e-10, limit=500)[0]
    return np.sqrt(val / np.pi)


def test_inner_loop_stops_at_the_first_relative_change_below_tol():
    """Reading A5 for the moment loop: run it to r_max with tol 0, check each
    recorded change against ||H_j - H_{j-1}|| / ||H_j|| by quadrature of the
    intermediate models' frequency responses, then set tol between the
    smallest change and every earlier one: the loop must stop on exactly
    that step (J = its index + 2 blocks).  Scaling F by 1e3 and C_p by
    1e-3 scales every H by the same factor and must change nothing."""
    pen, ms, ks, f, cp = beam_system(n_el=20, m=1, alpha=0.2, beta=0.05)
    shifts = [0.5, 3.0, 20.0]
    _, _, full = airga_loop.airga(ms, ks, pen.alpha, pen.beta, f[:, :1], cp, None, shifts,
                                  rmax=8, tol_inner=0.0, max_outer=1)
    h = full[0]
    ch = h["inner_changes"]
    mods = h["inner_models"]
    assert len(ch) == len(mods) - 1 >= 3 and h["J"] == 8
    for j, c in enumerate(ch):
        num = _quad_h2(mods[j + 1], mods[j])
        den = _quad_h2(mods[j + 1], airga_loop.Model(mods[j + 1].mh, mods[j + 1].dh,
                                                      mods[j + 1].kh, 0 * mods[j + 1].fh,
                                                      mods[j + 1].cph))
        assert abs(c - num / den) <= 1e-6 * num / den, j
    t = int(np.argmin(ch))
    earlier = min(ch[:t]) if t > 0 else np.inf
    tol = 0.5 * (ch[t] + min(earlier, 2 * ch[t]))
    for scale in (1.0, 1e3):
        _, _, st = airga_loop.airga(ms, ks, pen.alpha, pen.beta, scale * f[:, :1], cp / scale,
                                    None, shifts, rmax=8, tol_inner=tol, max_outer=1)
        g = st[0]
        assert len(g["inner_changes"]) == t + 1
        assert g["J"] == t + 3 and g["sigmas"] == h["sigmas"][:t + 2] + [g["sigmas"][-1]]


def test_outer_loop_stops_on_the_relative_change():
    """Reading A5 for the outer loop: tol_outer = inf stops after the second
    iteration (the first with a change), tol_outer = 0 runs max_outer."""
    pen, ms, ks, f, cp = beam_system(n_el=20, m=1, alpha=0.2, beta=0.05)
    for tol, want in ((np.inf, 2), (0.0, 3)):
        _, _, hist = airga_loop.airga(ms, ks, pen.alpha, pen.beta, f[:, :1], cp, None,
                                      [0.5, 3.0, 20.0], rmax=4, tol_outer=tol, max_outer=3)
        assert len(hist) == want
        assert hist[0]["change"] is None and all(x["change"] > 0 for x in hist[1:])


# ----------------------------------------------------- complex expansion points

def _cbeam(n_el=40, seed=1):
    return beam.make_beam(n_el, ei_loguniform=(0.5, 2.0), surrogate=True, seed=seed)


CSHIFTS = [3.0 + 2.0j, 0.5 - 4.0j, 100.0 + 50.0j, 1.0 + 0.1j]


@pytest.mark.parametrize("s", CSHIFTS)
def test_complex_reference_solve_matches_the_dense_solve(s):
    pen = _cbeam()
    f = np.random.default_rng(0).standard_normal((2, pen.n))
    a = pencil.shifted_operator_complex(pen, s).toarray()
    # K(s) is complex symmetric, not Hermitian
    assert np.array_equal(a, a.T) and not np.allclose(a, a.conj().T)
    x = np.linalg.solve(a, f.T).T
    for prec in ("f64", "dd"):
        y = direct.reference_solve_complex(pen, s, f, prec)
        assert np.linalg.norm(y - x) <= 1e-13 * np.linalg.norm(x), prec


def test_complex_reference_reduces_to_the_real_one_and_respects_conjugation():
    pen = _cbeam()
    f = np.random.default_rng(1).standard_normal((1, pen.n))
    for s in (0.7, 25.0):
        y = direct.reference_solve_complex(pen, s, f, "dd")
        z = direct.reference_solve(pen, s, f, "dd")
        assert np.abs(y.imag).max() == 0.0
        assert np.linalg.norm(y.real - z) <= 1e-15 * np.linalg.norm(z)
    # M, K and F are real, so K(conj s) = conj K(s) and X(conj s) = conj X(s)
    for s in CSHIFTS:
        a = direct.reference_solve_complex(pen, s, f, "dd")
        b = direct.reference_solve_complex(pen, np.conj(s), f, "dd")
        assert np.linalg.norm(b - a.conj()) <= 1e-14 * np.linalg.norm(a)


def test_complex_shift_assembly_in_double_double_is_exact():
    from fractions import Fraction as Fr
    pen = _cbeam(6)
    s = 3.0 + 2.0j
    rh, rl, ih, il, w = direct.shifted_band_cdd(pen, s)
    mb, _ = direct.lower_band(pencil.csr(pen.n, pen.row_ptr, pen.col_idx, pen.m_val), w)
    kb, _ = direct.lower_band(pencil.csr(pen.n, pen.row_ptr, pen.col_idx, pen.k_val), w)
    sr, si, al, be = Fr(3.0), Fr(2.0), Fr(pen.alpha), Fr(pen.beta)
    # (s^2 + alpha s) M + (1 + beta s) K with s = sr + i si, exactly
    a_re, a_im = sr * sr - si * si + al * sr, 2 * sr * si + al * si
    b_re, b_im = 1 + be * sr, be * si
    for e in range(mb.size):
        m, k = Fr(mb.flat[e]), Fr(kb.flat[e])
        want_re, want_im = a_re * m + b_re * k, a_im * m + b_im * k
        for hi, lo, want in ((rh, rl, want_re), (ih, il, want_im)):
            got = Fr(hi.flat[e]) + Fr(lo.flat[e])
            assert abs(got - want) <= abs(want) * Fr(1, 2 ** 100) + Fr(1, 2 ** 1000)


@pytest.mark.parametrize("s", CSHIFTS)
def test_complex_spai_columns_are_least_squares_optimal(s):
    pen = _cbeam(30)
    a = pencil.shifted_operator_complex(pen, s)
    fac = spai.spai_build(a, symmetrize=False)
    d = a.diagonal()
    sc = 1 / np.sqrt(d)
    ah = (sp.diags(sc) @ a @ sp.diags(sc)).toarray()
    hat = sp.csr_matrix((fac.hat, pen.col_idx, pen.row_ptr), shape=(pen.n, pen.n)).toarray()
    for j in range(pen.n):
        jj = pen.col_idx[pen.row_ptr[j]:pen.row_ptr[j + 1]]
        res = np.eye(pen.n)[:, j] - ah[:, jj] @ hat[jj, j]
        # normal equations of the complex problem: B^H r = 0
        assert np.linalg.norm(ah[:, jj].conj().T @ res) <= 1e-12 * np.linalg.norm(ah[:, jj]) * max(
            np.linalg.norm(res), 1e-300)
        # the full n-row problem gives the same column
        full, *_ = np.linalg.lstsq(ah[:, jj], np.eye(pen.n)[:, j], rcond=None)
        assert np.allclose(hat[jj, j], full, rtol=0, atol=1e-11 * np.abs(full).max())
        assert abs(fac.objective[j] - np.linalg.norm(res)) <= 1e-12 * max(1, fac.objective[j])


def test_complex_spai_special_cases():
    pen = _cbeam(8)
    s = 3.0 + 2.0j
    a = pencil.shifted_operator_complex(pen, s)
    # symmetric average: the factor is complex symmetric (plain transpose)
    p = spai.spai_build(a).matrix().toarray()
    assert np.allclose(p, p.T, rtol=0, atol=1e-15 * np.abs(p).max())
    # a real shift gives the real factor
    ar = pencil.shifted_operator_complex(pen, 7.0)
    pr = spai.spai_build(ar).values
    assert np.allclose(pr.real, spai.spai_build(pencil.shifted_operator(pen, 7.0)).values,
                       rtol=1e-13, atol=0)
    assert np.abs(pr.imag).max() == 0.0
    # the full pattern gives the inverse
    n = pen.n
    dense = sp.csr_matrix(a.toarray() + 0 * np.ones((n, n)))
    full = sp.csr_matrix((np.asarray(a.toarray()).ravel(), np.tile(np.arange(n), n),
                          np.arange(0, n * n + 1, n)), shape=(n, n))
    inv = spai.spai_build(full, equilibrate=False, symmetrize=False).matrix().toarray()
    assert np.allclose(inv, np.linalg.inv(dense.toarray()), rtol=0,
                       atol=1e-10 * np.abs(np.linalg.inv(dense.toarray())).max())
    # complex alpha: the Frobenius minimiser of ||I - alpha K||, by brute force
    al = spai.spai_build(a, cols=[0]).alpha
    f = lambda z: np.linalg.norm(np.eye(n) - z * a.toarray())  # noqa: E731
    for dz in (1e-3, 1e-3j, -1e-3, -1e-3j):
        assert f(al) <= f(al * (1 + dz))


def test_complex_update_alpha_is_the_frobenius_minimiser():
    # ||K_old - alpha K_new||_F over complex alpha = x + i y is a real linear
    # least-squares problem in (x, y): stack the real and imaginary parts
    pen = _cbeam(12)
    for s_old, s_new in ((3.0 + 2.0j, 3.3 + 2.1j), (1.0 + 0.1j, 0.5 - 4.0j)):
        ko = pencil.shifted_operator_complex(pen, s_old).toarray().ravel()
        kn = pencil.shifted_operator_complex(pen, s_new).toarray().ravel()
        a = np.stack([np.concatenate([kn.real, kn.imag]),
                      np.concatenate([-kn.imag, kn.real])], axis=1)
        xy, *_ = np.linalg.lstsq(a, np.concatenate([ko.real, ko.imag]), rcond=None)
        al = spai.update_alpha(pencil.shifted_operator_complex(pen, s_old),
                               pencil.shifted_operator_complex(pen, s_new))
        assert abs(al - complex(xy[0], xy[1])) <= 1e-13 * abs(al)
    # real matrices: the formula of Section 3.2 (a real number)
    ar, br = pencil.shifted_operator(pen, 2.0), pencil.shifted_operator(pen, 2.5)
    al = spai.update_alpha(ar, br)
    assert isinstance(al, float)
    assert abs(al - np.vdot(br.toarray(), ar.toarray()) / np.vdot(br.toarray(), br.toarray())) <= \
        1e-14 * abs(al)


@pytest.mark.parametrize("s_old,s_new", [(3.0 + 2.0j, 3.6 + 2.3j), (100.0 + 50.0j, 60.0 + 45.0j),
                                         (1.0 + 2.0j, 1.5 + 2.5j)])
def test_complex_update_columns_are_least_squares_optimal(s_old, s_new):
    # solved columns satisfy the normal equations of min ||khat_old_j -
    # Khat_new(:, J) q|| (Khat = S K S, S from the principal square root of
    # diag K(s_new)); skipped ones are alpha e_j; Q = S Qhat S^{-1}
    pen = _cbeam(30)
    ao = pencil.shifted_operator_complex(pen, s_old)
    an = pencil.shifted_operator_complex(pen, s_new)
    q = spai.spai_update(ao, an, tol=0.05)
    assert 0 < q.skipped.sum() < pen.n, q.skipped.sum()
    sc = 1 / np.sqrt(an.diagonal())
    kn = (sp.diags(sc) @ an @ sp.diags(sc)).toarray()
    ko = (sp.diags(sc) @ ao @ sp.diags(sc)).toarray()
    qm = q.matrix().toarray()
    qhat = np.diag(1 / sc) @ qm @ np.diag(sc)
    for j in range(pen.n):
        jj = pen.col_idx[pen.row_ptr[j]:pen.row_ptr[j + 1]]
        assert np.count_nonzero(qhat[:, j][np.setdiff1d(np.arange(pen.n), jj)]) == 0
        if q.skipped[j]:
            want = np.zeros(pen.n, complex)
            want[j] = q.alpha
            assert np.allclose(qhat[:, j], want, rtol=1e-14, atol=0)
            continue
        res = ko[:, j] - kn[:, jj] @ qhat[jj, j]
        assert np.linalg.norm(kn[:, jj].conj().T @ res) <= 1e-12 * np.linalg.norm(kn[:, jj]) * \
            np.linalg.norm(ko[:, j])
        assert abs(q.objective[j] - np.linalg.norm(res)) <= 1e-12 * np.linalg.norm(ko[:, j])
    # real shifts given as complex numbers: the real update
    qr = spai.spai_update(pencil.shifted_operator_complex(pen, 4.0),
                          pencil.shifted_operator_complex(pen, 4.6), tol=0.05)
    qx = spai.spai_update(pencil.shifted_operator(pen, 4.0), pencil.shifted_operator(pen, 4.6),
                          tol=0.05)
    assert np.array_equal(qr.skipped, qx.skipped)
    # (the complex and real least-squares routines round differently)
    assert np.allclose(qr.values.real, qx.values, rtol=0, atol=1e-12 * np.abs(qx.values).max())
    assert np.abs(qr.values.imag).max() == 0.0


def test_cocg_with_an_update_chain_reaches_the_solution():
    # the chain Q P (P built at s_old, Q its update to s_new) preconditions
    # COCG on K(s_new) to the dense solution, with the flexible beta
    pen = _cbeam(50)
    f = np.random.default_rng(5).standard_normal(pen.n)
    s_old, s_new = 3.0 + 2.0j, 3.9 + 2.6j
    ao = pencil.shifted_operator_complex(pen, s_old)
    an = pencil.shifted_operator_complex(pen, s_new)
    p1 = spai.spai_build(ao)
    q2 = spai.spai_update(ao, an, tol=0.01)
    r = pcg.cocg(lambda v: an @ v, lambda v: spai.chain_apply([p1, q2], v), f, tol=1e-12,
                 max_iter=4000)
    x = np.linalg.solve(an.toarray(), f)
    assert r.status == pcg.CONVERGED
    assert np.linalg.norm(r.x - x) <= 1e-9 * np.linalg.norm(x)


def test_cocg_matches_the_dense_solve_and_cg_on_real_data():
    pen = _cbeam(50)
    rng = np.random.default_rng(3)
    f = rng.standard_normal(pen.n)
    for s in CSHIFTS:
        a = pencil.shifted_operator_complex(pen, s)
        p = spai.spai_build(a).matrix()
        r = pcg.cocg(lambda v: a @ v, lambda v: p @ v, f, tol=1e-12, max_iter=4000)
        x = np.linalg.solve(a.toarray(), f)
        assert r.status == pcg.CONVERGED
        assert np.linalg.norm(r.x - x) <= 1e-9 * np.linalg.norm(x)
    # real data: COCG is CG (same iterates as the oracle's PCG, both betas)
    a = pencil.shifted_operator(pen, 20.0)
    p = spai.spai_build(a).matrix()
    for form in ("flexible", "fr"):
        r1 = pcg.cocg(lambda v: a @ v, lambda v: p @ v, f, tol=1e-10, beta=form)
        r2 = pcg.pcg(lambda v: a @ v, lambda v: p @ v, f, tol=1e-10, beta=form)
        assert r1.iters == r2.iters
        assert np.linalg.norm(r1.x - r2.x) <= 1e-12 * np.linalg.norm(r2.x)


def test_cocg_terminates_and_keeps_the_residuals_conjugate_orthogonal():
    # n = 12, complex symmetric K and C: the residuals are orthogonal in the
    # bilinear form through C (r_i^T C r_k = 0, i != k), which ends the
    # iteration within n steps in exact arithmetic
    rng = np.random.default_rng(5)
    n = 12
    g = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    k = (2 + 1j) * np.eye(n) + 0.1 * (g + g.T)
    h = rng.standard_normal((n, n)) + 0.3j * rng.standard_normal((n, n))
    c = np.eye(n) + 0.05 * (h + h.T)
    f = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    r = pcg.cocg(lambda v: k @ v, lambda v: c @ v, f, tol=1e-12, max_iter=3 * n, keep=True,
                 beta="fr")
    assert r.status == pcg.CONVERGED and r.iters <= n + 2
    res = r.residuals
    for i in range(len(res)):
        for j in range(i + 1, len(res)):
            zj = c @ res[j]
            assert abs(res[i] @ zj) <= 1e-8 * np.linalg.norm(res[i]) * np.linalg.norm(zj)
    assert np.linalg.norm(r.x - np.linalg.solve(k, f)) <= 1e-10 * np.linalg.norm(r.x)
    # mu = p^T K p = 0 stops the iteration as a breakdown
    z = np.array([1.0, 1j])
    kk = np.eye(2)
    br = pcg.cocg(lambda v: kk @ v, lambda v: v, z, tol=1e-12)
    assert br.status == pcg.BREAKDOWN and br.iters == 0


def test_reference_solves_equal_the_single_shift_reference():
    # the bands of M and K extracted once give bit-identical references
    pen = beam.make_beam(150, ei_loguniform=(0.5, 2.0), surrogate=True, seed=4)
    f = np.random.default_rng(2).standard_normal((2, pen.n))
    shifts = [1.0, 37.0, 2500.0]
    for prec in ("f64", "dd"):
        many = direct.reference_solves(pen, shifts, f, prec, workers=2)
        seen = []
        direct.reference_solves(pen, shifts, f, prec, workers=2,
                                each=lambda i, x: seen.append((i, x)))
        for k, s in enumerate(shifts):
            one = direct.reference_solve(pen, s, f, prec)
            assert np.array_equal(many[k], one)
            assert seen[k][0] == k and np.array_equal(seen[k][1], one)
