"""GPU: complex expansion points (K(s) complex symmetric) against the
oracle: the shifted matrix, the complex SPAI (column least squares,
equilibrated and symmetrised with the plain transpose), and batched COCG --
its iterates after k steps against the oracle's COCG with the same factor,
its solutions against the complex double-double reference -- at small sizes
with ragged slices and at the full 1,000,000-DOF size the benchmark times."""
import numpy as np
import pytest
import torch

from gpu_util import airga, beam, direct, grid_pencil, pencil, rel_err, set_pencil, spai, to_dev
from oracle import pcg as opcg

pytestmark = pytest.mark.gpu

SHIFTS = [3.0 + 2.0j, 0.5 - 4.0j, 100.0 + 50.0j, 1.0 + 0.1j]


@pytest.fixture(scope="module")
def ctx():
    c = airga.Context(0)
    yield c
    c.close()


def sur_beam(n_el=1037, seed=11):
    return beam.make_beam(n_el, ei_loguniform=(0.5, 2.0), surrogate=True, seed=seed)


def factor_matrix(pen, vals):
    import scipy.sparse as sp
    return sp.csr_matrix((vals, pen.col_idx, pen.row_ptr), shape=(pen.n, pen.n))


def test_complex_assembly(ctx):
    pen = sur_beam(301)
    set_pencil(ctx, pen)
    for s in SHIFTS:
        got = ctx.assemble_shift_complex(s).cpu().numpy()
        ref = pencil.shifted_values_complex(pen.m_val, pen.k_val, pen.alpha, pen.beta, s)
        scale = np.abs(pen.m_val) * abs(s * s + pen.alpha * s) + np.abs(pen.k_val) * abs(1 + pen.beta * s)
        assert np.all(np.abs(got - ref) <= 4e-16 * scale + 1e-300)


@pytest.mark.parametrize("which", ["beam", "grid"])
def test_complex_spai_matches_oracle(ctx, which):
    pen = sur_beam(301) if which == "beam" else grid_pencil(23, 17)
    set_pencil(ctx, pen)
    for s in SHIFTS:
        a = pencil.shifted_operator_complex(pen, s)
        for sym in (False, True):
            ref = spai.spai_build(a, symmetrize=sym)
            p = ctx.spai_build_complex(s, symmetrize=sym)
            vals, obj = (t.cpu().numpy() for t in p.export_complex())
            assert np.all(np.abs(obj - ref.objective) <= 1e-12 * np.maximum(1.0, ref.objective))
            assert np.all(np.abs(vals - ref.values) <= 1e-9 * np.abs(ref.values).max()), (s, sym)
            if sym:
                m = factor_matrix(pen, vals)
                assert abs(m - m.T).max() <= 1e-15 * np.abs(vals).max()
            info = p.info()
            assert info.is_complex == 1 and info.shift == s.real and info.shift_im == s.imag
            assert np.isclose(info.alpha + 1j * info.alpha_im, ref.alpha, rtol=1e-12)


def test_complex_spai_normal_equations_agree_with_rotations(ctx):
    """On the beam (equilibrated, rows of consecutive columns) the complex
    SPAI solves each column from its normal equations, whose Gram matrix is
    a block of conj(Khat) Khat; the Givens kernel solves the same problems
    by rotations.  The two agree to cond(Khat(I, J))^2 eps (cond below 15
    after equilibration here), on ragged slices, with and without the
    symmetric average; the unequilibrated build takes the rotations only and
    is bit-identical either way."""
    pen = sur_beam(1037)
    set_pencil(ctx, pen)
    for s in SHIFTS + [1e4 * np.exp(1j * np.pi / 6)]:
        for sym in (False, True):
            g = ctx.spai_build_complex(s, symmetrize=sym)
            r = ctx.spai_build_complex(s, symmetrize=sym, general_only=True)
            vg, og = (t.cpu().numpy() for t in g.export_complex())
            vr, orr = (t.cpu().numpy() for t in r.export_complex())
            assert np.abs(vg - vr).max() <= 1e-12 * np.abs(vr).max(), (s, sym)
            assert np.all(np.abs(og - orr) <= 1e-12 * np.maximum(1.0, orr)), (s, sym)
        g = ctx.spai_build_complex(s, equilibrate=False)
        r = ctx.spai_build_complex(s, equilibrate=False, general_only=True)
        assert torch.equal(g.export_complex()[0], r.export_complex()[0])


@pytest.mark.parametrize("which", ["beam", "grid"])
@pytest.mark.parametrize("s_old,s_new", [(3.0 + 2.0j, 3.6 + 2.3j), (100.0 + 50.0j, 60.0 + 45.0j),
                                         (1.0 + 2.0j, 1.5 + 2.5j)])
def test_complex_update_matches_oracle(ctx, which, s_old, s_new):
    """The SPAI update at complex points (Section 3.2 with complex alpha,
    skip test, complex column least squares, Q = S Qhat S^-1) against the
    oracle: alpha, the skipped columns and every value.  A column whose skip
    test came within 1e-8 of its threshold in the oracle may fall either way
    and is left out of the value comparison."""
    pen = sur_beam(301) if which == "beam" else grid_pencil(23, 17)
    set_pencil(ctx, pen)
    old = ctx.spai_build_complex(s_old)
    q = ctx.spai_update_complex(old, s_new, tol=0.05)
    ref = spai.spai_update(pencil.shifted_operator_complex(pen, s_old),
                           pencil.shifted_operator_complex(pen, s_new), tol=0.05)
    info = q.info()
    assert info.is_complex == 1 and info.shift == s_new.real and info.shift_im == s_new.imag
    assert abs(complex(info.alpha, info.alpha_im) - ref.alpha) <= 1e-12 * abs(ref.alpha)
    tie = ref.margin < 1e-8
    flags = q.skip_flags().cpu().numpy().astype(bool)
    assert np.array_equal(flags[~tie], ref.skipped[~tie])
    assert info.skipped_cols == int(flags.sum())
    vals, obj = (t.cpu().numpy() for t in q.export_complex())
    row = np.repeat(np.arange(pen.n), np.diff(pen.row_ptr))
    sel = ~tie[pen.col_idx]    # entry (r, c) belongs to column c
    if info.scalar_only:
        assert ref.skipped.all()
    assert np.all(np.abs(vals - ref.values)[sel] <= 1e-9 * np.abs(ref.values).max()), (s_old, s_new)
    assert np.all(np.abs(obj - ref.objective)[~tie] <= 1e-12 * np.maximum(1.0, ref.objective[~tie]))
    assert row.size == vals.size
    # the normal-equation kernel (beam) and the rotations agree, flags exactly
    qg = ctx.spai_update_complex(old, s_new, tol=0.05, general_only=True)
    assert torch.equal(qg.skip_flags(), q.skip_flags())
    assert qg.info().skipped_cols == info.skipped_cols
    vg, og = (t.cpu().numpy() for t in qg.export_complex())
    assert np.abs(vg - vals).max() <= 1e-12 * np.abs(vals).max()
    assert np.all(np.abs(og - obj) <= 1e-12 * np.maximum(1.0, obj))


def test_complex_builds_and_updates_many_equal_single_calls(ctx):
    """The many-point calls give exactly the single calls' factors (values,
    objectives, alpha, skip counts), including an update that skips every
    column (the scalar alpha I) and a repeated old factor; a bad entry
    fails the whole call."""
    pen = sur_beam(400)
    set_pencil(ctx, pen)
    pts = [3.0 + 2.0j, 30.0 * np.exp(1j * np.pi / 6), 100.0 + 50.0j]
    many = ctx.spai_build_complex_many(pts)
    one = [ctx.spai_build_complex(z) for z in pts]
    for m_, o_ in zip(many, one):
        vm, om = (t.cpu().numpy() for t in m_.export_complex())
        vo, oo = (t.cpu().numpy() for t in o_.export_complex())
        assert np.array_equal(vm, vo) and np.array_equal(om, oo)
    new = [pts[0] * 1.2, pts[1] * (1 + 1e-9), pts[2] * 0.9, pts[0] * 0.8]
    olds = [one[0], one[1], one[2], one[0]]
    um = ctx.spai_update_complex_many(olds, new, tol=0.05)
    uo = [ctx.spai_update_complex(p, z, tol=0.05) for p, z in zip(olds, new)]
    assert um[1].info().scalar_only == 1
    for m_, o_ in zip(um, uo):
        im, io = m_.info(), o_.info()
        assert (im.alpha, im.alpha_im, im.skipped_cols, im.chain_len, im.scalar_only) == \
            (io.alpha, io.alpha_im, io.skipped_cols, io.chain_len, io.scalar_only)
        vm, om = (t.cpu().numpy() for t in m_.export_complex())
        vo, oo = (t.cpu().numpy() for t in o_.export_complex())
        assert np.array_equal(vm, vo) and np.array_equal(om, oo)
    F = to_dev(np.random.default_rng(3).standard_normal((1, pen.n)), torch.float64)
    Xm, _ = ctx.cocg_solve(new, um, F, tol=1e-10)
    Xo, _ = ctx.cocg_solve(new, uo, F, tol=1e-10)
    assert torch.equal(Xm, Xo)
    assert ctx.spai_build_complex_many([]) == [] and ctx.spai_update_complex_many([], []) == []
    with pytest.raises(airga.AirgaError) as e:
        ctx.spai_update_complex_many([one[0], ctx.spai_build(5.0)], [pts[0], pts[1]])
    assert e.value.status == airga.EINVAL
    with pytest.raises(airga.AirgaError) as e:
        ctx.spai_build_complex_many([1.0 + 1.0j, complex(float("nan"), 0.0)])
    assert e.value.status == airga.EINVAL


def test_cocg_with_a_complex_update_chain(ctx):
    """P_1 built at s_1, Q_2 and Q_3 its updates along s_2, s_3 (each with
    solved columns): COCG at s_3 with the chain Q_3 Q_2 P_1 follows the
    oracle's COCG with the oracle's own chain (iterates after k steps, to the
    factors' agreement) and reaches the complex double-double reference; an
    update that skips every column is the scalar alpha I, which the solve
    drops from the chain."""
    pen = sur_beam(1037)
    set_pencil(ctx, pen)
    # points on the benchmark's ray sigma e^(i pi/6) where both updates solve
    # some columns and skip others; nearer the origin (1 + 2i) every chain
    # stalls in the oracle's COCG as well (as in the real chains from s = 1)
    pts = [complex(v * np.exp(1j * np.pi / 6)) for v in (30.0, 34.0, 38.0)]
    p1 = ctx.spai_build_complex(pts[0])
    q2 = ctx.spai_update_complex(p1, pts[1], tol=0.05)
    q3 = ctx.spai_update_complex(q2, pts[2], tol=0.05)
    i2, i3 = q2.info(), q3.info()
    assert 0 < i2.skipped_cols < pen.n and 0 < i3.skipped_cols < pen.n
    assert i3.chain_len == 3
    ops = [pencil.shifted_operator_complex(pen, z) for z in pts]
    chain = [spai.spai_build(ops[0]), spai.spai_update(ops[0], ops[1], tol=0.05),
             spai.spai_update(ops[1], ops[2], tol=0.05)]
    assert all(np.min(f.margin) > 1e-8 for f in chain[1:])   # no skip test near its threshold
    rng = np.random.default_rng(9)
    f = rng.standard_normal((2, pen.n))
    F = to_dev(f, torch.float64)
    for k in (1, 2, 5):
        X, st = ctx.cocg_solve([pts[2]], [q3], F, tol=1e-30, max_iter=k)
        for c in range(2):
            assert st[c]["iters"] == k
            r = opcg.cocg(lambda v: ops[2] @ v, lambda v: spai.chain_apply(chain, v), f[c],
                          tol=1e-30, max_iter=k)
            assert rel_err(X[0, c].cpu().numpy(), r.x) < 1e-9, (k, c)
    X, st = ctx.cocg_solve([pts[2]], [q3], F, tol=1e-10)
    ref = direct.reference_solve_complex(pen, pts[2], f, "dd")
    for c in range(2):
        assert st[c]["status"] == airga.SYS_CONVERGED
        assert rel_err(X[0, c].cpu().numpy(), ref[c]) < 1e-8
    # an update that skips every column: alpha I, exported as such
    s1 = pts[0] * (1 + 1e-9)
    qs = ctx.spai_update_complex(p1, s1, tol=0.05)
    assert qs.info().scalar_only == 1 and qs.info().chain_len == 1
    al = complex(qs.info().alpha, qs.info().alpha_im)
    diag = pen.col_idx == np.repeat(np.arange(pen.n), np.diff(pen.row_ptr))
    assert np.array_equal(qs.export_complex()[0].cpu().numpy(), np.where(diag, al, 0.0))
    Xa, sa = ctx.cocg_solve([s1], [qs], F, tol=1e-10)
    refs = direct.reference_solve_complex(pen, s1, f, "dd")
    for c in range(2):
        assert sa[c]["status"] == airga.SYS_CONVERGED
        assert rel_err(Xa[0, c].cpu().numpy(), refs[c]) < 1e-8
    # refusals
    with pytest.raises(airga.AirgaError) as e:
        ctx.spai_update_complex(ctx.spai_build(2.0), 2.0 + 1.0j)
    assert e.value.status == airga.EINVAL
    with pytest.raises(airga.AirgaError) as e:
        ctx.spai_update(p1, 3.0)
    assert e.value.status == airga.EUNSUPPORTED


@pytest.mark.parametrize("form,oform", [(airga.BETA_FLEXIBLE, "flexible"),
                                        (airga.BETA_CLASSICAL, "fr")])
def test_cocg_iterates_follow_the_oracle(ctx, form, oform):
    """After k steps the GPU iterate equals the oracle's COCG with the
    oracle's own factor (to the factors' agreement), for both direction
    updates."""
    pen = sur_beam(400)
    set_pencil(ctx, pen)
    rng = np.random.default_rng(4)
    f = rng.standard_normal((2, pen.n))
    s = 2.0 + 1.5j
    p = ctx.spai_build_complex(s)
    a = pencil.shifted_operator_complex(pen, s)
    cm = spai.spai_build(a).matrix()
    for k in (1, 3, 8):
        X, st = ctx.cocg_solve([s], [p], to_dev(f, torch.float64), tol=1e-30, max_iter=k,
                               beta_form=form)
        for c in range(2):
            assert st[c]["status"] == airga.SYS_MAXIT and st[c]["iters"] == k
            r = opcg.cocg(lambda v: a @ v, lambda v: cm @ v, f[c], tol=1e-30, max_iter=k, beta=oform)
            assert rel_err(X[0, c].cpu().numpy(), r.x) < 1e-10, (k, c)


def test_batched_cocg_matches_the_reference(ctx):
    pen = sur_beam()
    set_pencil(ctx, pen)
    rng = np.random.default_rng(2)
    f = np.stack([beam.tip_load(pen.n)[0], rng.standard_normal(pen.n)])
    precs = [ctx.spai_build_complex(s) for s in SHIFTS]
    X, st = ctx.cocg_solve(SHIFTS, precs, to_dev(f, torch.float64), tol=1e-10)
    Xh = X.cpu().numpy()
    for k, s in enumerate(SHIFTS):
        ref = direct.reference_solve_complex(pen, s, f, "dd")
        for c in range(2):
            e = st[2 * k + c]
            assert e["status"] == airga.SYS_CONVERGED, (s, c, e)
            assert e["relres"] <= 2e-10   # the true residual at exit
            assert rel_err(Xh[k, c], ref[c]) < 1e-8, (s, c)
    # without a preconditioner the iterations grow (up to the cap: at
    # s = 0.5 - 4i the recurrence stalls near 5e-9), and the error is up to
    # cond(K(s)) times the residual (2.7e-8 at s = 3 + 2i for relres 1e-10)
    _, st0 = ctx.cocg_solve(SHIFTS, None, to_dev(f, torch.float64), tol=1e-10, max_iter=20000)
    assert sum(e["iters"] for e in st) < sum(e["iters"] for e in st0)


@pytest.mark.parametrize("form,oform", [(airga.BETA_FLEXIBLE, "flexible"),
                                        (airga.BETA_CLASSICAL, "fr")])
def test_mixed_cocg_inner_iterates_follow_the_oracle(ctx, form, oform):
    """MIXED mode, one sweep of k float32 COCG steps from X = 0: X is the
    oracle's float64 COCG iterate after k steps to float32 accuracy, for
    both direction updates."""
    pen = sur_beam(400)
    set_pencil(ctx, pen)
    f = np.random.default_rng(4).standard_normal((2, pen.n))
    s = 2.0 + 1.5j
    p = ctx.spai_build_complex(s)
    a = pencil.shifted_operator_complex(pen, s)
    cm = spai.spai_build(a).matrix()
    for k in (2, 4, 8):
        X, st = ctx.cocg_solve([s], [p], to_dev(f, torch.float64), tol=1e-30, mode=airga.MODE_MIXED,
                               inner_tol=1e-12, inner_max=k, poll_every=2, max_sweeps=1,
                               beta_form=form)
        for c in range(2):
            assert st[c]["status"] == airga.SYS_MAXIT and st[c]["iters"] == k
            assert st[c]["sweeps"] == 1
            r = opcg.cocg(lambda v: a @ v, lambda v: cm @ v, f[c], tol=1e-30, max_iter=k,
                          beta=oform)
            assert rel_err(X[0, c].cpu().numpy(), r.x) < 1e-3, (k, c)


def test_mixed_cocg_chain_iterates_follow_the_oracle(ctx):
    """MIXED mode with an update chain Q_3 Q_2 P_1 (the float copies of
    every factor), one sweep of k steps: the oracle's float64 COCG with the
    oracle's own chain, to float32 accuracy."""
    pen = sur_beam(1037)
    set_pencil(ctx, pen)
    pts = [complex(v * np.exp(1j * np.pi / 6)) for v in (30.0, 34.0, 38.0)]
    q3 = ctx.spai_update_complex(ctx.spai_update_complex(ctx.spai_build_complex(pts[0]), pts[1],
                                                         tol=0.05), pts[2], tol=0.05)
    assert q3.info().chain_len == 3
    ops = [pencil.shifted_operator_complex(pen, z) for z in pts]
    chain = [spai.spai_build(ops[0]), spai.spai_update(ops[0], ops[1], tol=0.05),
             spai.spai_update(ops[1], ops[2], tol=0.05)]
    f = np.random.default_rng(9).standard_normal((2, pen.n))
    for k in (2, 6):
        X, st = ctx.cocg_solve([pts[2]], [q3], to_dev(f, torch.float64), tol=1e-30,
                               mode=airga.MODE_MIXED, inner_tol=1e-12, inner_max=k, poll_every=2,
                               max_sweeps=1)
        for c in range(2):
            assert st[c]["iters"] == k
            r = opcg.cocg(lambda v: ops[2] @ v, lambda v: spai.chain_apply(chain, v), f[c],
                          tol=1e-30, max_iter=k)
            assert rel_err(X[0, c].cpu().numpy(), r.x) < 1e-3, (k, c)


def test_mixed_cocg_matches_the_reference(ctx):
    """MIXED mode on the four points (factors and an update chain): every
    system reaches the float64 residual tol and the complex double-double
    reference, in a few sweeps."""
    pen = sur_beam()
    set_pencil(ctx, pen)
    rng = np.random.default_rng(2)
    f = np.stack([beam.tip_load(pen.n)[0], rng.standard_normal(pen.n)])
    F = to_dev(f, torch.float64)
    precs = [ctx.spai_build_complex(s) for s in SHIFTS]
    X, st = ctx.cocg_solve(SHIFTS, precs, F, tol=1e-10, mode=airga.MODE_MIXED)
    _, s64 = ctx.cocg_solve(SHIFTS, precs, F, tol=1e-10)
    Xh = X.cpu().numpy()
    for k, s in enumerate(SHIFTS):
        ref = direct.reference_solve_complex(pen, s, f, "dd")
        for c in range(2):
            e = st[2 * k + c]
            assert e["status"] == airga.SYS_CONVERGED, (s, c, e)
            assert e["relres"] <= 1e-10 and 2 <= e["sweeps"] <= 4, (s, c, e)
            assert rel_err(Xh[k, c], ref[c]) < 1e-8, (s, c)
            # float32 sweeps restart the Krylov space: at most a few times
            # the float64 iterations
            assert e["iters"] <= 3 * s64[2 * k + c]["iters"] + 64, (e, s64[2 * k + c])
    # a chain Q_3 Q_2 P_1 (float copies of every factor)
    pts = [complex(v * np.exp(1j * np.pi / 6)) for v in (30.0, 34.0, 38.0)]
    q3 = ctx.spai_update_complex(ctx.spai_update_complex(ctx.spai_build_complex(pts[0]), pts[1],
                                                         tol=0.05), pts[2], tol=0.05)
    assert q3.info().chain_len == 3
    X, st = ctx.cocg_solve([pts[2]], [q3], F, tol=1e-10, mode=airga.MODE_MIXED)
    ref = direct.reference_solve_complex(pen, pts[2], f, "dd")
    for c in range(2):
        assert st[c]["status"] == airga.SYS_CONVERGED and st[c]["relres"] <= 1e-10, st[c]
        assert rel_err(X[0, c].cpu().numpy(), ref[c]) < 1e-8


def test_mixed_cocg_edges_and_errors(ctx):
    pen = sur_beam(70)   # n = 140: three slices, the last ragged
    set_pencil(ctx, pen)
    f = np.zeros((2, pen.n))
    f[1, -2] = 1.0
    s = 4.0 + 3.0j
    p = ctx.spai_build_complex(s)
    F = to_dev(f, torch.float64)
    # a zero load is settled by the first residual: X = 0, no sweep
    X, st = ctx.cocg_solve([s], [p], F, mode=airga.MODE_MIXED)
    assert st[0]["status"] == airga.SYS_CONVERGED and st[0]["iters"] == 0 and st[0]["sweeps"] == 0
    assert torch.count_nonzero(X[0, 0]).item() == 0
    ref = direct.reference_solve_complex(pen, s, f[1:], "dd")[0]
    assert st[1]["status"] == airga.SYS_CONVERGED
    assert rel_err(X[0, 1].cpu().numpy(), ref) < 1e-8
    # no preconditioner; the sweep cap and the total iteration cap
    X, st = ctx.cocg_solve([s], None, F, mode=airga.MODE_MIXED)
    assert st[1]["status"] == airga.SYS_CONVERGED
    assert rel_err(X[0, 1].cpu().numpy(), ref) < 1e-8
    _, st = ctx.cocg_solve([s], [p], F, tol=1e-30, mode=airga.MODE_MIXED, max_sweeps=2)
    assert st[1]["status"] == airga.SYS_MAXIT and st[1]["sweeps"] == 2
    _, st = ctx.cocg_solve([s], [p], F, tol=1e-30, mode=airga.MODE_MIXED, max_iter=5,
                           inner_tol=1e-12, inner_max=4, poll_every=2)
    assert st[1]["status"] == airga.SYS_MAXIT and st[1]["sweeps"] == 2 and st[1]["iters"] == 8
    # a non-finite load: that system NONFINITE at once (X = 0), the other
    # one unaffected
    fn = f.copy()
    fn[0, 5] = np.nan
    X, st = ctx.cocg_solve([s], [p], to_dev(fn, torch.float64), mode=airga.MODE_MIXED)
    assert st[0]["status"] == airga.SYS_NONFINITE and st[0]["sweeps"] == 0
    assert torch.count_nonzero(X[0, 0]).item() == 0
    assert st[1]["status"] == airga.SYS_CONVERGED
    assert rel_err(X[0, 1].cpu().numpy(), ref) < 1e-8
    for bad in (dict(inner_tol=0.0), dict(inner_tol=1.0), dict(max_sweeps=0), dict(inner_max=-1)):
        with pytest.raises(airga.AirgaError) as e:
            ctx.cocg_solve([s], [p], F, mode=airga.MODE_MIXED, **bad)
        assert e.value.status == airga.EINVAL, bad
    with pytest.raises(airga.AirgaError) as e:
        ctx.cocg_solve([s], [p], F, mode=7)
    assert e.value.status == airga.EINVAL


def test_complex_edge_cases_and_errors(ctx):
    pen = sur_beam(70)   # n = 140: three slices, the last ragged
    set_pencil(ctx, pen)
    f = np.zeros((2, pen.n))
    f[1, -2] = 1.0      # a zero load converges at once with X = 0
    s = 4.0 + 3.0j
    p = ctx.spai_build_complex(s)
    X, st = ctx.cocg_solve([s], [p], to_dev(f, torch.float64))
    assert st[0]["status"] == airga.SYS_CONVERGED and st[0]["iters"] == 0
    assert torch.count_nonzero(X[0, 0]).item() == 0
    ref = direct.reference_solve_complex(pen, s, f[1:], "dd")[0]
    assert rel_err(X[0, 1].cpu().numpy(), ref) < 1e-8
    # a real shift through the complex path equals the real solve
    pr = ctx.spai_build_complex(25.0)
    Xc, _ = ctx.cocg_solve([25.0], [pr], to_dev(f, torch.float64))
    Xr = direct.reference_solve(pen, 25.0, f[1:], "dd")[0]
    assert np.abs(Xc[0, 1].cpu().numpy().imag).max() == 0.0
    assert rel_err(Xc[0, 1].cpu().numpy().real, Xr) < 1e-8
    # the real and complex calls refuse each other's factors
    real = ctx.spai_build(25.0)
    F = to_dev(f, torch.float64)
    with pytest.raises(airga.AirgaError) as e:
        ctx.pcg_solve([s.real], [p], F)
    assert e.value.status == airga.EINVAL
    with pytest.raises(airga.AirgaError) as e:
        ctx.cocg_solve([25.0], [real], F)
    assert e.value.status == airga.EINVAL
    with pytest.raises(airga.AirgaError) as e:
        ctx.cocg_solve([s + 1.0], [p], F)   # built at another shift
    assert e.value.status == airga.EINVAL
    with pytest.raises(airga.AirgaError) as e:
        ctx.spai_update(p, 30.0)
    assert e.value.status == airga.EUNSUPPORTED
    with pytest.raises(airga.AirgaError) as e:
        p.export()
    assert e.value.status == airga.EINVAL


def test_complex_full_size(ctx):
    """n = 1e6 surrogate beam, m = 4 seeded loads, 16 complex points
    s_k = sigma_k e^{i pi/6}, sigma_k logspace(0, 4, 16): all 64 systems in
    one batched COCG, in float64 and in MIXED mode, every one against the
    complex double-double reference (8 threads)."""
    pen, f, sig, _ = beam.make_workload("c3", surrogate=True)
    shifts = [complex(v) for v in np.asarray(sig) * np.exp(1j * np.pi / 6)]
    set_pencil(ctx, pen)
    precs = [ctx.spai_build_complex(s) for s in shifts]
    F = to_dev(f, torch.float64)
    X, st = ctx.cocg_solve(shifts, precs, F, tol=1e-10)
    assert all(e["status"] == airga.SYS_CONVERGED for e in st), [e for e in st if e["status"]]
    Xh = X.cpu().numpy()
    del X
    X, sm = ctx.cocg_solve(shifts, precs, F, tol=1e-10, mode=airga.MODE_MIXED)
    assert all(e["status"] == airga.SYS_CONVERGED and e["relres"] <= 1e-10 for e in sm), \
        [e for e in sm if e["status"]]
    Xm = X.cpu().numpy()
    del X
    errs = {}

    def check(k, ref):
        for c in range(f.shape[0]):
            errs[(k, c)] = rel_err(Xh[k, c], ref[c])
            errs[("mixed", k, c)] = rel_err(Xm[k, c], ref[c])
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(8) as ex:
        for k, ref in enumerate(ex.map(lambda s: direct.reference_solve_complex(pen, s, f, "dd"),
                                       shifts)):
            check(k, ref)
    bad = {key: e for key, e in errs.items() if not e < 1e-8}
    assert len(errs) == 128 and not bad, bad


def test_complex_updates_full_size(ctx):
    """n = 1e6: the 16 complex points' factors updated to points moved by
    up to 5% (seeded), every column's skip decision and every solved
    column's least squares on the full pencil, then COCG with the chains on
    all 64 systems, in float64 and in MIXED mode, every one within 1e-8 of
    the complex double-double reference.  Systems whose recurrence residual
    stalls above tol (COCG's short recurrences assume a complex symmetric
    preconditioner, which a chain is not) stop at the cap and must still
    meet 1e-8."""
    pen, f, sig, _ = beam.make_workload("c3", surrogate=True)
    e = np.exp(1j * np.pi / 6)
    drift = np.random.default_rng(7).uniform(-1.0, 1.0, len(sig))
    pts = [complex(v * e) for v in np.asarray(sig)]
    new = [complex(z * (1.0 + 0.05 * d)) for z, d in zip(pts, drift)]
    set_pencil(ctx, pen)
    old = [ctx.spai_build_complex(s) for s in pts]
    upd = [ctx.spai_update_complex(p, s) for p, s in zip(old, new)]
    infos = [u.info() for u in upd]
    assert any(0 < i.skipped_cols < pen.n for i in infos)
    F = to_dev(f, torch.float64)
    X, st = ctx.cocg_solve(new, upd, F, tol=1e-10, max_iter=2000)
    assert all(s["status"] in (airga.SYS_CONVERGED, airga.SYS_MAXIT) for s in st)
    assert sum(s["status"] == airga.SYS_CONVERGED for s in st) >= 56
    Xh = X.cpu().numpy()
    del X
    # MIXED mode: each sweep restarts from the float64 residual
    X, sm = ctx.cocg_solve(new, upd, F, tol=1e-10, max_iter=2000, mode=airga.MODE_MIXED)
    assert all(s["status"] in (airga.SYS_CONVERGED, airga.SYS_MAXIT) for s in sm)
    assert sum(s["status"] == airga.SYS_CONVERGED for s in sm) >= 56
    Xm = X.cpu().numpy()
    del X
    from concurrent.futures import ThreadPoolExecutor
    errs = {}
    with ThreadPoolExecutor(8) as ex:
        for k, ref in enumerate(ex.map(lambda s: direct.reference_solve_complex(pen, s, f, "dd"),
                                       new)):
            for c in range(f.shape[0]):
                errs[(k, c)] = rel_err(Xh[k, c], ref[c])
                errs[("mixed", k, c)] = rel_err(Xm[k, c], ref[c])
    bad = {key: v for key, v in errs.items() if not v < 1e-8}
    assert len(errs) == 128 and not bad, bad
