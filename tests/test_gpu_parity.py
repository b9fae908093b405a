"""GPU parity: the HIP library (through the C ABI) against the CPU oracle on
the same seeded inputs, at sizes the oracle finishes in seconds that span
several 64-row slices and a ragged tail."""
import numpy as np
import pytest
import torch

from gpu_util import (airga, beam, csr_of, direct, grid_pencil, pencil, reference, rel_err,
                      set_pencil, spai, to_dev)
from oracle import pcg as opcg

pytestmark = pytest.mark.gpu

SOLVE_TOL = 1e-8  # relative error vs the oracle solve for float64 and mixed solves


@pytest.fixture(scope="module")
def ctx():
    c = airga.Context(0)
    yield c
    c.close()


def sur_beam(n_el=1037, lu=(0.5, 2.0), seed=11):
    return beam.make_beam(n_el, ei_loguniform=lu, surrogate=True, seed=seed)


# ------------------------------------------------------------------ pencil

@pytest.mark.parametrize("n_el", [1, 37, 1037])
def test_pencil_info_and_assembly(ctx, n_el):
    pen = sur_beam(n_el)
    set_pencil(ctx, pen)
    info = ctx.pencil_info()
    assert info.n == pen.n and info.nnz == pen.nnz
    assert info.max_row_len == (2 if n_el == 1 else 4 if n_el == 2 else 6)
    assert info.bandwidth == (1 if n_el == 1 else 3)
    assert np.isclose(info.gram_mm, np.dot(pen.m_val, pen.m_val), rtol=1e-13)
    assert np.isclose(info.gram_mk, np.dot(pen.m_val, pen.k_val), rtol=1e-13)
    assert np.isclose(info.gram_kk, np.dot(pen.k_val, pen.k_val), rtol=1e-13)
    for s in (1.0, 37.5, 1e4):
        got = ctx.assemble_shift(s).cpu().numpy()
        ref = pencil.shifted_values(pen.m_val, pen.k_val, pen.alpha, pen.beta, s)
        a, b = s * s + pen.alpha * s, 1 + pen.beta * s
        bound = 8e-16 * (np.abs(a * pen.m_val) + np.abs(b * pen.k_val)) + 1e-300
        assert np.all(np.abs(got - ref) <= bound)


def test_apply_shift(ctx):
    pen = sur_beam()
    set_pencil(ctx, pen)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, pen.n))
    for s in (2.0, 500.0):
        y = ctx.apply_shift(s, to_dev(x, torch.float64)).cpu().numpy()
        a = pencil.shifted_operator(pen, s)
        ref = np.stack([a @ xi for xi in x])
        scale = np.stack([abs(a) @ np.abs(xi) for xi in x])
        assert np.all(np.abs(y - ref) <= 1e-14 * scale + 1e-300)


def test_shift_diagnostics(ctx):
    pen = sur_beam(200)
    set_pencil(ctx, pen)
    for so, sn in ((1.0, 1.01), (10.0, 37.0), (1e3, 999.0)):
        d = ctx.shift_diagnostics(so, sn)
        i_a, d_a = pencil.frobenius_diagnostics(pen, so, sn)
        assert np.isclose(d[0], i_a, rtol=1e-9)
        assert np.isclose(d[1], d_a, rtol=1e-9)
        an = pencil.shifted_operator(pen, sn)
        ao = pencil.shifted_operator(pen, so)
        assert np.isclose(d[2], spai.spai_build(an, cols=[0]).alpha, rtol=1e-12)
        assert np.isclose(d[3], spai.update_alpha(ao, an), rtol=1e-12)


def test_invalid_pencils_are_rejected(ctx):
    pen = sur_beam(20)
    bad = [
        ("asymmetric", lambda rp, ci: (rp, np.where(np.arange(ci.size) == 2, ci + 1, ci))),
        ("unsorted", lambda rp, ci: (rp, np.concatenate([ci[:4][::-1], ci[4:]]))),
        ("out of range", lambda rp, ci: (rp, np.where(np.arange(ci.size) == 5, 10 ** 6, ci))),
    ]
    for name, f in bad:
        rp, ci = f(pen.row_ptr.copy(), pen.col_idx.copy())
        with pytest.raises(airga.AirgaError) as ei:
            ctx.set_pencil(to_dev(rp, torch.int32), to_dev(ci, torch.int32),
                           to_dev(pen.m_val, torch.float64), to_dev(pen.k_val, torch.float64),
                           pen.alpha, pen.beta)
        assert ei.value.status == airga.EINVAL, name
    # a missing diagonal: drop the diagonal entry of row 0
    rp, ci = pen.row_ptr.copy(), pen.col_idx.copy()
    keep = np.ones(ci.size, bool)
    keep[0] = False  # row 0 starts with its diagonal (column 0)
    rp2 = rp.copy()
    rp2[1:] -= 1
    with pytest.raises(airga.AirgaError) as ei:
        ctx.set_pencil(to_dev(rp2, torch.int32), to_dev(ci[keep], torch.int32),
                       to_dev(pen.m_val[keep], torch.float64), to_dev(pen.k_val[keep], torch.float64),
                       pen.alpha, pen.beta)
    assert ei.value.status == airga.EINVAL
    # calls after a failed set_pencil see no pencil
    with pytest.raises(airga.AirgaError) as ei:
        ctx.assemble_shift(1.0, torch.empty(pen.nnz, dtype=torch.float64, device="cuda"))
    assert ei.value.status == airga.ESTATE


# -------------------------------------------------------------------- SPAI

def _check_factor(fac_gpu_vals, fac_gpu_obj, ref, cols, rtol_vals=1e-9):
    obj_ref = ref.objective[cols]
    assert np.all(np.abs(fac_gpu_obj[cols] - obj_ref) <= 1e-12 * np.maximum(1.0, obj_ref))
    assert np.all(np.abs(fac_gpu_vals - ref.values) <= rtol_vals * np.abs(ref.values).max())


@pytest.mark.parametrize("sur,s,lu", [(True, 1.0, (0.5, 2.0)), (True, 250.0, (0.1, 10.0)),
                                      (False, 100.0, None)])
def test_spai_build_matches_oracle(ctx, sur, s, lu):
    pen = beam.make_beam(301, ei_loguniform=lu, surrogate=sur, seed=2)
    set_pencil(ctx, pen)
    a = pencil.shifted_operator(pen, s)
    # raw (unsymmetrised) columns: values, objectives and optimality
    ref = spai.spai_build(a, symmetrize=False)
    p = ctx.spai_build(s, symmetrize=False)
    vals, obj = (t.cpu().numpy() for t in p.export())
    _check_factor(vals, obj, ref, np.arange(pen.n), rtol_vals=1e-9 if sur else 1e-7)
    # the default (symmetrised) factor
    ref_s = spai.spai_build(a)
    vals_s, obj_s = (t.cpu().numpy() for t in ctx.spai_build(s).export())
    _check_factor(vals_s, obj_s, ref_s, np.arange(pen.n), rtol_vals=1e-9 if sur else 1e-7)
    info = p.info()
    assert info.chain_len == 1 and info.skipped_cols == 0 and info.scalar_only == 0
    assert np.isclose(info.alpha, ref.alpha, rtol=1e-12)
    # the GPU columns are least-squares optimal in their own right
    d = a.diagonal()
    sc = 1 / np.sqrt(d)
    ah = (np.diag(sc) @ a.toarray() @ np.diag(sc))
    phat = csr_of(pen, vals).toarray() / np.outer(sc, sc)
    for j in range(0, pen.n, 7):
        jj = pen.col_idx[pen.row_ptr[j]:pen.row_ptr[j + 1]]
        res = np.eye(pen.n)[:, j] - ah[:, jj] @ phat[jj, j]
        assert np.linalg.norm(ah[:, jj].T @ res) <= 1e-11 * np.linalg.norm(ah[:, jj]) * max(np.linalg.norm(res), 1e-300)


def test_spai_build_symmetrize_and_unscaled(ctx):
    pen = sur_beam(150)
    set_pencil(ctx, pen)
    a = pencil.shifted_operator(pen, 3.0)
    for eq, sym in ((True, False), (False, False), (False, True)):
        ref = spai.spai_build(a, equilibrate=eq, symmetrize=sym)
        vals, obj = (t.cpu().numpy() for t in ctx.spai_build(3.0, equilibrate=eq, symmetrize=sym).export())
        _check_factor(vals, obj, ref, np.arange(pen.n), rtol_vals=1e-8)


def test_spai_on_a_two_dimensional_pattern(ctx):
    pen = grid_pencil(23, 17)
    set_pencil(ctx, pen)
    for s in (0.5, 20.0):
        a = pencil.shifted_operator(pen, s)
        ref = spai.spai_build(a)
        vals, obj = (t.cpu().numpy() for t in ctx.spai_build(s).export())
        _check_factor(vals, obj, ref, np.arange(pen.n), rtol_vals=1e-10)


@pytest.mark.parametrize("s_old,s_new,tol", [(100.0, 101.0, 0.01), (10.0, 13.0, 0.01),
                                             (10.0, 10.5, 0.0), (4.0, 4.0, 0.01)])
def test_spai_update_matches_oracle(ctx, s_old, s_new, tol):
    pen = sur_beam(400)
    set_pencil(ctx, pen)
    a_old = pencil.shifted_operator(pen, s_old)
    a_new = pencil.shifted_operator(pen, s_new)
    ref = spai.spai_update(a_old, a_new, tol=tol)
    p_old = ctx.spai_build(s_old)
    q = ctx.spai_update(p_old, s_new, tol=tol)
    vals, obj = (t.cpu().numpy() for t in q.export())
    info = q.info()
    assert np.isclose(info.alpha, ref.alpha, rtol=1e-12)
    # skip decisions are exact except within 1e-12 of the threshold
    d = a_new.diagonal()
    s = 1 / np.sqrt(d)
    oh = (np.diag(s) @ a_old.toarray() @ np.diag(s))
    nh = (np.diag(s) @ a_new.toarray() @ np.diag(s))
    ratio = np.linalg.norm(oh - ref.alpha * nh, axis=0) / np.linalg.norm(oh, axis=0)
    clear = np.abs(ratio - tol) > 1e-12
    assert info.skipped_cols == int(ref.skipped.sum()) or not np.all(clear)
    _check_factor(vals, obj, ref, np.arange(pen.n)[clear], rtol_vals=1e-9)
    assert bool(info.scalar_only) == ref.scalar_only
    if s_old == s_new:
        assert info.scalar_only and np.isclose(info.alpha, 1.0, rtol=1e-15)


def test_chain_apply_matches_oracle(ctx):
    pen = sur_beam(300)
    set_pencil(ctx, pen)
    shifts = [5.0, 5.3, 5.9]
    facs = [spai.spai_build(pencil.shifted_operator(pen, shifts[0]))]
    handles = [ctx.spai_build(shifts[0])]
    for so, sn in zip(shifts[:-1], shifts[1:]):
        facs.append(spai.spai_update(pencil.shifted_operator(pen, so),
                                     pencil.shifted_operator(pen, sn), tol=0.0))
        handles.append(ctx.spai_update(handles[-1], sn, tol=0.0))
    assert handles[-1].info().chain_len == 3
    r = np.random.default_rng(3).standard_normal((2, pen.n))
    z = handles[-1].apply(to_dev(r, torch.float64)).cpu().numpy()
    ref = np.stack([spai.chain_apply(facs, ri) for ri in r])
    assert np.allclose(z, ref, rtol=1e-11, atol=1e-12 * np.abs(ref).max())


def test_spai_rejects_long_rows_and_bad_shift(ctx):
    n = 9
    rng = np.random.default_rng(0)
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    k = q @ np.diag(rng.uniform(1, 2, n)) @ q.T
    m = np.eye(n) + 0.01 * (k + k.T)
    rp = np.arange(0, n * n + 1, n, dtype=np.int32)
    ci = np.tile(np.arange(n, dtype=np.int32), n)
    ctx.set_pencil(to_dev(rp, torch.int32), to_dev(ci, torch.int32),
                   to_dev(m.ravel(), torch.float64), to_dev(k.ravel(), torch.float64), 0.01, 0.001)
    with pytest.raises(airga.AirgaError) as ei:
        ctx.spai_build(1.0)
    assert ei.value.status == airga.EUNSUPPORTED
    # the solver itself handles rows of up to 16 entries (no preconditioner)
    f = np.zeros((1, n)); f[0, 3] = 1.0
    X, st = ctx.pcg_solve([2.0], [None], to_dev(f, torch.float64), tol=1e-13)
    ref = np.linalg.solve((4 + 0.02) * m + (1 + 0.002) * k, f[0])
    assert st[0]["status"] == airga.SYS_CONVERGED
    assert rel_err(X.cpu().numpy()[0, 0], ref) < 1e-11
    pen = sur_beam(10)
    set_pencil(ctx, pen)
    for s in (0.0, -1.0, float("nan")):
        with pytest.raises(airga.AirgaError) as ei:
            ctx.spai_build(s)
        assert ei.value.status == airga.EINVAL


# ------------------------------------------------------------------- solves

@pytest.mark.parametrize("mode", [airga.MODE_FP64, airga.MODE_MIXED])
def test_batched_solve_matches_reference(ctx, mode):
    pen = sur_beam(1037, lu=(0.1, 10.0))
    set_pencil(ctx, pen)
    rng = np.random.default_rng(5)
    f, _ = beam.node_loads(pen.n, 3, rng)
    shifts = [1.0, 7.0, 130.0, 9000.0]
    precs = [ctx.spai_build(s) for s in shifts]
    X, st = ctx.pcg_solve(shifts, precs, to_dev(f, torch.float64), tol=1e-10, mode=mode)
    Xh = X.cpu().numpy()
    ref = reference(pen, shifts, f)
    for k, s in enumerate(shifts):
        for c in range(3):
            e = st[k * 3 + c]
            assert e["status"] == airga.SYS_CONVERGED, (s, c, e)
            assert e["relres"] <= 1e-10
            assert rel_err(Xh[k, c], ref[k, c]) < SOLVE_TOL, (s, c)


@pytest.mark.parametrize("form,oracle_beta", [(airga.BETA_FLEXIBLE, "flexible"),
                                              (airga.BETA_CLASSICAL, "fr")])
def test_fp64_iterates_follow_the_oracle_recurrence(ctx, form, oracle_beta):
    """Both direction updates against the oracle's (the symmetrised build is a
    symmetric factor, so the classical ratio applies too)."""
    pen = sur_beam(700)
    set_pencil(ctx, pen)
    f = beam.tip_load(pen.n)
    for s in (1.0, 100.0):
        a = pencil.shifted_operator(pen, s)
        pm = spai.spai_build(a).matrix()
        ref = opcg.pcg(lambda v: a @ v, lambda v: pm @ v, f[0], tol=1e-10, max_iter=5000,
                       beta=oracle_beta)
        X, st = ctx.pcg_solve([s], [ctx.spai_build(s)], to_dev(f, torch.float64), tol=1e-10,
                              beta_form=form)
        assert st[0]["status"] == airga.SYS_CONVERGED
        assert abs(st[0]["iters"] - ref.iters) <= 2, (st[0], ref.iters)
        assert rel_err(X.cpu().numpy()[0, 0], ref.x) < 1e-9
        # stopping after exactly the oracle's iteration count gives the same iterate
        k = min(ref.iters, 6)
        r6 = opcg.pcg(lambda v: a @ v, lambda v: pm @ v, f[0], tol=0.0, max_iter=k,
                      beta=oracle_beta)
        X6, st6 = ctx.pcg_solve([s], [ctx.spai_build(s)], to_dev(f, torch.float64), tol=0.0,
                                max_iter=k, beta_form=form)
        assert st6[0]["status"] == airga.SYS_MAXIT and st6[0]["iters"] == k
        assert rel_err(X6.cpu().numpy()[0, 0], r6.x) < 1e-12


def test_mixed_inner_iterates_follow_the_oracle(ctx):
    """MIXED mode stopped by max_iter inside its first sweep: X is the float32
    PCG iterate after k steps (the sweep's correction added to X = 0), the
    oracle's float64 iterate to float32 accuracy, for odd and even k."""
    pen = sur_beam(700)
    set_pencil(ctx, pen)
    f = beam.tip_load(pen.n)
    F = to_dev(f, torch.float64)
    for s in (1.0, 100.0):
        a = pencil.shifted_operator(pen, s)
        pm = spai.spai_build(a).matrix()
        p = ctx.spai_build(s)
        for k in (1, 2, 3, 6, 7):
            r = opcg.pcg(lambda v: a @ v, lambda v: pm @ v, f[0], tol=0.0, max_iter=k,
                         beta="flexible")
            X, st = ctx.pcg_solve([s], [p], F, tol=1e-30, mode=airga.MODE_MIXED, max_iter=k,
                                  inner_tol=1e-12, max_sweeps=1, poll_every=2)
            assert st[0]["status"] == airga.SYS_MAXIT and st[0]["iters"] == k, (s, k, st[0])
            assert rel_err(X.cpu().numpy()[0, 0], r.x) < 1e-3, (s, k)


def test_solve_with_update_chain(ctx):
    pen = sur_beam(900)
    set_pencil(ctx, pen)
    f = beam.tip_load(pen.n)
    p1 = ctx.spai_build(20.0)
    q2 = ctx.spai_update(p1, 21.0, tol=0.0)   # a real factor
    q3 = ctx.spai_update(q2, 21.2, tol=0.01)  # collapses to a scalar
    assert q2.info().chain_len == 2 and q3.info().scalar_only == 1 and q3.info().chain_len == 2
    # oracle with the same chain
    a1, a2, a3 = (pencil.shifted_operator(pen, s) for s in (20.0, 21.0, 21.2))
    assert spai.spai_update(a2, a3, tol=0.01).scalar_only
    facs = [spai.spai_build(a1), spai.spai_update(a1, a2, tol=0.0)]
    ref = opcg.pcg(lambda v: a2 @ v, lambda v: spai.chain_apply(facs, v), f[0], tol=1e-10)
    for mode in (airga.MODE_FP64, airga.MODE_MIXED):
        X, st = ctx.pcg_solve([21.0, 21.2], [q2, q3], to_dev(f, torch.float64), tol=1e-10, mode=mode)
        refs = reference(pen, [21.0, 21.2], f)
        assert all(e["status"] == airga.SYS_CONVERGED for e in st), st
        assert rel_err(X.cpu().numpy()[0, 0], refs[0, 0]) < SOLVE_TOL
        assert rel_err(X.cpu().numpy()[1, 0], refs[1, 0]) < SOLVE_TOL
        if mode == airga.MODE_FP64:
            assert abs(st[0]["iters"] - ref.iters) <= 2


def test_two_dimensional_pattern_solve(ctx):
    pen = grid_pencil(31, 29)
    set_pencil(ctx, pen)
    f = np.zeros((2, pen.n)); f[0, 17] = 1; f[1, 500] = 1
    shifts = [0.5, 3.0]
    precs = [ctx.spai_build(s) for s in shifts]
    for mode in (airga.MODE_FP64, airga.MODE_MIXED):
        X, st = ctx.pcg_solve(shifts, precs, to_dev(f, torch.float64), mode=mode)
        ref = reference(pen, shifts, f, "f64")
        for k in range(2):
            for c in range(2):
                assert st[2 * k + c]["status"] == airga.SYS_CONVERGED
                assert rel_err(X.cpu().numpy()[k, c], ref[k, c]) < SOLVE_TOL


def test_edge_cases(ctx):
    pen = sur_beam(37)  # n = 74: two slices, ragged tail
    set_pencil(ctx, pen)
    n = pen.n
    f = np.zeros((3, n))
    f[1, n - 2] = 1.0
    f[2, 5] = np.nan
    p = ctx.spai_build(3.0)
    for mode in (airga.MODE_FP64, airga.MODE_MIXED):
        X, st = ctx.pcg_solve([3.0], [p], to_dev(f, torch.float64), mode=mode)
        Xh = X.cpu().numpy()
        assert st[0]["status"] == airga.SYS_CONVERGED and st[0]["iters"] == 0 and not np.any(Xh[0, 0])
        assert st[1]["status"] == airga.SYS_CONVERGED
        assert st[2]["status"] == airga.SYS_NONFINITE
        _, st1 = ctx.pcg_solve([3.0], [p], to_dev(f[1:2], torch.float64), mode=mode, max_iter=1,
                               tol=1e-14)
        assert st1[0]["status"] == airga.SYS_MAXIT and st1[0]["iters"] == 1
        # without a starting guess X is written whatever it held: zero for a
        # zero right-hand side (also when no system iterates at all)
        ref1 = reference(pen, [3.0], f[1:2])
        for fx in (f[:2], np.zeros((2, n))):
            Xn = torch.full((1, 2, n), float("nan"), dtype=torch.float64, device="cuda")
            _, st2 = ctx.pcg_solve([3.0], [p], to_dev(fx, torch.float64), Xn, mode=mode)
            Xh2 = Xn.cpu().numpy()
            assert not np.any(Xh2[0, 0]) and st2[0]["status"] == airga.SYS_CONVERGED
            if fx[1].any():
                assert rel_err(Xh2[0, 1], ref1[0, 0]) < SOLVE_TOL
            else:
                assert not np.any(Xh2[0, 1])
    # no preconditioner at all
    X, st = ctx.pcg_solve([3.0], [None], to_dev(f[1:2], torch.float64))
    ref = reference(pen, [3.0], f[1:2])
    assert st[0]["status"] == airga.SYS_CONVERGED and rel_err(X.cpu().numpy()[0, 0], ref[0, 0]) < SOLVE_TOL
    # one element: n = 2
    tiny = sur_beam(1)
    set_pencil(ctx, tiny)
    ft = np.array([[1.0, 0.0]])
    X, st = ctx.pcg_solve([2.0], [ctx.spai_build(2.0)], to_dev(ft, torch.float64))
    ref = reference(tiny, [2.0], ft)
    assert st[0]["status"] == airga.SYS_CONVERGED and rel_err(X.cpu().numpy()[0, 0], ref[0, 0]) < 1e-12


def test_batch_with_a_ragged_second_chunk_of_systems(ctx):
    """70 systems (14 shifts x 5 columns): the row kernels read the systems'
    activity flags 64 at a time, so the second chunk holds 6 systems; they
    converge at different iterations across both chunks."""
    pen = sur_beam(300)
    set_pencil(ctx, pen)
    rng = np.random.default_rng(21)
    f = rng.standard_normal((5, pen.n))
    shifts = list(np.logspace(0, 3, 14))
    precs = ctx.spai_build_many(shifts)
    ref = reference(pen, shifts, f)
    for mode in (airga.MODE_FP64, airga.MODE_MIXED):
        X, st = ctx.pcg_solve(shifts, precs, to_dev(f, torch.float64), mode=mode, tol=1e-10)
        assert len(st) == 70 and all(e["status"] == airga.SYS_CONVERGED for e in st)
        iters = [e["iters"] for e in st]
        assert len(set(iters)) > 1
        Xh = X.cpu().numpy()
        for k in range(14):
            for c in range(5):
                assert rel_err(Xh[k, c], ref[k, c]) < SOLVE_TOL, (mode, k, c)


def test_warm_start_graph_and_profile_agree(ctx):
    pen = sur_beam(1037)
    set_pencil(ctx, pen)
    rng = np.random.default_rng(8)
    f, _ = beam.node_loads(pen.n, 2, rng)
    fd = to_dev(f, torch.float64)
    shifts = [1.5, 40.0]
    precs = [ctx.spai_build(s) for s in shifts]
    for mode in (airga.MODE_FP64, airga.MODE_MIXED):
        Xg, sg = ctx.pcg_solve(shifts, precs, fd, mode=mode, use_graph=True)
        Xn, sn = ctx.pcg_solve(shifts, precs, fd, mode=mode, use_graph=False)
        Xp, sp_ = ctx.pcg_solve(shifts, precs, fd, mode=mode, profile=True)
        assert torch.equal(Xg, Xn) and torch.equal(Xg, Xp)  # deterministic reductions
        assert [e["iters"] for e in sg] == [e["iters"] for e in sn]
        times = ctx.kernel_times()
        assert times["dir_spmv"][0] > 0 and times["dir_spmv"][1] > 0
        # resume from a loose solve
        X1, s1 = ctx.pcg_solve(shifts, precs, fd, mode=mode, tol=1e-4)
        X2, s2 = ctx.pcg_solve(shifts, precs, fd, X=X1, mode=mode, x0_given=True)
        ref = reference(pen, shifts, f)
        for k in range(2):
            for c in range(2):
                assert s2[2 * k + c]["status"] == airga.SYS_CONVERGED
                assert rel_err(X2.cpu().numpy()[k, c], ref[k, c]) < SOLVE_TOL
        assert sum(e["iters"] for e in s2) < sum(e["iters"] for e in sg)


def c1_float64_floor(pen, f, s):
    """The accuracy binary64 itself reaches on the literal 1000-DOF beam at
    s = 100 (condition number about 3e10): the oracle's binary64 banded
    Cholesky and its plain float64 PCG to 1e-10, each against the
    double-double reference.  Both stop near 1e-8, so no float64 solver can
    be held to 1e-8 here; the GPU is held to twice the larger of the two."""
    ref = direct.reference_solve(pen, s, f, "dd")[0]
    chol = rel_err(direct.reference_solve(pen, s, f, "f64")[0], ref)
    a = pencil.shifted_operator(pen, s)
    pmat = spai.spai_build(a).matrix()
    r = opcg.pcg(lambda v: a @ v, lambda v: pmat @ v, f[0], tol=1e-10, max_iter=40000)
    assert r.status == opcg.CONVERGED
    return ref, chol, rel_err(r.x, ref)


def test_literal_cantilever_c1(ctx):
    """n = 1000 Hermite cantilever, EI = 1, single shift s = 100, tip load,
    SPAI on the pattern of K(s), CG to 1e-10 relative residual.  Tolerance:
    twice the binary64 floor measured on the oracle (1.8e-8 for its banded
    Cholesky, 1.1e-8 for its PCG), which itself is pinned below 3e-8."""
    pen, f, shifts, _ = beam.make_workload("c1")
    ref, chol, opcg_err = c1_float64_floor(pen, f, shifts[0])
    floor = max(chol, opcg_err)
    assert 5e-9 < floor < 3e-8, (chol, opcg_err)
    set_pencil(ctx, pen)
    p = ctx.spai_build(shifts[0])
    X, st = ctx.pcg_solve(list(shifts), [p], to_dev(f, torch.float64), tol=1e-10, max_iter=40000)
    assert st[0]["status"] == airga.SYS_CONVERGED, st
    assert rel_err(X.cpu().numpy()[0, 0], ref) < 2 * floor
    # mixed precision: float32 cannot resolve this system (condition number
    # near 1/eps_32), so the first capped sweep hands it to the float64 finish
    Xm, sm = ctx.pcg_solve(list(shifts), [p], to_dev(f, torch.float64), tol=1e-10, max_iter=40000,
                           mode=airga.MODE_MIXED)
    assert sm[0]["status"] == airga.SYS_CONVERGED and sm[0]["finished_fp64"] == 1, sm
    assert rel_err(Xm.cpu().numpy()[0, 0], ref) < 2 * floor


def indefinite_pencil(n):
    """A pencil with positive diagonals whose K(s) is indefinite for small s:
    K tridiagonal with 1 on the diagonal and 2 beside it (eigenvalues
    1 + 4 cos(k pi / (n + 1)), some negative), M = 1e-3 I."""
    rp, ci, kv, mv = [0], [], [], []
    for i in range(n):
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                ci.append(j)
                kv.append(1.0 if j == i else 2.0)
                mv.append(1e-3 if j == i else 0.0)
        rp.append(len(ci))
    return beam.Pencil(n=n, row_ptr=np.array(rp, np.int32), col_idx=np.array(ci, np.int32),
                       m_val=np.array(mv), k_val=np.array(kv), alpha=0.0, beta=0.0)


@pytest.mark.parametrize("mode", [airga.MODE_FP64, airga.MODE_MIXED])
def test_breakdown_on_an_indefinite_shifted_matrix(ctx, mode):
    """(p, K(s) p) <= 0 stops a system with BREAKDOWN, as in the oracle:
    without a preconditioner the first direction is the load f, and
    f^T K(s) f < 0 for the alternating-sign load.  In the same batch, a load
    along an eigenvector of K(s) with a positive eigenvalue lambda converges
    in one step to f / lambda."""
    n = 150
    pen = indefinite_pencil(n)
    set_pencil(ctx, pen)
    s = 0.5
    a = pencil.shifted_operator(pen, s)
    alt = np.array([(-1.0) ** i for i in range(n)])
    assert alt @ (a @ alt) < 0
    v1 = np.sin(np.arange(1, n + 1) * np.pi / (n + 1))
    lam = s * s * 1e-3 + 1.0 + 4.0 * np.cos(np.pi / (n + 1))
    assert np.linalg.norm(a @ v1 - lam * v1) < 1e-13 * lam * np.linalg.norm(v1)
    f = np.stack([alt, v1])
    ref = opcg.pcg(lambda v: a @ v, lambda v: v, f[0], tol=1e-10, max_iter=400)
    assert ref.status == opcg.BREAKDOWN and ref.iters == 0
    X, st = ctx.pcg_solve([s], [None], to_dev(f, torch.float64), tol=1e-10, max_iter=400, mode=mode)
    assert st[0]["status"] == airga.SYS_BREAKDOWN and st[0]["iters"] == 0, st
    if mode == airga.MODE_FP64:
        assert st[1]["status"] == airga.SYS_CONVERGED, st
        assert rel_err(X.cpu().numpy()[0, 1], v1 / lam) < 1e-12
    else:
        # the float32 sweep lands within float32 rounding of f / lambda; the
        # next directions are rounding noise, on which the indefinite K(s)
        # may curve either way, so the float64 refinement either converges
        # or reports the breakdown, after that first step
        assert st[1]["status"] in (airga.SYS_CONVERGED, airga.SYS_BREAKDOWN), st
        assert st[1]["relres"] < 1e-6 and rel_err(X.cpu().numpy()[0, 1], v1 / lam) < 1e-6


@pytest.mark.parametrize("inner_max", [8, 16])
def test_mixed_handover_to_float64_finish(ctx, inner_max):
    """Systems still iterating at the per-sweep cap leave the float32 sweeps
    and finish in float64 from their current X, batched; every system still
    meets the oracle tolerance, the flags name the handed ones, and a cap
    too large to bind hands none over."""
    pen = beam.make_beam(1500, ei_loguniform=(0.1, 10.0), surrogate=True, seed=6)
    set_pencil(ctx, pen)
    rng = np.random.default_rng(2)
    f = np.stack([beam.tip_load(pen.n)[0], rng.standard_normal(pen.n)])
    shifts = [1.0, 8.0, 300.0]
    precs = [ctx.spai_build(s) for s in shifts]
    ref = reference(pen, shifts, f)
    F = to_dev(f, torch.float64)
    X, st = ctx.pcg_solve(shifts, precs, F, tol=1e-10, mode=airga.MODE_MIXED, inner_max=inner_max)
    Xh = X.cpu().numpy()
    for k in range(3):
        for c in range(2):
            e = st[2 * k + c]
            assert e["status"] == airga.SYS_CONVERGED, e
            assert rel_err(Xh[k, c], ref[k, c]) < SOLVE_TOL, (k, c, e)
    assert any(e["finished_fp64"] for e in st)
    # without the cap nothing is handed over; float32 refinement alone then
    # fails on the low shift (its condition number defeats float32), and
    # says so: every system reported converged meets the tolerance
    X2, st2 = ctx.pcg_solve(shifts, precs, F, tol=1e-10, mode=airga.MODE_MIXED, inner_max=100000)
    assert not any(e["finished_fp64"] for e in st2)
    Xh2 = X2.cpu().numpy()
    for k in range(3):
        for c in range(2):
            e = st2[2 * k + c]
            if e["status"] == airga.SYS_CONVERGED:
                assert rel_err(Xh2[k, c], ref[k, c]) < SOLVE_TOL, (k, c, e)
            else:
                assert e["status"] == airga.SYS_MAXIT and e["relres"] > 1e-10, e


# --------------------------------------------------------- moment matching

def test_gpu_solves_make_the_projection_interpolate():
    """Galerkin projection onto GPU solves X(s_i) and first moments (RHS
    -(2 s M + D) X(s_i), Section 2) interpolates the full transfer function
    and its derivative at the expansion points; H from an independent dense
    solve.  Pins the solve chain as a whole."""
    from oracle import moments
    c = airga.Context(0)
    try:
        p = beam.make_beam(190, ei_loguniform=(0.5, 2.0), surrogate=True, seed=4)
        set_pencil(c, p)
        m, k = beam.pencil_dense(p)
        d = p.alpha * m + p.beta * k
        f = beam.tip_load(p.n)          # (1, n)
        cp = f.copy()
        shifts = [1.5, 40.0, 900.0]
        precs = [c.spai_build(s) for s in shifts]
        X0, st0 = c.pcg_solve(shifts, precs, to_dev(f, torch.float64), tol=1e-12,
                              mode=airga.MODE_MIXED)
        assert all(e["status"] == airga.SYS_CONVERGED for e in st0)
        x0 = X0.cpu().numpy()[:, 0, :]  # (nshift, n)
        xs = []
        for i, s in enumerate(shifts):
            rhs = -((2 * s) * m + d) @ x0[i]
            X1, st1 = c.pcg_solve([s], [precs[i]], to_dev(rhs[None, :], torch.float64),
                                  tol=1e-12, mode=airga.MODE_FP64)
            assert st1[0]["status"] == airga.SYS_CONVERGED
            xs += [x0[i][:, None], X1.cpu().numpy()[0, 0][:, None]]
        v = moments.orth_basis(xs)
        red = moments.project(m, k, p.alpha, p.beta, f.T, cp, v)

        def h_full(s):
            return cp @ np.linalg.solve(s * s * m + s * d + k, f.T)

        for s in shifts:
            assert np.allclose(moments.reduced_transfer(*red, s), h_full(s), rtol=1e-9)
            e = 1e-4 * s
            dfull = (h_full(s + e) - h_full(s - e)) / (2 * e)
            dred = (moments.reduced_transfer(*red, s + e) - moments.reduced_transfer(*red, s - e)) / (2 * e)
            assert np.allclose(dred, dfull, rtol=1e-5)
    finally:
        c.close()
