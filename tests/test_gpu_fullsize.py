"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark times (batched mixed precision, all shifts and columns at once):
every system against the oracle's reference solve, SPAI columns on samples
the oracle computes one by one."""
import numpy as np
import pytest
import torch

from gpu_util import airga, beam, direct, pencil, rel_err, set_pencil, spai, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = airga.Context(0)
    yield c
    c.close()


def _sample_cols(n, rng, k=300):
    edge = np.array([0, 1, 2, 3, n - 4, n - 3, n - 2, n - 1])
    return np.unique(np.concatenate([edge, rng.choice(n, k, replace=False)]))


def test_c4_surrogate_full_size(ctx):
    """n = 1e6, m = 4 seeded loads, 16 shifts logspace(0, 4, 16), mixed."""
    pen, f, shifts, rng = beam.make_workload("c3", surrogate=True)
    set_pencil(ctx, pen)
    precs = [ctx.spai_build(s) for s in shifts]
    # SPAI columns at sampled positions against the oracle's column solves
    cols = _sample_cols(pen.n, np.random.default_rng(1))
    for k in (0, 7, 15):
        ref = spai.spai_build(pencil.shifted_operator(pen, shifts[k]), cols=cols)
        _, obj = precs[k].export()
        obj = obj.cpu().numpy()
        assert np.all(np.abs(obj[cols] - ref.objective[cols]) <= 1e-12 * np.maximum(1, ref.objective[cols]))
    X, st = ctx.pcg_solve(list(shifts), precs, to_dev(f, torch.float64), tol=1e-10,
                          mode=airga.MODE_MIXED)
    Xh = X.cpu().numpy()
    for k, s in enumerate(shifts):
        ref = direct.reference_solve(pen, s, f, "dd")
        for c in range(f.shape[0]):
            e = st[k * f.shape[0] + c]
            assert e["status"] == airga.SYS_CONVERGED, (s, c, e)
            assert rel_err(Xh[k, c], ref[c]) < 1e-8, (s, c)


def test_c3_batched_fp64_full_size(ctx):
    """Same systems in float64 (batched, no refinement)."""
    pen, f, shifts, rng = beam.make_workload("c3", surrogate=True)
    set_pencil(ctx, pen)
    sel = [0, 5, 10, 15]
    precs = [ctx.spai_build(shifts[k]) for k in sel]
    X, st = ctx.pcg_solve([shifts[k] for k in sel], precs, to_dev(f, torch.float64), tol=1e-10,
                          mode=airga.MODE_FP64)
    Xh = X.cpu().numpy()
    for i, k in enumerate(sel):
        ref = direct.reference_solve(pen, shifts[k], f, "dd")
        for c in range(f.shape[0]):
            assert st[i * f.shape[0] + c]["status"] == airga.SYS_CONVERGED
            assert rel_err(Xh[i, c], ref[c]) < 1e-8


def test_c2_surrogate_update_sequence(ctx):
    """n = 1e5, tip load, 8 shifts: build at every shift, then vertical
    updates to drifted shifts (all columns skip -> scalar factors)."""
    pen, f, shifts, rng = beam.make_workload("c2", surrogate=True)
    drifted = beam.drift_shifts(shifts, 1e-3, rng)
    set_pencil(ctx, pen)
    precs = [ctx.spai_build(s) for s in shifts]
    upd = [ctx.spai_update(p, s) for p, s in zip(precs, drifted)]
    X, st = ctx.pcg_solve(list(drifted), upd, to_dev(f, torch.float64), tol=1e-10,
                          mode=airga.MODE_MIXED)
    Xh = X.cpu().numpy()
    for k, s in enumerate(drifted):
        ref = direct.reference_solve(pen, s, f, "dd")
        assert st[k]["status"] == airga.SYS_CONVERGED
        assert rel_err(Xh[k, 0], ref[0]) < 1e-8
    # update skip counts against the oracle at sampled columns
    cols = _sample_cols(pen.n, np.random.default_rng(2))
    for k in (0, 4, 7):
        ref = spai.spai_update(pencil.shifted_operator(pen, shifts[k]),
                               pencil.shifted_operator(pen, drifted[k]), tol=0.01, cols=cols)
        info = upd[k].info()
        assert np.isclose(info.alpha, ref.alpha, rtol=1e-12)
        if info.skipped_cols == pen.n:
            assert ref.skipped[cols].all()


def test_c5_surrogate_full_size_sampled(ctx):
    """n = 1e7, heterogeneous EI, m = 4, 32 shifts (128 systems) mixed;
    every system must converge, and a sample of shifts is checked against
    the oracle's float64 reference solve (the surrogate is well conditioned:
    float64 and double-double references agree to 1e-13)."""
    pen, f, shifts, rng = beam.make_workload("c5", surrogate=True)
    set_pencil(ctx, pen)
    precs = [ctx.spai_build(s) for s in shifts]
    X, st = ctx.pcg_solve(list(shifts), precs, to_dev(f, torch.float64), tol=1e-10,
                          mode=airga.MODE_MIXED)
    assert all(e["status"] == airga.SYS_CONVERGED for e in st), [e for e in st if e["status"]]
    assert max(e["relres"] for e in st) <= 1e-10
    for k in (0, 13, 31):
        ref = direct.reference_solve(pen, shifts[k], f, "f64")
        Xk = X[k].cpu().numpy()
        for c in range(f.shape[0]):
            assert rel_err(Xk[c], ref[c]) < 1e-8, (k, c)


def test_moment_blocks_full_size(ctx):
    """The moment-sequence block operations at n = 1e6 in the sizes the
    benchmark times: the 16 blocks (m = 4) of one pass orthogonalised
    against 4 earlier blocks, the thin QR of the 64 collected columns and
    the projection onto them.  Checked against the oracle on the full
    vectors (numpy)."""
    from oracle import moments
    pen, f, shifts, rng = beam.make_workload("c3", surrogate=True)
    set_pencil(ctx, pen)
    n, m, nb, nx = pen.n, 4, 4, 16
    g = np.random.default_rng(21)
    q, _ = np.linalg.qr(g.standard_normal((n * m, nb)))
    vs = [q[:, t].reshape(n, m) for t in range(nb)]
    xs = [g.standard_normal((n, m)) for _ in range(nx)]
    x = to_dev(np.hstack(xs).T, torch.float64)
    gam, fro = ctx.global_orth(to_dev(np.hstack(vs).T, torch.float64), x, m, normalize=True)
    for i in (0, 7, 15):
        rx, rg, rf = moments.global_orth(vs, xs[i])
        assert np.all(np.abs(gam[i] - rg) <= 1e-12 * np.abs(rg).max())
        assert abs(fro[i] - rf) <= 1e-12 * rf
    w = x.clone()
    r = ctx.block_qr(w)
    wq = w.cpu().numpy().T
    assert np.abs(wq.T @ wq - np.eye(nx * m)).max() < 1e-12
    w0 = x.cpu().numpy().T
    assert rel_err(wq @ r, w0) < 1e-13
    mh, kh = ctx.project(w)
    ms = pencil.csr(n, pen.row_ptr, pen.col_idx, pen.m_val)
    ks = pencil.csr(n, pen.row_ptr, pen.col_idx, pen.k_val)
    rm, _, rk, _, _ = moments.project(ms, ks, pen.alpha, pen.beta, np.zeros((n, 1)),
                                      np.zeros((1, n)), wq)
    assert np.abs(mh - rm).max() < 1e-12 * np.abs(rm).max()
    assert np.abs(kh - rk).max() < 1e-12 * np.abs(rk).max()
    y = ctx.pencil_apply(1.0, 0.0, x[:m]).cpu().numpy().T
    assert rel_err(y, moments.pencil_apply(ms, ks, 1.0, 0.0, w0[:, :m])) < 1e-14
