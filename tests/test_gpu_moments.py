"""GPU: the block operations of the moment sequence (Algorithm 1's steps
around the shifted solves) against the oracle: right-hand sides (a M + b K) X,
products A^T B over the rows, orthogonalisation in the trace inner product,
thin QR and Galerkin projection; then one pass of the moment sequence built
from them, pinned by interpolation of the full transfer function."""
import numpy as np
import pytest
import torch

from gpu_util import airga, beam, csr_of, rel_err, set_pencil, to_dev
from oracle import moments

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = airga.Context(0)
    yield c
    c.close()


def sur_beam(n_el, seed=3):
    return beam.make_beam(n_el, ei_loguniform=(0.5, 2.0), surrogate=True, seed=seed)


def rows_to_cols(t):
    """(k, n) device block -> n x k numpy array."""
    return t.cpu().numpy().T


@pytest.mark.parametrize("n_el", [37, 1200])
def test_pencil_apply_matches_oracle(ctx, n_el):
    pen = sur_beam(n_el)
    set_pencil(ctx, pen)
    ms, ks = csr_of(pen, pen.m_val), csr_of(pen, pen.k_val)
    x = np.random.default_rng(1).standard_normal((pen.n, 3))
    s = 40.0
    for a, b in ((1.0, 0.0), (0.0, 1.0), (-(2 * s + pen.alpha), -pen.beta), (s * s, 1.0 + s)):
        y = rows_to_cols(ctx.pencil_apply(a, b, to_dev(x.T, torch.float64)))
        ref = moments.pencil_apply(ms, ks, a, b, x)
        assert rel_err(y, ref) < 1e-14, (a, b)


@pytest.mark.parametrize("n", [74, 1037, 5000])
@pytest.mark.parametrize("k,l", [(1, 1), (5, 3), (64, 64), (70, 130)])
def test_gram_matches_oracle(ctx, n, k, l):
    pen = sur_beam(n // 2)
    set_pencil(ctx, pen)
    n = pen.n
    rng = np.random.default_rng(k * 1000 + l)
    a = rng.standard_normal((n, k))
    b = rng.standard_normal((n, l))
    g = ctx.gram(to_dev(a.T, torch.float64), to_dev(b.T, torch.float64)).cpu().numpy()
    ref = a.T @ b
    scale = np.outer(np.linalg.norm(a, axis=0), np.linalg.norm(b, axis=0))
    assert g.shape == (k, l)
    assert np.all(np.abs(g - ref) <= 1e-13 * scale)
    # repeated calls give identical bits (fixed-order sums)
    g2 = ctx.gram(to_dev(a.T, torch.float64), to_dev(b.T, torch.float64)).cpu().numpy()
    assert np.array_equal(g, g2)


def orthonormal_blocks(rng, n, m, j):
    q, _ = np.linalg.qr(rng.standard_normal((n * m, j)))
    return [q[:, t].reshape(n, m) for t in range(j)]


@pytest.mark.parametrize("nb,nx", [(0, 1), (1, 1), (3, 5), (16, 16)])
@pytest.mark.parametrize("orthonormal", [True, False])
def test_global_orth_matches_oracle(ctx, nb, nx, orthonormal):
    pen = sur_beam(500)
    set_pencil(ctx, pen)
    n, m = pen.n, 4
    rng = np.random.default_rng(10 * nb + nx)
    if orthonormal:
        vs = orthonormal_blocks(rng, n, m, nb)
    else:
        # a general basis: the loop order then matters
        vs = [rng.standard_normal((n, m)) * (1.0 + t) for t in range(nb)]
    xs = [rng.standard_normal((n, m)) for _ in range(nx)]
    v = to_dev(np.hstack(vs).T, torch.float64) if nb else None
    for normalize in (False, True):
        x = to_dev(np.hstack(xs).T, torch.float64)
        gam, fro = ctx.global_orth(v, x, m, normalize=normalize)
        xo = rows_to_cols(x)
        for i in range(nx):
            rx, rg, rf = moments.global_orth(vs, xs[i])
            gs = np.abs(rg).max() if nb else 1.0
            assert np.all(np.abs(gam[i] - rg) <= 1e-12 * max(gs, 1.0)), (i, gam[i], rg)
            assert abs(fro[i] - rf) <= 1e-12 * max(rf, np.linalg.norm(xs[i]))
            got = xo[:, i * m:(i + 1) * m]
            want = rx / rf if normalize else rx
            assert rel_err(got, want) < 1e-11 * max(1.0, np.linalg.norm(xs[i]) / rf), (i, normalize)


def test_global_orth_zero_block_stays_zero(ctx):
    pen = sur_beam(100)
    set_pencil(ctx, pen)
    x = torch.zeros((4, pen.n), dtype=torch.float64, device="cuda")
    gam, fro = ctx.global_orth(None, x, 4, normalize=True)
    assert fro[0] == 0.0 and not torch.any(x)


@pytest.mark.parametrize("k", [1, 7, 33, 64])
def test_block_qr_matches_oracle(ctx, k):
    pen = sur_beam(700)
    set_pencil(ctx, pen)
    w = np.random.default_rng(k).standard_normal((pen.n, k))
    t = to_dev(w.T, torch.float64)
    r = ctx.block_qr(t)
    q = rows_to_cols(t)
    rq, rr = moments.thin_qr(w)
    assert np.allclose(np.tril(r, -1), 0.0) and np.all(np.diag(r) > 0)
    assert np.abs(q.T @ q - np.eye(k)).max() < 1e-13
    assert rel_err(q @ r, w) < 1e-14
    assert np.abs(q - rq).max() < 1e-12 and np.abs(r - rr).max() < 1e-12 * np.abs(rr).max()


def test_block_qr_ill_conditioned_and_dependent(ctx):
    pen = sur_beam(700)
    set_pencil(ctx, pen)
    rng = np.random.default_rng(3)
    k = 24
    # condition number 1e10: orthonormal columns scaled over ten decades, mixed
    u, _ = np.linalg.qr(rng.standard_normal((pen.n, k)))
    vq, _ = np.linalg.qr(rng.standard_normal((k, k)))
    w = (u * np.logspace(0, -10, k)) @ vq.T
    t = to_dev(w.T, torch.float64)
    r = ctx.block_qr(t)
    q = rows_to_cols(t)
    assert np.abs(q.T @ q - np.eye(k)).max() < 1e-12
    assert rel_err(q @ r, w) < 1e-13
    # same span as the oracle's Q (columns agree up to the conditioning)
    rq, _ = moments.thin_qr(w)
    assert np.abs(q[:, :8] - rq[:, :8]).max() < 1e-9
    # a zero column: no Q exists with a positive R diagonal
    w[:, 5] = 0.0
    with pytest.raises(airga.AirgaError) as ei:
        ctx.block_qr(to_dev(w.T, torch.float64))
    assert ei.value.status == airga.ENOTSPD


@pytest.mark.parametrize("k", [1, 10, 64])
def test_project_matches_oracle(ctx, k):
    pen = sur_beam(900)
    set_pencil(ctx, pen)
    q, _ = moments.thin_qr(np.random.default_rng(k).standard_normal((pen.n, k)))
    mh, kh = ctx.project(to_dev(q.T, torch.float64))
    ms, ks = csr_of(pen, pen.m_val), csr_of(pen, pen.k_val)
    rm, _, rk, _, _ = moments.project(ms, ks, pen.alpha, pen.beta, np.zeros((pen.n, 1)),
                                      np.zeros((1, pen.n)), q)
    assert np.abs(mh - rm).max() < 1e-13 * np.abs(rm).max()
    assert np.abs(kh - rk).max() < 1e-13 * np.abs(rk).max()


def test_block_ops_reject_bad_sizes(ctx):
    pen = sur_beam(50)
    set_pencil(ctx, pen)
    x = torch.zeros((65, pen.n), dtype=torch.float64, device="cuda")
    with pytest.raises(airga.AirgaError) as ei:
        ctx.block_qr(x)
    assert ei.value.status == airga.EUNSUPPORTED
    with pytest.raises(airga.AirgaError) as ei:
        ctx.global_orth(torch.zeros((68, pen.n), dtype=torch.float64, device="cuda"),
                        torch.zeros((4, pen.n), dtype=torch.float64, device="cuda"), 4)
    assert ei.value.status == airga.EUNSUPPORTED
    with pytest.raises(airga.AirgaError) as ei:
        ctx.gram(torch.zeros((257, pen.n), dtype=torch.float64, device="cuda"), x)
    assert ei.value.status == airga.EUNSUPPORTED


def test_moment_sequence_pass_interpolates(ctx):
    """One pass of Algorithm 1 on the GPU (m = 2 inputs, three expansion
    points): solves X(s_i) = K(s_i)^{-1} F, the thin QR of each block (the
    algorithm's first step after the solves),
    V_1 = X(sigma) / ||X(sigma)||_F, the moment solve with right-hand side
    M V_1, orthogonalisation of every block against V_1 in the trace inner
    product, the thin QR of the collected blocks together with V_1, and the
    projection.  The range of the basis then holds X(s_i) for every i, so the
    reduced transfer function equals the full one at the expansion points
    (Section 2); the full one comes from dense solves on the CPU."""
    pen = sur_beam(95, seed=4)
    set_pencil(ctx, pen)
    n, m = pen.n, 2
    mm, kk = beam.pencil_dense(pen)
    dd = pen.alpha * mm + pen.beta * kk
    rng = np.random.default_rng(7)
    f, _ = beam.node_loads(n, m, rng)            # (m, n)
    cp = rng.standard_normal((3, n))
    shifts = [2.0, 30.0, 500.0]
    precs = [ctx.spai_build(s) for s in shifts]
    X, st = ctx.pcg_solve(shifts, precs, to_dev(f, torch.float64), tol=1e-12)
    assert all(e["status"] == airga.SYS_CONVERGED for e in st)
    blocks = X.reshape(len(shifts) * m, n).contiguous()      # rows: (shift, column)
    # X(s_i) <- Q of its thin QR, block by block
    for i in range(len(shifts)):
        b = blocks[i * m:(i + 1) * m].clone()
        ctx.block_qr(b)
        blocks[i * m:(i + 1) * m] = b
    sig = 1                                                 # sigma = shifts[1]
    v1 = blocks[sig * m:(sig + 1) * m].clone()
    ctx.global_orth(None, v1, m, normalize=True)
    rhs = ctx.pencil_apply(1.0, 0.0, v1)
    Xm, stm = ctx.pcg_solve([shifts[sig]], [precs[sig]], rhs, tol=1e-12)
    assert all(e["status"] == airga.SYS_CONVERGED for e in stm)
    blocks[sig * m:(sig + 1) * m] = -Xm[0]
    gam, fro = ctx.global_orth(v1, blocks, m, normalize=True)
    assert np.all(fro > 0)
    w = torch.cat([v1, blocks]).contiguous()
    r = ctx.block_qr(w)
    assert np.all(np.diag(r) > 0)
    mh, kh = ctx.project(w)
    wn = w.cpu().numpy().T
    assert np.abs(wn.T @ wn - np.eye(wn.shape[1])).max() < 1e-12
    dh = pen.alpha * mh + pen.beta * kh
    fh, ch = wn.T @ f.T, cp @ wn
    for s in shifts:
        full = cp @ np.linalg.solve(s * s * mm + s * dd + kk, f.T)
        red = moments.reduced_transfer(mh, dh, kh, fh, ch, s)
        assert np.allclose(red, full, rtol=1e-8, atol=1e-12 * np.abs(full).max()), s
