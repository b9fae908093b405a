"""GPU: one iteration of AIRGA's outer loop (Algorithm 1) composed from the
library's entry points -- batched SPAI builds and PCG solves, the block
operations of the moment sequence, the projection, and the decisions of the
outer iteration (moment errors, H2 changes, poles and the next expansion
points) -- against the oracle's iteration with exact sparse solves, with
readings A1-A6 on both sides.  Then the vertical step the paper builds its
cheap update for (Algorithm 3): every preconditioner updated to the new
expansion points, and the solves there."""
import numpy as np
import pytest
import torch

from gpu_util import airga, beam, set_pencil, to_dev
from oracle import airga_loop, pencil

pytestmark = pytest.mark.gpu

ALPHA, BETA = 0.1, 0.02
SHIFTS = [1.0, 30.0, 500.0]
RMAX = 12


@pytest.fixture(scope="module")
def ctx():
    c = airga.Context(0)
    yield c
    c.close()


def system(n_el=60, m=2, seed=3):
    pen = beam.make_beam(n_el, ei_loguniform=(0.5, 2.0), surrogate=True, seed=seed,
                         alpha=ALPHA, beta=BETA)
    n = pen.n
    f, _ = beam.node_loads(n, m, np.random.default_rng(1))
    cp = np.zeros((1, n))
    cp[0, n - 2] = 1.0
    return pen, f, cp


def gpu_iteration(ctx, pen, f, cp, shifts, rmax, precs, tol_inner=1e-6):
    """Algorithm 1's inner part for one outer iteration, every step through
    the C ABI (the control flow mirrors the oracle's)."""
    n, m, l = pen.n, f.shape[0], len(shifts)
    fd = to_dev(f, torch.float64)
    cpd = to_dev(cp, torch.float64)
    X, st = ctx.pcg_solve(list(shifts), precs, fd, tol=1e-12)
    assert all(e["status"] == airga.SYS_CONVERGED for e in st)
    xs = X.reshape(l * m, n).contiguous()
    for i in range(l):
        b = xs[i * m:(i + 1) * m].clone()
        ctx.block_qr(b)
        xs[i * m:(i + 1) * m] = b

    def model_of(w):
        mh, kh = ctx.project(w)
        fh = ctx.gram(w, fd).cpu().numpy()
        cph = ctx.gram(w, cpd).cpu().numpy().T
        return (mh, kh, fh, cph, None)

    def next_block(q):
        v = xs[q * m:(q + 1) * m].clone()
        ctx.global_orth(None, v, m, normalize=True)
        return v

    vs, sigmas, step_errors, inner = [], [], [], []
    errors, prev = None, None
    j = 1
    while j < rmax // m:
        q = 0 if errors is None else int(np.argmax(errors))
        sigmas.append(q)
        vs.append(next_block(q))
        rhs = ctx.pencil_apply(1.0, 0.0, vs[-1])
        y, st = ctx.pcg_solve([shifts[q]], [precs[q]], rhs, tol=1e-12)
        assert all(e["status"] == airga.SYS_CONVERGED for e in st)
        xs[q * m:(q + 1) * m] = -y[0]
        _, before = ctx.global_orth(None, xs.clone(), m)
        _, after = ctx.global_orth(torch.cat(vs).contiguous(), xs, m)
        errors = after / before
        step_errors.append(errors)
        w = xs.clone()
        ctx.global_orth(None, w, m, normalize=True)
        ctx.block_qr(w)
        mi = model_of(w)
        if prev is not None:
            ch = airga.h2_distance(mi, prev, ALPHA, BETA) / airga.h2_distance(mi, None, ALPHA, BETA)
            inner.append(ch)
            if ch < tol_inner:
                j += 1
                break
        prev = mi
        j += 1
    q = 0 if errors is None else int(np.argmax(errors))
    sigmas.append(q)
    vs.append(next_block(q))
    v = torch.cat(vs).contiguous()
    ctx.block_qr(v)
    final = model_of(v)
    nxt = airga.next_shifts(airga.qep_poles(final[0], final[1], ALPHA, BETA), l)
    return dict(sigmas=sigmas, J=len(vs), step_errors=step_errors, inner=inner, model=final,
                next=nxt)


def oracle_iterations(pen, f, cp, count):
    n = pen.n
    ms = pencil.csr(n, pen.row_ptr, pen.col_idx, pen.m_val)
    ks = pencil.csr(n, pen.row_ptr, pen.col_idx, pen.k_val)
    _, _, hist = airga_loop.airga(ms, ks, pen.alpha, pen.beta, f.T, cp, None, SHIFTS, rmax=RMAX,
                                  max_outer=count)
    return ms, ks, hist


def test_outer_iteration_matches_the_oracle(ctx):
    pen, f, cp = system()
    set_pencil(ctx, pen)
    ms, ks, hist = oracle_iterations(pen, f, cp, 2)
    h0 = hist[0]
    # every argmax of the oracle's run is decided by a clear margin
    for e in h0["step_errors"]:
        top = np.sort(e)[::-1]
        assert top[0] - top[1] > 1e-4 * top[0]
    precs = ctx.spai_build_many(SHIFTS)
    g = gpu_iteration(ctx, pen, f, cp, SHIFTS, RMAX, precs)
    assert g["sigmas"] == h0["sigmas"] and g["J"] == h0["J"]
    for ge, oe in zip(g["step_errors"], h0["step_errors"]):
        assert np.allclose(ge, oe, rtol=1e-6, atol=0)
    assert np.allclose(g["inner"], h0["inner_changes"], rtol=1e-5, atol=1e-9)
    mh, kh, fh, cph, _ = g["model"]
    om = h0["model"]
    assert np.abs(mh - om.mh).max() <= 1e-8 * np.abs(om.mh).max()
    assert np.abs(kh - om.kh).max() <= 1e-8 * np.abs(om.kh).max()
    red = airga_loop.Model(mh, ALPHA * mh + BETA * kh, kh, fh, cph)
    # The GPU solves stop at a relative residual of 1e-12, so the moment
    # blocks carry errors up to cond(K(s)) * 1e-12 (a few 1e-6 here), which
    # the chain of moment solves and the projection carry into the reduced
    # transfer function; the oracle's solves are exact.
    mm, kk = beam.pencil_dense(pen)
    dd = ALPHA * mm + BETA * kk
    eps = 1e-12 * max(np.linalg.cond(s * s * mm + s * dd + kk) for s in SHIFTS)
    # (this beam's response is at rounding level, ~1e-40, beyond s ~ 10:
    # compared where it is not)
    for s in (0.01, 0.1, 1.0):
        got, want = red.transfer(s), om.transfer(s)
        err = np.abs(got - want).max() / np.abs(want).max()
        assert err <= 50 * eps, (s, err, eps)
    # both interpolate the full model at sigma_1, whose solve starts the basis
    s1 = SHIFTS[h0["sigmas"][0]]
    full = cp @ np.linalg.solve(s1 * s1 * mm + s1 * dd + kk, f.T)
    for h in (red.transfer(s1), om.transfer(s1)):
        assert np.abs(h - full).max() <= 50 * eps * np.abs(full).max()
    # the next expansion points (the oracle's second iteration starts there)
    assert np.allclose(g["next"], hist[1]["shifts"], rtol=1e-6, atol=0)


def test_next_iteration_solves_at_the_new_expansion_points(ctx):
    """The next outer iteration's solves, at the expansion points the first
    one chose, reach the dense reference.  (Updating the previous factors
    instead, Algorithm 3, assumes small changes of the points; across this
    first step they move by up to four decades and the updated chains need
    far more iterations, which is only printed here.)"""
    pen, f, cp = system()
    set_pencil(ctx, pen)
    precs = ctx.spai_build_many(SHIFTS)
    g = gpu_iteration(ctx, pen, f, cp, SHIFTS, RMAX, precs)
    new = [float(s) for s in g["next"]]
    assert all(0 < s < SHIFTS[0] for s in new)
    fresh = ctx.spai_build_many(new)
    fd = to_dev(f, torch.float64)
    X, st = ctx.pcg_solve(new, fresh, fd, tol=1e-10)
    assert all(e["status"] == airga.SYS_CONVERGED for e in st), st
    upd = ctx.spai_update_many(precs, new)
    _, stu = ctx.pcg_solve(new, upd, fd, tol=1e-10, max_iter=3000)
    print("expansion points", new)
    print("fresh builds: iterations", [e["iters"] for e in st])
    print("updated factors: (status, iterations)", [(e["status"], e["iters"]) for e in stu])
    mm, kk = beam.pencil_dense(pen)
    dd = ALPHA * mm + BETA * kk
    for k, s in enumerate(new):
        ref = np.linalg.solve(s * s * mm + s * dd + kk, f.T)
        for c in range(f.shape[0]):
            nr = np.linalg.norm(ref[:, c])
            assert np.linalg.norm(X[k, c].cpu().numpy() - ref[:, c]) <= 1e-7 * nr
