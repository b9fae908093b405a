"""GPU: the LDS-staged kernels for banded pencils (bandwidth <= 64) against the
general sliced-ELL kernels and the oracle.  The staged PCG kernels compute
the same arithmetic in the same order, so solves must agree bit for bit; so
must SPAI factors, except for narrow bands, whose staged kernel folds the
least-squares rows in another order.  Every tile configuration must also
meet the oracle tolerance."""
import numpy as np
import pytest
import torch

from gpu_util import airga, beam, grid_pencil, pencil, reference, rel_err, set_pencil, spai, to_dev

pytestmark = pytest.mark.gpu

SOLVE_TOL = 1e-8
TILES = [(64, 1), (64, 2), (64, 4), (128, 1), (128, 2), (128, 4), (256, 1)]


@pytest.fixture(scope="module")
def ctx():
    c = airga.Context(0)
    yield c
    c.close()


def pencils():
    # beam: bandwidth 3, rows of 4..6 (uniform slice width); chain: a 1-D
    # chain (tridiagonal, bandwidth 1, rows of 2..3 consecutive columns: the
    # normal-equation builds with rows shorter than 6 everywhere); grids:
    # 5-point, bandwidth nx (64 = the largest staged; 65 = general kernels only)
    return {"beam": beam.make_beam(1037, ei_loguniform=(0.5, 2.0), surrogate=True, seed=5),
            "chain": grid_pencil(1000, 1, seed=4),
            "grid64": grid_pencil(64, 23, seed=1), "grid65": grid_pencil(65, 9, seed=2)}


def _same(a, b, exact, tol=1e-13):
    """Bit-equal when the staged kernel folds rows in the general kernel's
    order; otherwise (narrow bands fold the row span in ascending order)
    equal up to rounding."""
    if exact:
        return np.array_equal(a, b)
    return np.all(np.abs(a - b) <= tol * max(np.abs(b).max(), 1e-300))


# Equilibrated builds on the beam solve each column from its normal equations
# (Gram matrices taken from Khat^2) where the general kernels rotate row by row:
# the two agree to cond(Khat(I, J))^2 eps, with cond below 60 on this beam
# after equilibration (about 8e-13).
GRAM_TOL = 1e-11


def _same_objective(a, b, tol):
    """The normal-equation builds take each column's objective from the
    quadratic form 1 - 2 g^T p + p^T G p, whose value (the squared residual)
    is accurate to a few units of the rounding of 1, absolutely: small
    objectives (the chain's, 1e-4..1e-2) agree in their squares, others to
    tol relative to the largest."""
    close = np.abs(a - b) <= tol * max(np.abs(b).max(), 1e-300)
    return np.all(close | (np.abs(a * a - b * b) <= 1e-13))


@pytest.mark.parametrize("name", ["beam", "chain", "grid64", "grid65"])
def test_spai_staged_equals_general(ctx, name):
    pen = pencils()[name]
    set_pencil(ctx, pen)
    narrow = name in ("beam", "chain")
    exact = not narrow  # narrow bands take the row-span order
    for s, eq, sym in ((3.0, True, True), (40.0, True, False), (7.0, False, False)):
        a = ctx.spai_build(s, equilibrate=eq, symmetrize=sym)
        g = ctx.spai_build(s, equilibrate=eq, symmetrize=sym, general_only=True)
        va, oa = (t.cpu().numpy() for t in a.export())
        vg, og = (t.cpu().numpy() for t in g.export())
        btol = GRAM_TOL if (narrow and eq) else 1e-13
        same_obj = _same_objective(oa, og, btol) if (narrow and eq) else _same(oa, og, exact, btol)
        assert _same(va, vg, exact, btol) and same_obj, (name, s)
        # updates from the same old factor: some columns skipped, some solved
        for s_new, tol in ((s * 1.001, 0.01), (s * 1.3, 0.01), (s * 1.05, 0.0)):
            qa = ctx.spai_update(a, s_new, tol=tol)
            qg = ctx.spai_update(a, s_new, tol=tol, general_only=True)
            wa, pa = (t.cpu().numpy() for t in qa.export())
            wg, pg = (t.cpu().numpy() for t in qg.export())
            assert _same(wa, wg, exact) and _same(pa, pg, exact), (name, s, s_new)
            assert qa.info().skipped_cols == qg.info().skipped_cols


def test_spai_staged_at_bandwidth_64_matches_oracle(ctx):
    pen = pencils()["grid64"]
    set_pencil(ctx, pen)
    assert ctx.pencil_info().bandwidth == 64
    a = pencil.shifted_operator(pen, 2.0)
    ref = spai.spai_build(a)
    vals, obj = (t.cpu().numpy() for t in ctx.spai_build(2.0).export())
    assert np.all(np.abs(obj - ref.objective) <= 1e-12 * np.maximum(1.0, ref.objective))
    assert np.all(np.abs(vals - ref.values) <= 1e-10 * np.abs(ref.values).max())
    ref_u = spai.spai_update(a, pencil.shifted_operator(pen, 2.6), tol=0.0)
    q = ctx.spai_update(ctx.spai_build(2.0), 2.6, tol=0.0)
    vq, oq = (t.cpu().numpy() for t in q.export())
    assert np.all(np.abs(vq - ref_u.values) <= 1e-10 * np.abs(ref_u.values).max())


@pytest.mark.parametrize("name", ["beam", "grid64"])
@pytest.mark.parametrize("mode", [airga.MODE_FP64, airga.MODE_MIXED])
def test_solves_staged_equal_general(ctx, name, mode):
    pen = pencils()[name]
    set_pencil(ctx, pen)
    rng = np.random.default_rng(3)
    f = rng.standard_normal((2, pen.n))
    F = to_dev(f, torch.float64)
    shifts = [1.5, 30.0, 400.0]
    precs = [ctx.spai_build(s) for s in shifts]
    # update chains too (a second real factor: the direction kernel then
    # stores w in full for the chain kernel)
    upd = [ctx.spai_update(p, s * 1.1, tol=0.0) for p, s in zip(precs, shifts)]
    for pr, sh in ((precs, shifts), (upd, [s * 1.1 for s in shifts])):
        for tile in TILES[:1] + TILES[4:5] + TILES[6:]:
            Xa, sa = ctx.pcg_solve(sh, pr, F, mode=mode, tile=tile)
            Xg, sg = ctx.pcg_solve(sh, pr, F, mode=mode, tile=tile, general_only=True)
            assert torch.equal(Xa, Xg), (name, tile)
            assert sa == sg


@pytest.mark.parametrize("tile", TILES)
def test_every_tile_meets_the_oracle(ctx, tile):
    pen = beam.make_beam(800, ei_loguniform=(0.5, 2.0), surrogate=True, seed=9)
    set_pencil(ctx, pen)
    f = np.stack([beam.tip_load(pen.n)[0], np.random.default_rng(4).standard_normal(pen.n)])
    shifts = [2.0, 90.0]
    ref = reference(pen, shifts, f)
    F = to_dev(f, torch.float64)
    precs = [ctx.spai_build(s) for s in shifts]
    upd = [ctx.spai_update(p, s * 1.2, tol=0.0) for p, s in zip(precs, shifts)]
    ref_u = reference(pen, [s * 1.2 for s in shifts], f)
    for mode in (airga.MODE_FP64, airga.MODE_MIXED):
        X, st = ctx.pcg_solve(shifts, precs, F, mode=mode, tile=tile)
        Xh = X.cpu().numpy()
        for k in range(2):
            for c in range(2):
                assert st[k * 2 + c]["status"] == airga.SYS_CONVERGED
                assert rel_err(Xh[k, c], ref[k, c]) < SOLVE_TOL, (tile, mode, k, c)
        # update chains (a second factor per shift) through the chain kernel
        X, st = ctx.pcg_solve([s * 1.2 for s in shifts], upd, F, mode=mode, tile=tile)
        Xh = X.cpu().numpy()
        for k in range(2):
            for c in range(2):
                assert rel_err(Xh[k, c], ref_u[k, c]) < SOLVE_TOL, (tile, mode, k, c)
    assert ctx.tile_config() == tile


def test_forced_tile_rejects_unknown_configuration(ctx):
    pen = beam.make_beam(50, surrogate=True)
    set_pencil(ctx, pen)
    F = to_dev(beam.tip_load(pen.n), torch.float64)
    with pytest.raises(airga.AirgaError) as ei:
        ctx.pcg_solve([1.0], None, F, tile=(192, 1))
    assert ei.value.status == airga.EINVAL


@pytest.mark.parametrize("name", ["beam", "grid8", "grid65"])
def test_batched_updates_equal_single_updates(ctx, name):
    """airga_spai_update_many gives exactly the single updates: factor values,
    objectives, alpha and skip counts, for skipped and solved columns, over
    more than one batch of 16 (and through the one-by-one fallback where the
    staged rows do not fit, or with general_only), with and without the
    diagonal equilibration."""
    pen = {"beam": beam.make_beam(1037, ei_loguniform=(0.5, 2.0), surrogate=True, seed=5),
           "grid8": grid_pencil(8, 150, seed=3), "grid65": grid_pencil(65, 9, seed=2)}[name]
    set_pencil(ctx, pen)
    base = [1.0 * 1.6 ** k for k in range(18)]
    olds = [ctx.spai_build(s) for s in base]
    # drifts from none (all columns skip) to large (columns solved)
    new = [s * (1.0 + (0.0 if k % 3 == 0 else 1e-4 if k % 3 == 1 else 0.2)) for k, s in enumerate(base)]
    for tol, general, eq in ((0.01, False, True), (0.0, False, True), (0.01, True, True),
                             (0.01, False, False)):
        many = ctx.spai_update_many(olds, new, tol=tol, general_only=general, equilibrate=eq)
        for k, (p, s) in enumerate(zip(olds, new)):
            one = ctx.spai_update(p, s, tol=tol, general_only=general, equilibrate=eq)
            vm, om = (t.cpu().numpy() for t in many[k].export())
            vo, oo = (t.cpu().numpy() for t in one.export())
            im, io = many[k].info(), one.info()
            assert np.array_equal(vm, vo) and np.array_equal(om, oo), (name, k, tol)
            assert im.alpha == io.alpha and im.skipped_cols == io.skipped_cols, (name, k)
            assert im.scalar_only == io.scalar_only and im.chain_len == io.chain_len
    assert ctx.spai_update_many([], []) == []


@pytest.mark.parametrize("name", ["beam", "chain", "grid8", "grid65"])
def test_batched_builds_equal_single_builds(ctx, name):
    """airga_spai_build_many gives exactly the single builds (values,
    objectives, alpha) over more than one batch of 16, with and without
    equilibration and symmetrisation; grid65 (bandwidth 65) and general_only
    take the one-by-one path."""
    pen = {"beam": beam.make_beam(1037, ei_loguniform=(0.5, 2.0), surrogate=True, seed=5),
           "chain": grid_pencil(1000, 1, seed=4),
           "grid8": grid_pencil(8, 150, seed=3), "grid65": grid_pencil(65, 9, seed=2)}[name]
    set_pencil(ctx, pen)
    shifts = [0.7 * 1.7 ** k for k in range(18)]
    for eq, sym, general in ((True, True, False), (False, False, False), (True, True, True)):
        many = ctx.spai_build_many(shifts, equilibrate=eq, symmetrize=sym, general_only=general)
        for k, s in enumerate(shifts):
            one = ctx.spai_build(s, equilibrate=eq, symmetrize=sym, general_only=general)
            vm, om = (t.cpu().numpy() for t in many[k].export())
            vo, oo = (t.cpu().numpy() for t in one.export())
            assert np.array_equal(vm, vo) and np.array_equal(om, oo), (name, k, eq, sym)
            assert many[k].info().alpha == one.info().alpha
    assert ctx.spai_build_many([]) == []
