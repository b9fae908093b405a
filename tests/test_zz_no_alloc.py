"""GPU: airga_gram_noalloc, the allocation-free A^T B, against airga_gram on
the same inputs.  Two calls in a row, the second smaller, so a result cannot
lean on what an earlier call left in the shared partial-sum array.  Where the
no-allocation entry point sums exactly as airga_gram does (k, l <= 64 and at
most 1024 row blocks per tile) the bits must agree; where its fixed array
makes each block cover more rows the results agree to rounding."""
import numpy as np
import pytest
import torch

from gpu_util import airga, beam, set_pencil, to_dev

pytestmark = pytest.mark.gpu


def _pair(ctx, n, k, l, seed):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n, k))
    b = rng.standard_normal((n, l))
    ad, bd = to_dev(a.T, torch.float64), to_dev(b.T, torch.float64)
    ref = ctx.gram(ad, bd).cpu().numpy()
    out = torch.full((l, k), float("nan"), dtype=torch.float64, device=ad.device)
    got = ctx.gram_noalloc(ad, bd, out).cpu().numpy()
    scale = np.outer(np.linalg.norm(a, axis=0), np.linalg.norm(b, axis=0))
    return got, ref, a.T @ b, scale


def test_noalloc_gram_matches_gram_on_two_calls():
    ctx = airga.Context(0)
    try:
        # n = 200,000 rows, a 130 x 70 product: 6 output tiles, so the fixed
        # array holds 170 row blocks per tile against the 196 airga_gram uses
        pen = beam.make_beam(100_000, ei_loguniform=(0.5, 2.0), surrogate=True, seed=5)
        set_pencil(ctx, pen)
        got, ref, exact, scale = _pair(ctx, pen.n, 130, 70, 1)
        assert got.shape == (130, 70)
        assert np.all(np.isfinite(got))
        assert np.all(np.abs(got - ref) <= 1e-13 * scale)
        assert np.all(np.abs(got - exact) <= 1e-13 * scale)
        # second call, smaller: 5 x 3 on the same pencil, summed as airga_gram sums
        got, ref, exact, scale = _pair(ctx, pen.n, 5, 3, 2)
        assert np.array_equal(got, ref)
        assert np.all(np.abs(got - exact) <= 1e-13 * scale)
        # a smaller pencil, a full 64 x 64 tile, then a 1 x 1 product
        pen2 = beam.make_beam(518, ei_loguniform=(0.5, 2.0), surrogate=True, seed=6)
        set_pencil(ctx, pen2)
        for k, l, seed in ((64, 64, 3), (1, 1, 4)):
            got, ref, exact, scale = _pair(ctx, pen2.n, k, l, seed)
            assert np.array_equal(got, ref), (k, l)
            assert np.all(np.abs(got - exact) <= 1e-13 * scale), (k, l)
    finally:
        ctx.close()


def test_noalloc_gram_shares_the_array_across_contexts_and_checks_sizes():
    pen = beam.make_beam(700, ei_loguniform=(0.5, 2.0), surrogate=True, seed=7)
    c1, c2 = airga.Context(0), airga.Context(0)
    try:
        set_pencil(c1, pen)
        set_pencil(c2, pen)
        g1, r1, _, _ = _pair(c1, pen.n, 40, 9, 8)
        torch.cuda.synchronize()
        g2, r2, _, _ = _pair(c2, pen.n, 9, 40, 9)
        assert np.array_equal(g1, r1) and np.array_equal(g2, r2)
        a = torch.zeros((257, pen.n), dtype=torch.float64, device="cuda:0")
        out = torch.zeros((1, 257), dtype=torch.float64, device="cuda:0")
        with pytest.raises(airga.AirgaError) as e:
            c1.gram_noalloc(a, a[:1], out)
        assert e.value.status == airga.EUNSUPPORTED
    finally:
        c1.close()
        c2.close()
