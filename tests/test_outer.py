"""The library's decisions of AIRGA's outer iteration (Algorithm 1: poles of
the reduced quadratic pencil, the next expansion points, the H2 distance of
Section 5) against the oracle.  These are host computations of the C ABI:
they run here without a GPU.  The library works in the modal form of the
reduced model; the oracle uses the companion linearisation and the Lyapunov
Gramian of the difference system, so the two share no method."""
import os

import numpy as np
import pytest

from oracle import airga_loop
from paper_1606_01216_amd import airga

pytestmark = pytest.mark.skipif(not os.path.exists(airga.LIB_PATH), reason="libairga.so not built")


def random_reduced(rng, r, m=2, p=2, alpha=0.05, beta=0.02, velocity=True, scale=1.0):
    g = rng.standard_normal((r, r))
    mh = g @ g.T + r * np.eye(r)
    g = rng.standard_normal((r, r))
    kh = scale * (g @ g.T + 0.5 * np.eye(r))
    fh = rng.standard_normal((r, m))
    cph = rng.standard_normal((p, r))
    cvh = rng.standard_normal((p, r)) if velocity else None
    return (mh, kh, fh, cph, cvh), airga_loop.Model(mh, alpha * mh + beta * kh, kh, fh, cph, cvh)



@pytest.mark.parametrize("r", [1, 2, 7, 24, 64])
@pytest.mark.parametrize("alpha,beta", [(0.05, 0.02), (0.0, 0.5), (3.0, 0.0), (0.2, 1.5)])
def test_qep_poles_match_the_oracle(r, alpha, beta):
    rng = np.random.default_rng(100 * r + int(10 * alpha))
    (mh, kh, *_), mod = random_reduced(rng, r, alpha=alpha, beta=beta)
    got = airga.qep_poles(mh, kh, alpha, beta)
    want = airga_loop.qep_poles(mod.mh, mod.dh, mod.kh)
    assert got.size == want.size == 2 * r
    # match each library pole to its nearest oracle pole, one to one
    scale = np.abs(want).max()
    left = list(want)
    for z in got:
        i = int(np.argmin([abs(z - w) for w in left]))
        assert abs(z - left[i]) <= 1e-9 * scale, (z, left[i])
        left.pop(i)
    # the documented order: ascending undamped frequency, (+im, -im) pairs
    w2 = np.abs(got[0::2] * got[1::2])
    assert np.all(np.diff(w2) >= -1e-12 * w2.max())
    pair = got[0::2].imag > 0
    assert np.allclose(got[1::2][pair], got[0::2][pair].conj())


def test_qep_poles_real_roots_keep_their_small_member():
    # an overdamped mode: d^2 >> 4 w2, where the textbook formula loses the
    # small root to cancellation
    mh, kh = np.array([[1.0]]), np.array([[1e-6]])
    p = airga.qep_poles(mh, kh, 1e3, 0.0)
    assert p.imag.tolist() == [0.0, 0.0]
    small = p.real[0]
    assert abs(small * small + 1e3 * small + 1e-6) <= 1e-18
    assert abs(p.real[0] * p.real[1] - 1e-6) <= 1e-18


@pytest.mark.parametrize("l", [1, 3, 6])
def test_next_shifts_match_the_oracle(l):
    rng = np.random.default_rng(l)
    (mh, kh, *_), mod = random_reduced(rng, 8, alpha=0.3, beta=0.9)
    poles = airga.qep_poles(mh, kh, 0.3, 0.9)
    got = airga.next_shifts(poles, l)
    want = airga_loop.next_shifts(airga_loop.qep_poles(mod.mh, mod.dh, mod.kh), l)
    assert np.allclose(got, want, rtol=1e-9, atol=0)
    assert np.all(np.diff(got) >= 0)


def test_next_shifts_hand_example_and_errors():
    poles = np.array([-1 + 10j, -1 - 10j, -0.5 + 2j, -0.5 - 2j, -3.0 + 0j, -40.0 + 0j])
    assert airga.next_shifts(poles, 3).tolist() == [0.5, 1.0, 3.0]
    with pytest.raises(airga.AirgaError) as ei:
        airga.next_shifts(poles, 5)
    assert ei.value.status == airga.EINVAL


@pytest.mark.parametrize("ra,rb", [(1, 1), (3, 2), (12, 7), (40, 40)])
@pytest.mark.parametrize("velocity", [False, True])
def test_h2_distance_matches_the_oracle(ra, rb, velocity):
    rng = np.random.default_rng(10 * ra + rb)
    ta, ma = random_reduced(rng, ra, velocity=velocity)
    tb, mb = random_reduced(rng, rb, velocity=velocity)
    got = airga.h2_distance(ta, tb, 0.05, 0.02)
    want = airga_loop.h2_distance(ma, mb)
    assert abs(got - want) <= 1e-9 * want
    na = airga.h2_distance(ta, None, 0.05, 0.02)
    assert abs(na - airga_loop.h2_distance(ma)) <= 1e-10 * na


def test_h2_distance_of_nearly_equal_models():
    # the distance is a difference of squared norms: resolved to ~1e-8 of the norm
    rng = np.random.default_rng(5)
    ta, ma = random_reduced(rng, 10)
    mh, kh, fh, cph, cvh = ta
    fh2 = fh * (1 + 1e-5)
    mb = airga_loop.Model(ma.mh, ma.dh, ma.kh, fh2, cph, cvh)
    got = airga.h2_distance(ta, (mh, kh, fh2, cph, cvh), 0.05, 0.02)
    norm = airga.h2_distance(ta, None, 0.05, 0.02)
    assert abs(got - 1e-5 * norm) <= 1e-8 * norm
    assert abs(got - airga_loop.h2_distance(ma, mb)) <= 1e-8 * norm
    assert airga.h2_distance(ta, ta, 0.05, 0.02) <= 1e-7 * norm


def test_h2_distance_one_dof_closed_form():
    m, d, k = 2.0, 0.6, 3.0
    # Dh = alpha Mh + beta Kh = d with beta = 0, alpha = d / m
    model = (np.array([[m]]), np.array([[k]]), np.array([[1.0]]), np.array([[1.0]]), None)
    val = airga.h2_distance(model, None, d / m, 0.0)
    assert abs(val ** 2 - 1 / (2 * d * k)) <= 1e-13 / (2 * d * k)


def test_outer_functions_reject_bad_input():
    eye = np.eye(3)
    with pytest.raises(airga.AirgaError) as ei:
        airga.qep_poles(-eye, eye, 0.1, 0.1)
    assert ei.value.status == airga.ENOTSPD
    with pytest.raises(airga.AirgaError) as ei:
        airga.qep_poles(eye, eye, float("nan"), 0.1)
    assert ei.value.status == airga.EINVAL
    model = (eye, eye, np.ones((3, 1)), np.ones((1, 3)), None)
    # no damping: the H2 norm is infinite
    with pytest.raises(airga.AirgaError) as ei:
        airga.h2_distance(model, None, 0.0, 0.0)
    assert ei.value.status == airga.EINVAL
    other = (eye, eye, np.ones((3, 2)), np.ones((1, 3)), None)
    with pytest.raises(airga.AirgaError) as ei:
        airga.h2_distance(model, other, 0.1, 0.1)
    assert ei.value.status == airga.EINVAL
    # non-finite entries anywhere are rejected, not carried into the result
    bad = eye.copy()
    bad[0, 1] = bad[1, 0] = np.nan
    for mh, kh in ((bad, eye), (eye, bad)):
        with pytest.raises(airga.AirgaError) as ei:
            airga.qep_poles(mh, kh, 0.1, 0.1)
        assert ei.value.status == airga.EINVAL
    for m_ in ((bad, eye, np.ones((3, 1)), np.ones((1, 3)), None),
               (eye, eye, np.full((3, 1), np.inf), np.ones((1, 3)), None),
               (eye, eye, np.ones((3, 1)), np.ones((1, 3)), np.full((1, 3), np.nan))):
        with pytest.raises(airga.AirgaError) as ei:
            airga.h2_distance(m_, None, 0.1, 0.1)
        assert ei.value.status == airga.EINVAL
    with pytest.raises(airga.AirgaError) as ei:
        airga.h2_distance(model, None, float("nan"), 0.1)
    assert ei.value.status == airga.EINVAL
    with pytest.raises(airga.AirgaError) as ei:
        airga.next_shifts(np.array([1.0, np.nan]) + 0j, 1)
    assert ei.value.status == airga.EINVAL


def test_bench_times_the_decisions():
    # bench.py's host-side measurement runs without a GPU and reports each call
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import bench
    out = bench.measure_outer(r=8, m=2, p=1, l=3, reps=2)
    assert out["r"] == 8 and out["l"] == 3
    assert all(out[k] >= 0 for k in ("qep_poles_ms", "next_shifts_ms", "h2_distance_ms"))
