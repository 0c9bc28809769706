"""Pins of the oracle's primal-dual (Chambolle-Pock) ROF solver and of the
decomposition run with it, against what the mathematics fixes:

  - the exact solutions the Chambolle-solver pins use (half-plane step, the
    event-driven 1-D plateau flow), which any ROF solver must reach;
  - a weak-duality certificate: for the primal iterate x and the feasible
    dual field p = -y / lambda, P(x) - D(p) >= 0 bounds ||x - u*||_2 by
    sqrt(2 (P(x) - D(p))) (the ROF objective is 1-strongly convex), so the
    primal-dual and the dual fixed-point solutions of one problem must lie
    within the sum of their certified radii of each other;
  - exact invariances of the iteration (constant image, one-homogeneity with
    a factor of 2, transposition) and mean preservation;
  - the decomposition by either solver converging to the same bands.
  - the iteration's path at a finite count (the extrapolation theta = 1, the
    start xbar = x = g, returning x rather than xbar, the order of the dual
    and primal updates), by a worked example: the first iterates of Chambolle
    and Pock's Algorithm 1 on a two-level 2 x 2 image, derived by hand as
    exact fractions, once with the dual projection inactive and once with it
    saturated.  A mutation that only changes the path (theta = 0, another
    start, returning xbar) reaches the same fixed point and passes every
    other pin; it fails this one.
"""
import numpy as np
import pytest

from paper_2006_10004_amd import synth
from test_oracle_pins import plateau_flow


def primal(orc, g, lam, u):
    return 0.5 * np.sum((u - g) ** 2) + lam * orc.tv(u)


def dual(orc, g, lam, px, py):
    return 0.5 * np.sum(g ** 2) - 0.5 * np.sum((g - lam * orc.div(px, py)) ** 2)


def test_pdhg_half_plane_one_step(orc):
    a, b, c, dt = 4, 6, 1.0, 0.3
    f = synth.step_image(3, a, b, c).astype(np.float64)
    v, yx, yy = orc.rof_pdhg(f, dt, 2000)
    want = np.concatenate([np.full(a, c - dt / a), np.full(b, dt / b)])
    assert np.abs(v - want[None, :]).max() < 1e-12
    assert np.all(yy == 0.0)
    assert np.sqrt(yx ** 2 + yy ** 2).max() <= dt * (1 + 1e-12)  # |y| <= lambda


@pytest.mark.parametrize("tau,sigma", [(0.1, 1.2), (0.9, 0.13)])
def test_pdhg_unequal_steps_reach_the_same_solution(orc, tau, sigma):
    """Any steps with tau sigma ||grad||^2 <= 1 reach the ROF minimiser (the
    primal prox divides by 1 + tau, the dual step is sigma)."""
    a, b, c, dt = 5, 3, 0.75, 0.2  # c exact in float32
    f = synth.step_image(2, a, b, c).astype(np.float64)
    v, _, _ = orc.rof_pdhg(f, dt, 4000, tau=tau, sigma=sigma)
    want = np.concatenate([np.full(a, c - dt / a), np.full(b, dt / b)])
    assert np.abs(v - want[None, :]).max() < 1e-12


@pytest.mark.parametrize("t", [0.3, 0.9])
def test_pdhg_matches_exact_1d_flow(orc, t):
    levels = [0.2, 0.9, 0.4, 0.6, 0.1]
    lengths = [5, 3, 7, 4, 6]
    f = synth.plateau_image(3, levels, lengths).astype(np.float64)
    v, _, _ = orc.rof_pdhg(f, t, 3000)
    assert np.abs(v - plateau_flow(levels, lengths, t)[None, :]).max() < 1e-12


def test_pdhg_duality_certificate_and_agreement_with_chambolle(orc):
    g = synth.shapes_image(synth.ShapeSpec(24, 24, 1, 4, (0, 1), 3, 7, 0.5, 0.02, 0.2), 5)[0]
    g = g.astype(np.float64)
    lam = 0.05
    gaps = []
    for n in (100, 1000, 10000):
        x, yx, yy = orc.rof_pdhg(g, lam, n)
        px, py = -yx / lam, -yy / lam
        assert np.sqrt(px ** 2 + py ** 2).max() <= 1.0 + 1e-12
        gap = primal(orc, g, lam, x) - dual(orc, g, lam, px, py)
        assert gap >= -1e-12
        gaps.append(gap)
    assert gaps[0] > gaps[1] > gaps[2]
    assert gaps[2] < 1e-4
    # the dual fixed point's own certificate
    v, cx, cy = orc.rof(g, lam, 20000)
    gap_c = primal(orc, g, lam, v) - dual(orc, g, lam, cx, cy)
    assert gap_c >= -1e-12
    dist = np.sqrt(np.sum((x - v) ** 2))
    assert dist <= np.sqrt(2 * gaps[2]) + np.sqrt(2 * gap_c)
    assert np.abs(x - v).max() < 1e-3


def test_pdhg_constant_image_is_a_fixed_point(orc):
    g = np.full((7, 9), 0.37)
    v, yx, yy = orc.rof_pdhg(g, 0.2, 50)
    assert np.array_equal(v, g)
    assert np.all(yx == 0.0) and np.all(yy == 0.0)


def test_pdhg_one_homogeneity_exact(orc):
    g = synth.shapes_image(synth.ShapeSpec(20, 17, 1, 4, (0, 1), 2, 6, 0.5, 0.02, 0.3), 2)[0]
    g = g.astype(np.float64)
    v1, _, _ = orc.rof_pdhg(g, 0.07, 300)
    v2, _, _ = orc.rof_pdhg(2.0 * g, 0.14, 300)
    assert np.array_equal(v2, 2.0 * v1)


def test_pdhg_transpose_exact(orc):
    g = synth.shapes_image(synth.ShapeSpec(15, 22, 1, 4, (0, 1), 2, 6, 0.5, 0.02, 0.3), 4)[0]
    g = g.astype(np.float64)
    v, _, _ = orc.rof_pdhg(g, 0.05, 200)
    vt, _, _ = orc.rof_pdhg(np.ascontiguousarray(g.T), 0.05, 200)
    assert np.array_equal(vt, v.T)


def test_pdhg_preserves_the_mean(orc):
    g = synth.shapes_image(synth.ShapeSpec(18, 18, 1, 5, (0, 1), 2, 6, 0.5, 0.02, 0.3), 6)[0]
    g = g.astype(np.float64)
    v, _, _ = orc.rof_pdhg(g, 0.1, 500)
    assert abs(v.mean() - g.mean()) < 1e-14


def test_decompose_pdhg_against_chambolle_and_identities(orc):
    f = synth.shapes_image(synth.SMALL_64, 3)[0][::2, ::2].copy()  # 32 x 32
    kw = dict(dt=0.005, K=12, iters=4000, edges=[0, 1, 2, 4, 12])
    a = orc.decompose(f, solver="pdhg", **kw)
    b = orc.decompose(f, **kw)
    assert a["recon_err"] < 1e-12 and a["mean_err"] < 1e-12
    assert np.abs(a["bands"] - b["bands"]).max() < 2e-4
    assert np.abs(a["S"] - b["S"]).max() / np.abs(b["S"]).max() < 1e-2
    # one-homogeneity of the whole decomposition with the solver: 2f, 2dt
    f2 = (2.0 * f).astype(np.float32)
    c = orc.decompose(f2, dt=0.01, K=12, iters=300, edges=[0, 1, 2, 4, 12], solver="pdhg")
    d = orc.decompose(f, dt=0.005, K=12, iters=300, edges=[0, 1, 2, 4, 12], solver="pdhg")
    assert np.array_equal(c["bands"], 2.0 * d["bands"])


def test_decompose_pdhg_invalid_arguments(orc):
    f = np.zeros((8, 8), np.float32)
    with pytest.raises(KeyError):
        orc.decompose(f, 0.01, 3, 10, [0, 3], solver="admm")
    with pytest.raises(ValueError):
        orc.decompose(f, 0.01, 3, 10, [0, 3], solver="pdhg", sigma=-1.0)


# Worked example.  g has two identical rows (1, 0), so the vertical dual
# component stays 0 and the horizontal one lives at column 0 only (forward
# differences give 0 at the last column); with y = y[0, 0]:
#   grad xbar = xbar1 - xbar0,  div y = (y, -y),
#   y  <- y + sigma (xbar1 - xbar0), scaled back to |y| <= lambda,
#   x  <- (x + tau div y + tau g) / (1 + tau),   xbar <- 2 x_new - x_old,
# starting from x = xbar = g, y = 0.  With tau = sigma = 1/2:
#   lambda = 1 (projection never active):
#     y = -1/2, -2/3, -2/3, -11/18;  x0 = 5/6, 2/3, 5/9, 1/2
#   lambda = 3/10 (projection active from the first step, y = -3/10):
#     x0 = 9/10, 5/6, 71/90
# (x1 = 1 - x0 throughout, since the mean is preserved).
_WORKED = {
    1.0: [(-1 / 2, 5 / 6), (-2 / 3, 2 / 3), (-2 / 3, 5 / 9), (-11 / 18, 1 / 2)],
    0.3: [(-3 / 10, 9 / 10), (-3 / 10, 5 / 6), (-3 / 10, 71 / 90)],
}


@pytest.mark.parametrize("lam", sorted(_WORKED))
def test_pdhg_worked_example_first_iterates(orc, lam):
    g = np.array([[1.0, 0.0], [1.0, 0.0]])
    for n, (y, x0) in enumerate(_WORKED[lam], start=1):
        v, yx, yy = orc.rof_pdhg(g, lam, n, tau=0.5, sigma=0.5)
        np.testing.assert_allclose(v, [[x0, 1 - x0], [x0, 1 - x0]], rtol=0, atol=1e-15, err_msg="x after %d" % n)
        np.testing.assert_allclose(yx, [[y, 0.0], [y, 0.0]], rtol=0, atol=1e-15, err_msg="y after %d" % n)
        assert not yy.any()
