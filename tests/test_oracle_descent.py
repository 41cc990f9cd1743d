"""Pins for the gradient, exact line search and Algorithm 1 loop
(THEORY section: gradient, ELS and hard data matching paragraphs;
Algorithm 1)."""
import numpy as np
import pytest

import oracle
import synth


@pytest.fixture(scope="module")
def gc_problem():
    P = synth.make_problem("gradcheck_48x48x4")
    lo, hi, _ = P["schedule"][0]
    Q, _, _ = oracle.nullspace(oracle.gram(P["x0"], P["kdims"], lo, hi), P["rank"])
    return P, lo, hi, Q


def _rand_dir(shape, mask, rng):
    d = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    d[mask.astype(bool)] = 0.0
    return d


def test_gradient_matches_central_differences(gc_problem):
    """J is quadratic in x for fixed F, so the central difference
    (J(x + h d) - J(x - h d)) / 2h equals Re<g, d> up to rounding only
    (g = 2 dJ/d conj(x)); 200 random directions with d = 0 at observed
    locations, h = 1e-3."""
    P, lo, hi, Q = gc_problem
    x, kd, mask = P["x0"], P["kdims"], P["mask"]
    _, g, _ = oracle.objective_grad(x, mask, Q, kd, lo, hi)
    rng = np.random.default_rng(11)
    h = 1e-3
    worst = 0.0
    for _ in range(200):
        d = _rand_dir(x.shape, mask, rng)
        fd = (oracle.objective(x + h * d, Q, kd, lo, hi) - oracle.objective(x - h * d, Q, kd, lo, hi)) / (2 * h)
        an = float(np.vdot(g, d).real)
        worst = max(worst, abs(fd - an) / max(abs(an), 1e-300))
    assert worst < 1e-6


def test_gradient_zero_at_observed_and_outside_region():
    P = synth.make_problem("2d_64x64x4")
    x, kd, mask = P["x0"], P["kdims"], P["mask"]
    lo, hi = (0, 20, 18), (1, 44, 40)
    Q, _, _ = oracle.nullspace(oracle.gram(x, kd, lo, hi), P["rank"])
    _, g, _ = oracle.objective_grad(x, mask, Q, kd, lo, hi)
    assert np.all(g[mask.astype(bool)] == 0)
    inside = np.zeros(mask.shape, bool)
    inside[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] = True
    assert np.all(g[~inside] == 0)
    assert np.abs(g[inside & ~mask.astype(bool)]).max() > 0


def test_exact_line_search_is_parabola_vertex(gc_problem):
    """J(y - t g) is a parabola in t; its vertex from three evaluations equals
    the closed form, the decrease is ||g||^4 / (4 ||Z||^2), the new gradient
    is orthogonal to the old one, and eta = Re<Y, Z> / ||Z||^2."""
    P, lo, hi, Q = gc_problem
    x, kd, mask = P["x0"], P["kdims"], P["mask"]
    J, g, gn2 = oracle.objective_grad(x, mask, Q, kd, lo, hi)
    eta = oracle.line_search(g, Q, gn2, kd, lo, hi)
    f = lambda t: oracle.objective(x - t * g, Q, kd, lo, hi)
    t1 = 2.0 * eta
    f0, f1, f2 = f(0.0), f(t1 / 2), f(t1)
    # vertex of the parabola through (0, f0), (t1/2, f1), (t1, f2)
    a = (f2 - 2 * f1 + f0) / (2 * (t1 / 2) ** 2)
    b = (f1 - f0) / (t1 / 2) - a * (t1 / 2)
    assert -b / (2 * a) == pytest.approx(eta, rel=1e-8)
    Z = oracle.forward(g, Q, kd, lo, hi)
    zz = float(np.vdot(Z, Z).real)
    assert f(eta) == pytest.approx(J - gn2 ** 2 / (4 * zz), rel=1e-9)
    Y = oracle.forward(x, Q, kd, lo, hi)
    assert float(np.vdot(Y, Z).real) / zz == pytest.approx(eta, rel=1e-10)
    _, g2, _ = oracle.objective_grad(x - eta * g, mask, Q, kd, lo, hi)
    assert abs(np.vdot(g2, g).real) < 1e-9 * gn2


def test_full_mask_gives_zero_step():
    P = synth.make_problem("gradcheck_48x48x4")
    x, kd = P["x_true"], P["kdims"]
    lo, hi, _ = P["schedule"][0]
    Q, _, _ = oracle.nullspace(oracle.gram(x, kd, lo, hi), P["rank"])
    full = np.ones(P["mask"].shape, np.uint8)
    _, g, gn2 = oracle.objective_grad(x, full, Q, kd, lo, hi)
    assert gn2 == 0.0 and oracle.line_search(g, Q, gn2, kd, lo, hi) == 0.0
    xs = oracle.solve(x, full, kd, P["rank"], [(lo, hi, 2)])
    np.testing.assert_array_equal(xs, x)


def test_solve_monotone_and_data_consistent():
    """No-JL alternating minimisation: J never increases within the inner
    loop (ELS) nor across a nullspace update (the eigenvectors minimise over
    Q); observed samples stay bit-identical to the observations."""
    P = synth.make_problem("2d_64x64x4")
    x0, mask, kd, r = P["x0"], P["mask"], P["kdims"], P["rank"]
    sched = P["schedule"][:4]
    x = x0.astype(complex)
    prev_end = None
    for i, (lo, hi, steps) in enumerate(sched):
        Q, _, _ = oracle.nullspace(oracle.gram(x, kd, lo, hi), r)
        J_start = oracle.objective(x, Q, kd, lo, hi)
        if prev_end is not None:
            assert J_start <= prev_end * (1 + 1e-12)
        y = x
        Jprev = J_start
        for _ in range(steps):
            y, J, _, _ = oracle.descent_step(y, mask, Q, kd, lo, hi)
            assert J <= Jprev * (1 + 1e-12)
            Jprev = J
        x = y
        prev_end = oracle.objective(x, Q, kd, lo, hi)
    xs = oracle.solve(x0, mask, kd, r, sched)
    np.testing.assert_allclose(xs, x, rtol=0, atol=0)
    obs = mask.astype(bool)
    assert np.array_equal(xs[obs], x0[obs])
    assert oracle.ser(xs, P["x_true"]) > oracle.ser(x0, P["x_true"]) + 3.0


def test_solve_resume_matches_uninterrupted():
    P = synth.make_problem("2d_64x64x4")
    x0, mask, kd, r = P["x0"], P["mask"], P["kdims"], P["rank"]
    sched = P["schedule"][:3]
    full = oracle.solve(x0, mask, kd, r, sched, p=8, seed=9)
    part = oracle.solve(x0, mask, kd, r, sched[:1], p=8, seed=9)
    resumed = oracle.solve(part, mask, kd, r, sched, p=8, seed=9, start_outer=1)
    np.testing.assert_array_equal(resumed, full)
