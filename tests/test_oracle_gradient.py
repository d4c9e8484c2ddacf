"""Pins for the oracle's likelihood-ratio gradient.

* Score identity: for theta_j = ln c_j the path score is z_j(t) = n_j(t) - A_j(t), whose
  expectation is zero at every t.
* Closed form (immigration-death, mean m(t) = (k1/k2)(1 - exp(-k2 t))):
  dm/dln k1 = m, dm/dln k2 = -m + k1 t exp(-k2 t).  The estimator
  (1/N) sum_i (X_i - m_hat) z_ij must land within 5 standard errors.
* orc_grad's accumulation at grid crossings (A_j + a_j (t_g - t)) agrees with the
  end-of-horizon record of n_j and A_j (prefix property: a trajectory observed on
  [0, t_g] is the same trajectory).
"""
import math

import numpy as np

from oracle import oracle as orc
from paper_1007_1768_amd import inputs


def _records(m, seed, N, t):
    X = np.zeros((N, len(m["x0"])))
    Z = np.zeros((N, len(m["rates"])))
    for i in range(N):
        st, r = orc.trajectory(m, seed, i, t, np.array([t]))
        assert st == orc.OK
        X[i] = r["states"][0]
        Z[i] = r["n_fired"] - r["a_int"]
    return X, Z


def test_score_identity():
    for m, seed, t in [(inputs.immigration_death(), 1, 30.0), (inputs.viral(), 2, 10.0)]:
        N = 3000
        _, Z = _records(m, seed, N, t)
        for j in range(Z.shape[1]):
            sd = Z[:, j].std(ddof=1)
            if sd == 0:
                assert Z[:, j].mean() == 0
                continue
            assert abs(Z[:, j].mean()) < 5 * sd / math.sqrt(N), j


def test_immigration_death_gradient_closed_form():
    k1, k2 = 10.0, 0.1
    m = inputs.immigration_death(k1, k2)
    N = 6000
    for t in (5.0, 20.0, 60.0):
        X, Z = _records(m, 17, N, t)
        x = X[:, 0]
        mhat = x.mean()
        terms = (x - mhat)[:, None] * Z
        est = terms.mean(axis=0)
        se = terms.std(axis=0, ddof=1) / math.sqrt(N)
        mt = (k1 / k2) * (1 - math.exp(-k2 * t))
        exact = [mt, -mt + k1 * t * math.exp(-k2 * t)]
        for j in range(2):
            assert abs(est[j] - exact[j]) < 5 * se[j], (t, j, est[j], exact[j], se[j])
        # the oracle's gradient routine, with w = 1 at the single grid point t, is the same sum
        st, g, l1 = orc.grad(m, N, t, np.array([t]), 17, np.array([1.0]), np.array([mhat]))
        assert st == orc.OK
        assert np.allclose(g, est, rtol=0, atol=1e-12 * l1.max())
        assert np.allclose(l1, np.abs(terms).mean(axis=0), rtol=1e-12)


def test_grad_is_linear_in_weights_and_matches_grid_prefix():
    m = inputs.viral()
    t_end, G = 4.0, 9
    grid = inputs.uniform_grid(t_end, G)
    N = 400
    st, out = orc.run(m, N, t_end, grid, seed=2)
    mhat = out["mean"]
    rng = np.random.default_rng(0)
    w1 = rng.normal(size=mhat.shape)
    w2 = rng.normal(size=mhat.shape)
    _, g1, l1a = orc.grad(m, N, t_end, grid, 2, w1, mhat)
    _, g2, l1b = orc.grad(m, N, t_end, grid, 2, w2, mhat)
    _, g12, _ = orc.grad(m, N, t_end, grid, 2, w1 + w2, mhat)
    assert np.allclose(g12, g1 + g2, rtol=0, atol=1e-11 * (l1a + l1b).max())
    # a weight only at grid point g gives the same as a run that stops at t_g
    g = 5
    w = np.zeros_like(mhat)
    w[g] = w1[g]
    _, ga, la = orc.grad(m, N, t_end, grid, 2, w, mhat)
    _, gb, lb = orc.grad(m, N, grid[g], grid[:g + 1], 2, w[:g + 1], mhat[:g + 1])
    assert np.allclose(ga, gb, rtol=0, atol=1e-12 * la.max())
    assert np.allclose(la, lb, rtol=1e-12)


def test_jacobian_closed_form_immigration_death():
    """The Jacobian routine on its own: immigration-death's dm/dln k1 = m(t) and
    dm/dln k2 = -m + k1 t exp(-k2 t) at every grid point, within 5 standard errors."""
    k1, k2 = 10.0, 0.1
    m = inputs.immigration_death(k1, k2)
    N, t_end, G = 8000, 40.0, 5
    grid = inputs.uniform_grid(t_end, G)
    st, out = orc.run(m, N, t_end, grid, seed=23)
    assert st == orc.OK
    st, J, l1 = orc.jacobian(m, N, t_end, grid, 23, out["mean"])
    assert st == orc.OK
    for g, t in enumerate(grid):
        mt = (k1 / k2) * (1 - math.exp(-k2 * t))
        exact = [mt, -mt + k1 * t * math.exp(-k2 * t)]
        if t == 0.0:
            assert np.all(J[g] == 0.0)
            continue
        # standard error of a mean of (X - m) z terms: bounded by sqrt(E[(X - m)^2 z^2] / N);
        # Var X = m for the Poisson marginal, E[z_j^2] = E[n_j] = k1 t (births) or the
        # expected deaths (k1 t - m), and the product is bounded by 3 m E[z^2] (fourth moments)
        for j in range(2):
            ez2 = k1 * t if j == 0 else k1 * t - mt
            se = math.sqrt(3.0 * mt * ez2 / N)
            assert abs(J[g, 0, j] - exact[j]) < 5 * se, (t, j, J[g, 0, j], exact[j], se)


def test_jacobian_contracts_to_the_gradient():
    """sum_{g,s} w_{g,s} J_{g,s,j} is the gradient for any w (both from the oracle's own
    crossing visits; this ties the Jacobian to the pinned gradient routine)."""
    m = inputs.viral()
    t_end, G, N = 5.0, 11, 300
    grid = inputs.uniform_grid(t_end, G)
    st, out = orc.run(m, N, t_end, grid, seed=4)
    st, J, l1 = orc.jacobian(m, N, t_end, grid, 4, out["mean"])
    assert st == orc.OK
    w = np.random.default_rng(1).normal(size=out["mean"].shape)
    st, g, gl1 = orc.grad(m, N, t_end, grid, 4, w, out["mean"])
    assert np.allclose(np.einsum("gs,gsj->j", w, J), g, rtol=0, atol=1e-12 * gl1.max())
    # the L1 scales are consistent too
    assert np.all(np.einsum("gs,gsj->j", np.abs(w), l1) >= gl1 * (1 - 1e-12))


def test_immigration_death_variance_gradient_closed_form():
    """Poisson marginals: var(t) = m(t), so d var / d ln k has the mean's closed form.  The
    variance estimator (1/N) sum_i ((X_i - m_hat)^2 - v_hat) z_ij lands within 5 standard
    errors, and the oracle's gradient routine with wv = 1 (w = 0) computes that sum."""
    k1, k2 = 10.0, 0.1
    m = inputs.immigration_death(k1, k2)
    N = 8000
    for t in (5.0, 20.0, 60.0):
        X, Z = _records(m, 23, N, t)
        x = X[:, 0]
        mhat, vhat = x.mean(), x.var(ddof=1)
        terms = ((x - mhat) ** 2 - vhat)[:, None] * Z
        est = terms.mean(axis=0)
        se = terms.std(axis=0, ddof=1) / math.sqrt(N)
        mt = (k1 / k2) * (1 - math.exp(-k2 * t))
        exact = [mt, -mt + k1 * t * math.exp(-k2 * t)]
        for j in range(2):
            assert abs(est[j] - exact[j]) < 5 * se[j], (t, j, est[j], exact[j], se[j])
        st, g, l1 = orc.grad(m, N, t, np.array([t]), 23, np.array([0.0]), np.array([mhat]),
                             wv=np.array([1.0]), vhat=np.array([vhat]))
        assert st == orc.OK
        assert np.allclose(g, est, rtol=0, atol=1e-12 * l1.max())
        # the variance and mean parts add
        _, gm, _ = orc.grad(m, N, t, np.array([t]), 23, np.array([0.7]), np.array([mhat]))
        _, gb, lb = orc.grad(m, N, t, np.array([t]), 23, np.array([0.7]), np.array([mhat]),
                             wv=np.array([1.0]), vhat=np.array([vhat]))
        assert np.allclose(gb, gm + g, rtol=0, atol=1e-12 * lb.max())
