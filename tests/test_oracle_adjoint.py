"""Pins of the oracle's adjoint against finite differences (CPU)."""
import numpy as np
import pytest

import meshgen as mg
from oracle import adjoint, fem, local, solver


def _total_gradient(prob, x, A):
    from oracle import contact as oc
    F = local.deformation_gradients(x, prob.tets, prob.B)
    _, P = local.projections(F, A)
    cs = oc.constraint_set(x, prob.prox, prob.dhat)
    _, gB, _, _ = solver.barrier_terms(prob, x, cs)
    return solver.pd_gradient(prob, F, P) + gB


def _converged(prob, x0, a, R0, tol=1e-12):
    """Algorithm 1 to tol, then Newton steps on the true Hessian to round-off."""
    import scipy.sparse.linalg as spla
    A = fem.actuation_matrices(a, R0)
    x = solver.frame(prob, x0, A, tol=tol, max_iters=2000).x
    f = prob.free
    for _ in range(4):
        K = adjoint.energy_hessian(prob, x, a, R0)
        g = _total_gradient(prob, x, A)
        dx = np.zeros(3 * prob.n)
        dx[f] = -spla.splu(K[f][:, f].tocsc()).solve(g[f])
        x = x + dx.reshape(-1, 3)
    return x


def _loss(x, idx, target):
    d = x[idx] - target
    return float(np.sum(d * d)), d


def test_energy_hessian_matches_gradient_differences():
    sc = mg.slabs(0, nx=2, ny=2, nz=2, gap=1e-3)
    prob = solver.setup_scene(sc)
    rng = np.random.default_rng(0)
    a = 0.2 * sc.act_a
    x = sc.X + 2e-4 * rng.standard_normal(sc.X.shape) * (sc.dirichlet[:, None] == 0)
    K = adjoint.energy_hessian(prob, x, a, sc.act_R).toarray()
    A = fem.actuation_matrices(a, sc.act_R)

    def grad(xx):
        F = local.deformation_gradients(xx, prob.tets, prob.B)
        _, P = local.projections(F, A)
        return solver.pd_gradient(prob, F, P)

    v = rng.standard_normal(x.shape) * (sc.dirichlet[:, None] == 0)
    h = 1e-7
    fd = (grad(x + h * v) - grad(x - h * v)) / (2 * h)
    Kv = K @ v.reshape(-1)
    assert np.allclose(Kv, fd, rtol=1e-5, atol=1e-6 * np.abs(fd).max())


@pytest.mark.parametrize("contact", [False, True])
def test_adjoint_gradient_matches_finite_differences(contact):
    sc = mg.slabs(0, nx=2, ny=2, nz=1, gap=(1e-3 if contact else 0.02))
    prob = solver.setup_scene(sc)
    rng = np.random.default_rng(1)
    a = (1.0 if contact else 0.5) * sc.act_a
    x0 = sc.X.copy()
    xs = _converged(prob, x0, a, sc.act_R)
    if contact:
        from oracle import contact as oc
        assert oc.constraint_set(xs, prob.prox, prob.dhat).size > 0
    idx = rng.choice(np.nonzero(sc.dirichlet == 0)[0], 6, replace=False)
    target = xs[idx] + 1e-3 * rng.standard_normal((6, 3))
    _, d = _loss(xs, idx, target)
    dLdx = np.zeros_like(xs)
    dLdx[idx] = 2 * d
    g = adjoint.actuation_gradient(prob, xs, a, sc.act_R, dLdx)
    h = 1e-6
    for i in rng.choice(sc.m, 3, replace=False):
        ap, am = a.copy(), a.copy()
        ap[i] += h
        am[i] -= h
        Lp, _ = _loss(_converged(prob, xs, ap, sc.act_R), idx, target)
        Lm, _ = _loss(_converged(prob, xs, am, sc.act_R), idx, target)
        fd = (Lp - Lm) / (2 * h)
        assert abs(g[i] - fd) <= 1e-6 * max(abs(fd), 1e-2 * np.abs(g).max()), (i, g[i], fd)
