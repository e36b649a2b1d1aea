"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks an oracle function against something other than itself:
closed forms, invariants, special cases that reduce to a textbook formula,
brute force on tiny inputs, or finite differences.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import meshgen as mg
from oracle import barrier, ccd, contact, fem, geometry as geo, local, solver

RNG = np.random.default_rng(1234)


def rand_rot(k):
    return mg.random_rotations(np.random.default_rng(7), k)


# --------------------------------------------------------------------------
# Eq. (1): deformation gradient, rotation fit, element energy
# --------------------------------------------------------------------------
def test_affine_map_has_exact_deformation_gradient():
    sc = mg.slabs(0, nx=2, ny=2, nz=1)
    _, B, V = fem.rest_data(sc.X, sc.tets)
    M = np.array([[1.1, 0.2, -0.05], [0.03, 0.9, 0.1], [-0.2, 0.05, 1.3]])
    x = sc.X @ M.T + np.array([0.3, -0.1, 2.0])
    F = local.deformation_gradients(x, sc.tets, B)
    assert np.allclose(F, M[None], atol=1e-12)
    # G_i x_local = vec(F) row-major
    G = fem.gradient_operators(B)
    xl = x[sc.tets].reshape(-1, 12)
    assert np.allclose(np.einsum("mij,mj->mi", G, xl), F.reshape(-1, 9), atol=1e-12)


def test_rest_volumes_tile_the_hexes():
    sc = mg.slabs(0, nx=3, ny=2, nz=2, h=0.01)
    _, _, V = fem.rest_data(sc.X, sc.tets)
    assert np.allclose(V, 0.01 ** 3 / 6, rtol=1e-12)
    assert np.isclose(V.sum(), 2 * 3 * 2 * 2 * 0.01 ** 3, rtol=1e-12)


def test_inverted_rest_tet_is_rejected():
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0]])
    with pytest.raises(ValueError):
        fem.rest_data(X, np.array([[0, 2, 1, 3]]))
    with pytest.raises(ValueError):
        fem.rest_data(np.zeros((4, 3)), np.array([[0, 1, 2, 3]]))


def test_rotation_fit_recovers_constructed_rotation():
    k = 50
    R0 = rand_rot(k)
    L = RNG.standard_normal((k, 3, 3))
    S = L @ np.swapaxes(L, 1, 2) + 0.5 * np.eye(3)      # SPD
    M = R0 @ S
    # with A = I, F = M: the nearest rotation to R0 S (S SPD) is R0
    R = local.best_rotations(M, np.broadcast_to(np.eye(3), (k, 3, 3)))
    assert np.allclose(R, R0, atol=1e-12)


def test_rotation_fit_beats_sampled_rotations():
    F = RNG.standard_normal((6, 3, 3))
    A = RNG.standard_normal((6, 3, 3))
    A = 0.5 * (A + np.swapaxes(A, 1, 2)) + 2 * np.eye(3)
    R = local.best_rotations(F, A)
    assert np.allclose(np.linalg.det(R), 1.0)
    assert np.allclose(R @ np.swapaxes(R, 1, 2), np.eye(3), atol=1e-12)
    best = np.sum((F - R @ A) ** 2, axis=(1, 2))
    samples = mg.random_rotations(np.random.default_rng(3), 20000)
    for i in range(F.shape[0]):
        e = np.sum((F[i][None] - samples @ A[i]) ** 2, axis=(1, 2))
        assert best[i] <= e.min() + 1e-12


def test_element_energy_closed_form():
    """min_R ||F - R A||^2 = ||F||^2 + ||A||^2 - 2 (s1 + s2 + sign(det FA) s3)."""
    F = RNG.standard_normal((40, 3, 3))
    A = RNG.standard_normal((40, 3, 3))
    A = 0.5 * (A + np.swapaxes(A, 1, 2))
    s = np.linalg.svd(F @ A, compute_uv=False)
    sg = np.sign(np.linalg.det(F @ A))
    closed = (np.sum(F ** 2, axis=(1, 2)) + np.sum(A ** 2, axis=(1, 2))
              - 2 * (s[:, 0] + s[:, 1] + sg * s[:, 2]))
    E = local.element_energies(F, A, np.full(40, 2.0))
    assert np.allclose(E, closed, rtol=1e-12, atol=1e-12)


def test_identity_state_projects_to_identity():
    F = np.broadcast_to(np.eye(3), (5, 3, 3)).copy()
    R, P = local.projections(F, F.copy())
    assert np.allclose(P, np.eye(3)) and np.allclose(local.element_energies(F, F, np.ones(5)), 0)


def test_actuation_matrix_definition():
    R = rand_rot(4)
    a = np.array([0.0, 0.1, 0.2, 0.3])
    A = fem.actuation_matrices(a, R)
    for i in range(4):
        ev = np.sort(np.linalg.eigvalsh(A[i]))
        assert np.allclose(ev, np.sort([1 - a[i], 1 + a[i] / 2, 1 + a[i] / 2]))
        assert np.allclose(A[i] @ R[i][:, 0], (1 - a[i]) * R[i][:, 0])
    dA = fem.actuation_derivative(R)
    h = 1e-6
    fd = (fem.actuation_matrices(a + h, R) - fem.actuation_matrices(a - h, R)) / (2 * h)
    assert np.allclose(dA, fd, atol=1e-9)


# --------------------------------------------------------------------------
# Eq. (2): the constant PD matrix
# --------------------------------------------------------------------------
def test_pd_matrix_structure():
    sc = mg.slabs(0, nx=3, ny=3, nz=1)
    prob = solver.setup_scene(sc)
    H = prob.H.toarray()
    n = sc.n
    # translation invariance: rows sum to zero per coordinate
    for c in range(3):
        t = np.zeros(3 * n)
        t[c::3] = 1.0
        assert np.abs(H @ t).max() < 1e-9 * np.abs(H).max()
    # Kronecker structure H = H_s (x) I_3
    Hs = H[0::3, 0::3]
    assert np.allclose(H, np.kron(Hs, np.eye(3)), atol=1e-12 * np.abs(H).max())
    # SPD once the fixed vertices are removed
    f = prob.free
    ev = np.linalg.eigvalsh(H[np.ix_(f, f)])
    assert ev.min() > 0


def test_pd_gradient_is_energy_gradient():
    sc = mg.slabs(0, nx=2, ny=2, nz=1)
    prob = solver.setup_scene(sc)
    A = fem.actuation_matrices(sc.act_a, sc.act_R)
    x = sc.X + 1e-3 * RNG.standard_normal(sc.X.shape)

    def E(xx):
        F = local.deformation_gradients(xx, prob.tets, prob.B)
        return local.element_energies(F, A, prob.w).sum()

    F = local.deformation_gradients(x, prob.tets, prob.B)
    _, P = local.projections(F, A)
    g = solver.pd_gradient(prob, F, P)
    h = 1e-7
    for dof in RNG.choice(3 * sc.n, 12, replace=False):
        xp, xm = x.copy().reshape(-1), x.copy().reshape(-1)
        xp[dof] += h
        xm[dof] -= h
        fd = (E(xp.reshape(-1, 3)) - E(xm.reshape(-1, 3))) / (2 * h)
        assert np.isclose(g[dof], fd, rtol=1e-5, atol=1e-10 * np.abs(g).max())


def test_rest_state_with_identity_actuation_has_zero_gradient():
    sc = mg.slabs(0, nx=2, ny=2, nz=1)
    prob = solver.setup_scene(sc)
    A = fem.actuation_matrices(np.zeros(sc.m), sc.act_R)
    F = local.deformation_gradients(sc.X, prob.tets, prob.B)
    _, P = local.projections(F, A)
    assert np.abs(solver.pd_gradient(prob, F, P)).max() < 1e-10


# --------------------------------------------------------------------------
# distances between closed primitives
# --------------------------------------------------------------------------
def test_point_above_triangle_interior():
    a, b, c = np.array([0, 0, 0.0]), np.array([1, 0, 0.0]), np.array([0, 1, 0.0])
    p = np.array([0.2, 0.3, 0.37])
    d2, kind, idx = geo.point_triangle(p, a, b, c)
    assert np.isclose(d2[0], 0.37 ** 2) and kind[0] == geo.PT


def test_point_triangle_edge_and_vertex_regions():
    a, b, c = np.array([0, 0, 0.0]), np.array([1, 0, 0.0]), np.array([0, 1, 0.0])
    d2, kind, idx = geo.point_triangle(np.array([0.5, -0.2, 0.1]), a, b, c)
    assert np.isclose(d2[0], 0.2 ** 2 + 0.1 ** 2) and kind[0] == geo.PE and list(idx[0][:3]) == [0, 1, 2]
    d2, kind, idx = geo.point_triangle(np.array([-0.3, -0.4, 0.0]), a, b, c)
    assert np.isclose(d2[0], 0.25) and kind[0] == geo.PP and list(idx[0][:2]) == [0, 1]


def test_skew_and_parallel_segments():
    a0, a1 = np.array([0, 0, 0.0]), np.array([1, 0, 0.0])
    d2, kind, _ = geo.edge_edge(a0, a1, np.array([0.5, -1, 0.25]), np.array([0.5, 1, 0.25]))
    assert np.isclose(d2[0], 0.0625) and kind[0] == geo.EE
    # parallel, overlapping: distance is the offset
    d2, kind, _ = geo.edge_edge(a0, a1, np.array([0.2, 0.3, 0.0]), np.array([1.4, 0.3, 0.0]))
    assert np.isclose(d2[0], 0.09) and kind[0] in (geo.PE, geo.PP)
    # collinear, disjoint: gap between the ends
    d2, _, _ = geo.edge_edge(a0, a1, np.array([1.5, 0, 0.0]), np.array([3, 0, 0.0]))
    assert np.isclose(d2[0], 0.25)


def _sample_tri(a, b, c, n=120):
    u, v = np.meshgrid(np.linspace(0, 1, n), np.linspace(0, 1, n))
    ok = u + v <= 1
    u, v = u[ok], v[ok]
    return a + u[:, None] * (b - a) + v[:, None] * (c - a)


def _sample_seg(a, b, n=2000):
    t = np.linspace(0, 1, n)[:, None]
    return a + t * (b - a)


def test_distances_against_dense_sampling():
    rng = np.random.default_rng(5)
    for _ in range(25):
        p, a, b, c = rng.standard_normal((4, 3))
        d = np.sqrt(geo.point_triangle(p, a, b, c)[0][0])
        S = _sample_tri(a, b, c)
        ds = np.linalg.norm(S - p, axis=1).min()
        assert d <= ds + 1e-12 and ds - d < 0.05 * np.linalg.norm(b - a) + 0.05
        a0, a1, b0, b1 = rng.standard_normal((4, 3))
        d = np.sqrt(geo.edge_edge(a0, a1, b0, b1)[0][0])
        SA, SB = _sample_seg(a0, a1, 600), _sample_seg(b0, b1, 600)
        dd = np.linalg.norm(SA[:, None] - SB[None], axis=2).min()
        assert d <= dd + 1e-12 and dd - d < 1e-2


def test_feature_formula_matches_classified_distance():
    rng = np.random.default_rng(9)
    P = rng.standard_normal((500, 4, 3))
    d2, kind, idx = geo.point_triangle(P[:, 0], P[:, 1], P[:, 2], P[:, 3])
    assert np.allclose(barrier.squared_distance_by_feature(P, kind, idx), d2, rtol=1e-10, atol=1e-14)
    d2, kind, idx = geo.edge_edge(P[:, 0], P[:, 1], P[:, 2], P[:, 3])
    assert np.allclose(barrier.squared_distance_by_feature(P, kind, idx), d2, rtol=1e-10, atol=1e-14)


# --------------------------------------------------------------------------
# Eq. (3): barrier and derivatives
# --------------------------------------------------------------------------
DHAT, KAPPA = 5e-4, 1e3


def _b1(d):
    return -2 * (d - DHAT) * np.log(d / DHAT) - (d - DHAT) ** 2 / d


def _b2(d):
    return -2 * np.log(d / DHAT) - 4 * (d - DHAT) / d + (d - DHAT) ** 2 / d ** 2


def test_barrier_vanishes_smoothly_at_threshold():
    assert barrier.barrier(np.array([DHAT, 2 * DHAT]), DHAT).max() == 0
    assert np.isclose(_b1(DHAT), 0) and np.isclose(_b2(DHAT), 0)
    assert barrier.barrier(np.array([1e-6]), DHAT)[0] > 0


def test_single_point_triangle_closed_form():
    """Point at height h over a triangle interior: grad_p = kappa b'(h) n, Hess_pp = kappa b''(h) n n^T."""
    h = 2e-4
    tri = np.array([[0, 0, 0], [0.01, 0, 0], [0, 0.01, 0.0]])
    X4 = np.concatenate([np.array([[0.002, 0.003, h]]), tri])[None]
    d2, kind, idx = geo.point_triangle(X4[:, 0], X4[:, 1], X4[:, 2], X4[:, 3])
    E, G, H = barrier.pair_derivatives(X4, kind, idx, DHAT, KAPPA)
    n = np.array([0, 0, 1.0])
    assert np.isclose(E[0], KAPPA * barrier.barrier(np.array([h]), DHAT)[0], rtol=1e-12)
    assert np.allclose(G[0, :3], KAPPA * _b1(h) * n, rtol=1e-10)
    assert np.allclose(G[0].reshape(4, 3).sum(axis=0), 0, atol=1e-9 * np.abs(G).max())
    assert np.allclose(H[0, :3, :3], KAPPA * _b2(h) * np.outer(n, n), rtol=1e-9, atol=1e-9 * abs(_b2(h)) * KAPPA)


def _fd_pair(X4, dhat, kappa, eps):
    """Central FD of the barrier built from the min-over-candidates distance."""
    def energy(Y):
        Y = Y.reshape(1, 4, 3)
        if pair_is_pt:
            d2 = geo.point_triangle(Y[:, 0], Y[:, 1], Y[:, 2], Y[:, 3])[0]
        else:
            d2 = geo.edge_edge(Y[:, 0], Y[:, 1], Y[:, 2], Y[:, 3])[0]
        return kappa * barrier.barrier(np.sqrt(d2), dhat)[0]
    global pair_is_pt
    x = X4.reshape(-1)
    g = np.zeros(12)
    for i in range(12):
        e = np.zeros(12)
        e[i] = eps
        g[i] = (energy(x + e) - energy(x - e)) / (2 * eps)
    return g


def _grad_fn(X4, is_pt):
    def gfun(y):
        Y = y.reshape(1, 4, 3)
        f = geo.point_triangle if is_pt else geo.edge_edge
        d2, kind, idx = f(Y[:, 0], Y[:, 1], Y[:, 2], Y[:, 3])
        return barrier.pair_derivatives(Y, kind, idx, DHAT, KAPPA)[1][0]
    return gfun


@pytest.mark.parametrize("is_pt", [True, False])
def test_barrier_derivatives_against_finite_differences(is_pt):
    global pair_is_pt
    pair_is_pt = is_pt
    rng = np.random.default_rng(11 if is_pt else 12)
    checked = 0
    while checked < 6:
        base = rng.uniform(-0.005, 0.005, (3, 3))
        if is_pt:
            p = base.mean(axis=0) + rng.uniform(-1e-3, 1e-3, 3)
            n = np.cross(base[1] - base[0], base[2] - base[0])
            p = p + n / np.linalg.norm(n) * rng.uniform(1e-4, 4e-4)
            X4 = np.concatenate([p[None], base])[None]
            d2, kind, idx = geo.point_triangle(X4[:, 0], X4[:, 1], X4[:, 2], X4[:, 3])
        else:
            a0, a1 = base[0], base[1]
            mid = 0.5 * (a0 + a1)
            dirb = rng.standard_normal(3)
            off = rng.standard_normal(3)
            off /= np.linalg.norm(off)
            b0 = mid + off * 3e-4 - 0.004 * dirb / np.linalg.norm(dirb)
            b1 = mid + off * 3e-4 + 0.004 * dirb / np.linalg.norm(dirb)
            X4 = np.stack([a0, a1, b0, b1])[None]
            d2, kind, idx = geo.edge_edge(X4[:, 0], X4[:, 1], X4[:, 2], X4[:, 3])
        d = np.sqrt(d2[0])
        if not (5e-5 < d < 4.5e-4):
            continue
        E, G, H = barrier.pair_derivatives(X4, kind, idx, DHAT, KAPPA)
        eps = 1e-9
        g_fd = _fd_pair(X4[0], DHAT, KAPPA, eps)
        assert np.allclose(G[0], g_fd, rtol=2e-4, atol=2e-4 * np.abs(G[0]).max())
        gfun = _grad_fn(X4, is_pt)
        x = X4.reshape(-1)
        Hfd = np.zeros((12, 12))
        for i in range(12):
            e = np.zeros(12)
            e[i] = eps
            Hfd[:, i] = (gfun(x + e) - gfun(x - e)) / (2 * eps)
        assert np.allclose(H[0], Hfd, rtol=1e-4, atol=1e-4 * np.abs(H[0]).max())
        assert np.allclose(H[0], H[0].T, atol=1e-9 * np.abs(H[0]).max())
        assert np.allclose(G[0].reshape(4, 3).sum(axis=0), 0, atol=1e-8 * np.abs(G[0]).max())
        checked += 1


def test_psd_projection():
    rng = np.random.default_rng(2)
    M = rng.standard_normal((20, 12, 12))
    M = M + np.swapaxes(M, 1, 2)
    P = barrier.project_psd(M)
    for i in range(20):
        ev = np.linalg.eigvalsh(P[i])
        assert ev.min() > -1e-12 * np.abs(ev).max()
        # nearest PSD matrix in Frobenius norm: residual is negative semidefinite
        assert np.linalg.eigvalsh(M[i] - P[i]).max() < 1e-10
    Q = np.einsum("kij,klj->kil", M, M)
    assert np.allclose(barrier.project_psd(Q), Q, atol=1e-10)


# --------------------------------------------------------------------------
# constraint sets
# --------------------------------------------------------------------------
def _brute_sets(x, prox, dhat):
    pt, ee = [], []
    for v in prox.verts:
        for f, tri in enumerate(prox.tris):
            if v in tri:
                continue
            d2 = geo.point_triangle(x[v], x[tri[0]], x[tri[1]], x[tri[2]])[0][0]
            if d2 < dhat * dhat:
                pt.append((v, f))
    E = prox.edges
    for i in range(len(E)):
        for j in range(i + 1, len(E)):
            if len(set(E[i]) & set(E[j])):
                continue
            d2 = geo.edge_edge(x[E[i][0]], x[E[i][1]], x[E[j][0]], x[E[j][1]])[0][0]
            if d2 < dhat * dhat:
                ee.append((i, j))
    return np.array(pt, dtype=np.int64).reshape(-1, 2), np.array(ee, dtype=np.int64).reshape(-1, 2)


def test_constraint_set_equals_brute_force_on_tiny_mesh():
    sc = mg.slabs(0, nx=3, ny=3, nz=1, gap=1e-3)
    prox = contact.make_proxy(sc.surf_tris)
    rng = np.random.default_rng(4)
    x = sc.X.copy()
    upper = x[:, 2] > 0.0105
    x[upper, 2] -= 7e-4                              # gap 0.3 mm < dhat
    x += rng.uniform(-1e-4, 1e-4, x.shape)
    cs = contact.constraint_set(x, prox, DHAT)
    bpt, bee = _brute_sets(x, prox, DHAT)
    assert cs.size > 0
    assert np.array_equal(cs.pt, bpt) and np.array_equal(cs.ee, bee)


# --------------------------------------------------------------------------
# Eq. (4)-(11): the global step
# --------------------------------------------------------------------------
def _contact_state(seed=0):
    sc = mg.slabs(seed, nx=3, ny=3, nz=2, gap=1e-3)
    prob = solver.setup_scene(sc)
    x = sc.X.copy()
    x[x[:, 2] > 0.0205, 2] -= 7e-4
    x += np.random.default_rng(seed).uniform(-5e-5, 5e-5, x.shape) * (sc.dirichlet[:, None] == 0)
    return sc, prob, x


def test_sparse_lu_step_equals_dense_solve_and_schur_woodbury():
    sc, prob, x = _contact_state()
    A = fem.actuation_matrices(sc.act_a * 0.5, sc.act_R)
    F = local.deformation_gradients(x, prob.tets, prob.B)
    _, P = local.projections(F, A)
    cs = contact.constraint_set(x, prob.prox, prob.dhat)
    assert cs.size > 0
    _, gB, Bm, _ = solver.barrier_terms(prob, x, cs)
    g = solver.pd_gradient(prob, F, P) + gB
    f = prob.free
    K = (prob.H + Bm).toarray()[np.ix_(f, f)]
    dx_lu = -spla.splu((prob.H + Bm).tocsc()[f][:, f].tocsc()).solve(g[f])
    dx_dense = -np.linalg.solve(K, g[f])
    assert np.allclose(dx_lu, dx_dense, rtol=1e-10, atol=1e-12 * np.abs(dx_dense).max())
    # Eq. (6)-(8): split free DOFs into x1 (no contact) and x2 (proxy vertices)
    fv = f[0::3] // 3
    in2 = sc.region[fv] == 1
    d1 = (3 * fv[~in2][:, None] + np.arange(3)).reshape(-1)
    d2 = (3 * fv[in2][:, None] + np.arange(3)).reshape(-1)
    H = prob.H.toarray()
    Bd = Bm.toarray()
    assert np.abs(Bd[np.ix_(d1, d1)]).max() == 0 and np.abs(Bd[np.ix_(d1, d2)]).max() == 0
    H11, H12, H21, H22 = H[np.ix_(d1, d1)], H[np.ix_(d1, d2)], H[np.ix_(d2, d1)], H[np.ix_(d2, d2)]
    r1, r2 = -g[d1], -g[d2]
    L1 = np.linalg.cholesky(H11)
    Sig = H22 - H21 @ np.linalg.solve(H11, H12)
    B22 = Bd[np.ix_(d2, d2)]
    # Eq. (7): block factorisation reproduces the permuted matrix
    Lb = np.block([[L1, np.zeros_like(H12)], [H21 @ np.linalg.inv(L1).T, np.eye(len(d2))]])
    Db = np.block([[np.eye(len(d1)), np.zeros_like(H12)], [np.zeros_like(H21), Sig + B22]])
    Ub = np.block([[L1.T, np.linalg.solve(L1, H12)], [np.zeros_like(H21), np.eye(len(d2))]])
    Kp = np.block([[H11, H12], [H21, H22 + B22]])
    assert np.allclose(Lb @ Db @ Ub, Kp, rtol=1e-10, atol=1e-10 * np.abs(Kp).max())
    # Eq. (11) on the affected DOFs, in the form without B-check inverse
    c_rows = np.nonzero(np.abs(B22).sum(axis=1) > 0)[0]
    Bc = B22[np.ix_(c_rows, c_rows)]
    Sinv = np.linalg.inv(Sig)
    rt2 = r2 - H21 @ np.linalg.solve(H11, r1)
    z = Sinv @ rt2
    C = Sinv[np.ix_(c_rows, c_rows)]
    u = np.linalg.solve(np.linalg.inv(C) + Bc, np.linalg.solve(C, z[c_rows]))
    dx2 = z - Sinv[:, c_rows] @ (Bc @ u)
    dx1 = np.linalg.solve(H11, r1 - H12 @ dx2)
    full = np.zeros(3 * sc.n)
    full[d1], full[d2] = dx1, dx2
    assert np.allclose(full[f], dx_dense, rtol=1e-8, atol=1e-9 * np.abs(dx_dense).max())
    # Sigma^-1 equals the (2,2) block of the inverse PD matrix
    Hff_inv = np.linalg.inv(np.block([[H11, H12], [H21, H22]]))
    assert np.allclose(Sinv, Hff_inv[len(d1):, len(d1):], rtol=1e-8, atol=1e-8 * np.abs(Sinv).max())


# --------------------------------------------------------------------------
# CCD
# --------------------------------------------------------------------------
def test_ccd_point_approaching_static_triangle():
    tri = np.array([[0, 0, 0], [0.01, 0, 0], [0, 0.01, 0.0]])
    d0, v = 4e-4, 1e-3
    x = np.concatenate([tri, [[0.002, 0.003, d0]]])
    dx = np.zeros_like(x)
    dx[3, 2] = -v
    prox = contact.Proxy(verts=np.array([3]), tris=np.array([[0, 1, 2]]), edges=np.zeros((0, 2), np.int64))
    t = ccd.pair_step_bounds(x, dx, prox, np.array([[3, 0]]), np.zeros((0, 2), np.int64))
    assert np.isclose(t[0], min(1.0, (1 - ccd.ETA) * d0 / v), rtol=1e-12)
    dx[3, 2] = -1e-5
    t = ccd.pair_step_bounds(x, dx, prox, np.array([[3, 0]]), np.zeros((0, 2), np.int64))
    assert t[0] == 1.0


def test_ccd_keeps_every_pair_above_target_gap():
    sc, prob, x = _contact_state(1)
    rng = np.random.default_rng(8)
    dx = rng.standard_normal(x.shape) * 1e-3 * (sc.dirichlet[:, None] == 0)
    alpha_m, spt, see = ccd.step_bound(x, dx, prob.prox, prob.dhat)
    assert 0 < alpha_m < 1
    X4 = contact.pair_points(x, prob.prox, spt, see)
    d0 = np.sqrt(contact.pair_distances(x, prob.prox, spt, see)[0])
    for s in np.linspace(0, 1, 41):
        d = np.sqrt(contact.pair_distances(x + s * alpha_m * dx, prob.prox, spt, see)[0])
        assert np.all(d >= ccd.ETA * d0 * (1 - 1e-9))
    assert X4.shape[0] > 0


# --------------------------------------------------------------------------
# Algorithm 1: whole-frame invariants
# --------------------------------------------------------------------------
def test_zero_actuation_returns_rest_shape():
    sc = mg.slabs(0, nx=3, ny=3, nz=1)
    prob = solver.setup_scene(sc)
    A = fem.actuation_matrices(np.zeros(sc.m), sc.act_R)
    r = solver.frame(prob, sc.X, A, iters=3)
    assert np.abs(r.x - sc.X).max() < 1e-15
    rng = np.random.default_rng(0)
    x0 = sc.X + 2e-4 * rng.standard_normal(sc.X.shape) * (sc.dirichlet[:, None] == 0)
    r = solver.frame(prob, x0, A, tol=1e-13, max_iters=300)
    assert np.abs(r.x - sc.X).max() < 1e-11


def _plain_pd(prob, x, A, iters):
    """Plain projective dynamics: x <- H^-1 sum w G^T p on the free DOFs (Eq. 2)."""
    f = prob.free
    lu = spla.splu(prob.H.tocsc()[f][:, f].tocsc())
    x = x.copy().reshape(-1)
    fixed = np.setdiff1d(np.arange(x.size), f)
    for _ in range(iters):
        F = local.deformation_gradients(x.reshape(-1, 3), prob.tets, prob.B)
        _, P = local.projections(F, A)
        rhs = np.zeros(x.size)
        ge = prob.w[:, None] * np.einsum("mki,mk->mi", prob.G, P.reshape(-1, 9))
        np.add.at(rhs, fem.local_dofs(prob.tets).reshape(-1), ge.reshape(-1))
        rhs_f = rhs[f] - prob.H.tocsc()[f][:, fixed] @ x[fixed]
        x[f] = lu.solve(rhs_f)
    return x.reshape(-1, 3)


def test_no_contact_equals_plain_pd():
    sc = mg.slabs(0, nx=3, ny=3, nz=1, gap=0.02)
    prob = solver.setup_scene(sc)
    A = fem.actuation_matrices(0.3 * sc.act_a, sc.act_R)
    r = solver.frame(prob, sc.X, A, iters=6)
    assert max(r.n_pt) == 0 and max(r.n_ee) == 0 and all(a == 1.0 for a in r.alpha)
    ref = _plain_pd(prob, sc.X, A, 6)
    assert np.abs(r.x - ref).max() < 1e-12 * np.abs(sc.X).max()


def test_frames_stay_intersection_free_and_energy_decreases():
    sc = mg.slabs(0, nx=4, ny=4, nz=1, gap=1e-3)
    prob = solver.setup_scene(sc)
    x = sc.X.copy()
    for t in (0.5, 1.0):
        A = fem.actuation_matrices(t * sc.act_a, sc.act_R)
        r = solver.frame(prob, x, A, iters=8, trace=True)
        for rec in r.trace:
            assert 0 < rec.alpha <= rec.alpha_m <= 1
        # the total energy never increases along the iterates (line search on
        # E_hat, Algorithm 1), counted over every pair, active or not
        E = [_total_energy(prob, rec.x, A) for rec in r.trace] + [_total_energy(prob, r.x, A)]
        assert all(E[k + 1] <= E[k] + 1e-14 * abs(E[k]) for k in range(len(E) - 1)), E
        assert E[-1] < E[0]
        x = r.x
        dmin = contact.min_distance(x, prob.prox)
        assert dmin > 0
    assert max(r.n_pt) > 0


# --------------------------------------------------------------------------
# swept candidates, line-search barrier term, energy decrease (Algorithm 1)
# --------------------------------------------------------------------------
def _brute_swept(x0, x1, prox, margin):
    """Swept-box pairs by explicit loops over every pair of primitives.

    A vertex moving linearly from x0 to x1 stays inside the box spanned by its
    two end positions, so a primitive's swept box is the box of all of its
    corners at both ends.  Two boxes overlap with the margin when every axis
    interval, widened by the margin, intersects.
    """
    def box(ids):
        pts = [x0[i] for i in ids] + [x1[i] for i in ids]
        lo = [min(p[a] for p in pts) for a in range(3)]
        hi = [max(p[a] for p in pts) for a in range(3)]
        return lo, hi

    def overlap(b1, b2):
        return all(b1[0][a] <= b2[1][a] + margin and b2[0][a] <= b1[1][a] + margin for a in range(3))

    pt, ee = [], []
    for v in prox.verts:
        bv = box([v])
        for f, tri in enumerate(prox.tris):
            if v not in tri and overlap(bv, box(tri)):
                pt.append((v, f))
    E = prox.edges
    for i in range(len(E)):
        for j in range(i + 1, len(E)):
            if not set(E[i]) & set(E[j]) and overlap(box(E[i]), box(E[j])):
                ee.append((i, j))
    return np.array(pt, np.int64).reshape(-1, 2), np.array(ee, np.int64).reshape(-1, 2)


def test_swept_candidates_equal_brute_force_enumeration():
    sc = mg.slabs(0, nx=3, ny=3, nz=1, gap=1e-3)
    prox = contact.make_proxy(sc.surf_tris)
    rng = np.random.default_rng(11)
    x0 = sc.X + rng.uniform(-1e-4, 1e-4, sc.X.shape)
    dx = rng.standard_normal(sc.X.shape) * 6e-4
    dx[sc.X[:, 2] > 0.0105, 2] -= 1.5e-3             # upper face sweeps through the gap
    pt, ee = contact.candidates(x0, x0 + dx, prox, DHAT)
    bpt, bee = _brute_swept(x0, x0 + dx, prox, DHAT)
    assert len(pt) > 0 and len(ee) > 0
    assert np.array_equal(pt, bpt) and np.array_equal(ee, bee)


def test_swept_candidates_hold_a_pair_that_meets_only_mid_sweep():
    """A point passing straight through a triangle: apart by more than dhat at
    both ends of the motion, at distance 0 half-way.  Only a box over the
    whole motion (not over either end state) contains that pair."""
    tri = np.array([[0.0, 0.0, 0.0], [1e-2, 0.0, 0.0], [0.0, 1e-2, 0.0]])
    p0, p1 = np.array([-4e-3, 2e-3, 4e-3]), np.array([8e-3, 2e-3, -4e-3])
    x0 = np.vstack([tri, p0])
    x1 = np.vstack([tri, p1])
    prox = contact.Proxy(verts=np.array([3]), tris=np.array([[0, 1, 2]]), edges=np.zeros((0, 2), np.int64))
    for xa, xb in ((x0, x0), (x1, x1)):
        assert len(contact.candidates(xa, xb, prox, DHAT)[0]) == 0
    pt, _ = contact.candidates(x0, x1, prox, DHAT)
    assert pt.tolist() == [[3, 0]]
    # the distance along the motion does drop to zero half-way
    mid = 0.5 * (x0 + x1)
    assert geo.point_triangle(mid[3], *tri)[0][0] < 1e-30


def test_swept_candidates_contain_every_pair_that_comes_within_dhat():
    """Completeness, the property the step bound and the line search rely on:
    every pair whose distance drops below dhat anywhere along the linear
    motion (dense sampling of the motion) is a candidate."""
    sc = mg.slabs(2, nx=3, ny=3, nz=1, gap=1e-3)
    prox = contact.make_proxy(sc.surf_tris)
    rng = np.random.default_rng(5)
    x0 = sc.X + rng.uniform(-1e-4, 1e-4, sc.X.shape)
    dx = rng.standard_normal(sc.X.shape) * 3e-4
    dx[sc.X[:, 2] > 0.0105, 2] -= 9e-4
    pt, ee = contact.candidates(x0, x0 + dx, prox, DHAT)
    have_pt = {tuple(r) for r in pt.tolist()}
    have_ee = {tuple(r) for r in ee.tolist()}
    apt, aee = contact.candidates(x0, x0, prox, 1.0)   # every non-incident pair
    dmin = np.full(len(apt) + len(aee), np.inf)
    for s in np.linspace(0.0, 1.0, 201):
        dmin = np.minimum(dmin, contact.pair_distances(x0 + s * dx, prox, apt, aee)[0])
    close = dmin < DHAT * DHAT
    npt = len(apt)
    assert close[:npt].sum() > 0 and close[npt:].sum() > 0
    assert all(tuple(r) in have_pt for r in apt[close[:npt]].tolist())
    assert all(tuple(r) in have_ee for r in aee[close[npt:]].tolist())


def _total_energy(prob, x, A):
    """E_hat(x) = sum_i (w_i/2)||F_i - R_i A_i||^2 + kappa sum_k b(d_k) over every
    non-incident pair (pairs at d >= dhat contribute 0)."""
    F = local.deformation_gradients(x, prob.tets, prob.B)
    Ee = local.element_energies(F, A, prob.w).sum()
    cs = contact.constraint_set(x, prob.prox, prob.dhat)
    Eb = prob.kappa * barrier.barrier(np.sqrt(cs.d2), prob.dhat).sum()
    return Ee + Eb


def test_line_search_counts_pairs_that_enter_dhat_along_the_step():
    """A step that lowers the elastic energy but brings pairs that are not yet
    active to a small gap: the barrier differences over the swept candidates
    must reject the CCD bound (a search over the active set alone, or over
    the elastic energy alone, would accept it)."""
    sc = mg.slabs(0, nx=3, ny=3, nz=1, gap=1e-3)
    prob = solver.setup_scene(sc)
    A = fem.actuation_matrices(sc.act_a, sc.act_R)
    x = sc.X.copy()
    assert contact.constraint_set(x, prob.prox, prob.dhat).size == 0
    dx = np.zeros_like(x)
    low_face_of_upper = np.isclose(sc.X[:, 2], 0.01 + 1e-3)
    dx[low_face_of_upper, 2] = -8.5e-4               # gap 1 mm -> 0.15 mm
    alpha_m, spt, see = ccd.step_bound(x, dx, prob.prox, prob.dhat)
    assert alpha_m == 1.0                            # 0.15 mm is above the CCD target 0.1 mm
    F0 = local.deformation_gradients(x, prob.tets, prob.B)
    F1 = local.deformation_gradients(x + dx, prob.tets, prob.B)
    dE_elastic = local.element_energies(F1, A, prob.w).sum() - local.element_energies(F0, A, prob.w).sum()
    assert dE_elastic < 0
    assert _total_energy(prob, x + dx, A) > _total_energy(prob, x, A)
    alpha, halvings, ok = solver.line_search(prob, x, dx, A, alpha_m, spt, see)
    assert ok and halvings >= 1 and alpha < alpha_m
    assert _total_energy(prob, x + alpha * dx, A) <= _total_energy(prob, x, A)


# --------------------------------------------------------------------------
# IPC refinements: squared-distance barrier (form 1) and adaptive stiffness
# --------------------------------------------------------------------------
def _c0(D):
    """b(D) = -(D - Dh)^2 ln(D / Dh) and its D-derivatives, written out."""
    Dh = DHAT * DHAT
    return -((D - Dh) ** 2) * np.log(D / Dh)


def _c1(D):
    Dh = DHAT * DHAT
    return -2 * (D - Dh) * np.log(D / Dh) - (D - Dh) ** 2 / D


def _c2(D):
    Dh = DHAT * DHAT
    return -2 * np.log(D / Dh) - 4 * (D - Dh) / D + (D - Dh) ** 2 / D ** 2


def test_squared_barrier_vanishes_smoothly_and_selects_the_same_pairs():
    Dh = DHAT * DHAT
    assert barrier.barrier(np.array([DHAT, 2 * DHAT]), DHAT, form=1).max() == 0
    assert np.isclose(_c1(Dh), 0) and np.isclose(_c2(Dh), 0)
    d = np.array([1e-6, 1e-4, 4.9e-4])
    assert np.all(barrier.barrier(d, DHAT, form=1) > 0)
    assert np.allclose(barrier.barrier(d, DHAT, form=1), _c0(d * d), rtol=1e-13)
    # the written-out derivatives against central differences of b(D)
    for D in (1e-9, 1e-8, 1e-7):
        h = 1e-4 * D
        assert np.isclose((_c0(D + h) - _c0(D - h)) / (2 * h), _c1(D), rtol=1e-6)
        assert np.isclose((_c1(D + h) - _c1(D - h)) / (2 * h), _c2(D), rtol=1e-6)


def test_squared_barrier_single_point_triangle_closed_form():
    """Point at height h over a triangle interior, D = h^2: grad_p =
    kappa b'(D) 2 h n, Hess_pp = kappa (4 h^2 b''(D) + 2 b'(D)) n n^T."""
    h = 2e-4
    D = h * h
    tri = np.array([[0, 0, 0], [0.01, 0, 0], [0, 0.01, 0.0]])
    X4 = np.concatenate([np.array([[0.002, 0.003, h]]), tri])[None]
    d2, kind, idx = geo.point_triangle(X4[:, 0], X4[:, 1], X4[:, 2], X4[:, 3])
    E, G, H = barrier.pair_derivatives(X4, kind, idx, DHAT, KAPPA, form=1)
    n = np.array([0, 0, 1.0])
    assert np.isclose(E[0], KAPPA * _c0(D), rtol=1e-12)
    assert np.allclose(G[0, :3], KAPPA * _c1(D) * 2 * h * n, rtol=1e-10)
    assert np.allclose(G[0].reshape(4, 3).sum(axis=0), 0, atol=1e-9 * np.abs(G).max())
    Hnn = KAPPA * (4 * D * _c2(D) + 2 * _c1(D))
    assert np.allclose(H[0, :3, :3], Hnn * np.outer(n, n), rtol=1e-9, atol=1e-9 * abs(Hnn))


@pytest.mark.parametrize("is_pt", [True, False])
def test_squared_barrier_gradient_against_finite_differences(is_pt):
    rng = np.random.default_rng(21 if is_pt else 22)
    checked = 0
    while checked < 4:
        base = rng.uniform(-0.005, 0.005, (3, 3))
        if is_pt:
            nrm = np.cross(base[1] - base[0], base[2] - base[0])
            p = base.mean(axis=0) + nrm / np.linalg.norm(nrm) * rng.uniform(1e-4, 4e-4)
            X4 = np.concatenate([p[None], base])[None]
            f = geo.point_triangle
        else:
            mid = 0.5 * (base[0] + base[1])
            dirb, off = rng.standard_normal(3), rng.standard_normal(3)
            dirb /= np.linalg.norm(dirb)
            off /= np.linalg.norm(off)
            X4 = np.stack([base[0], base[1], mid + 3e-4 * off - 0.004 * dirb, mid + 3e-4 * off + 0.004 * dirb])[None]
            f = geo.edge_edge
        d2, kind, idx = f(X4[:, 0], X4[:, 1], X4[:, 2], X4[:, 3])
        if not (5e-5 < np.sqrt(d2[0]) < 4.5e-4):
            continue
        _, G, _ = barrier.pair_derivatives(X4, kind, idx, DHAT, KAPPA, form=1)

        def energy(y):
            Y = y.reshape(1, 4, 3)
            return KAPPA * _c0(f(Y[:, 0], Y[:, 1], Y[:, 2], Y[:, 3])[0][0])
        x = X4.reshape(-1)
        eps = 1e-9
        g_fd = np.array([(energy(x + eps * e) - energy(x - eps * e)) / (2 * eps) for e in np.eye(12)])
        assert np.allclose(G[0], g_fd, rtol=2e-4, atol=2e-4 * np.abs(G[0]).max())
        checked += 1


def _pressed_slabs(depth, seed=0, amp=5e-5, kappa=None):
    sc = mg.slabs(0, nx=4, ny=4, nz=2, gap=1e-3)
    if kappa is not None:
        sc.kappa = kappa
    x = sc.X.copy()
    top = sc.X[:, 2].max()
    x[sc.X[:, 2] > 0.5 * top, 2] -= depth
    rng = np.random.default_rng(seed)
    x += rng.uniform(-amp, amp, x.shape) * (sc.dirichlet[:, None] == 0)
    return sc, x


def test_balanced_kappa_minimises_the_gradient_residual():
    """The frame-start stiffness is the minimiser of |g_E + k g_b| over k in
    [kappa_0, 100 kappa_0]: checked against a dense scan of k (a soft kappa_0
    so that the minimiser lies inside the interval)."""
    sc, x = _pressed_slabs(9.5e-4, seed=3, kappa=0.01)
    prob = solver.setup_scene(sc, kappa_adapt=True)
    A = fem.actuation_matrices(sc.act_a, sc.act_R)
    cs = contact.constraint_set(x, prob.prox, prob.dhat)
    assert cs.size > 0
    k_star = solver.balanced_kappa(prob, x, A, cs)
    F = local.deformation_gradients(x, prob.tets, prob.B)
    _, P = local.projections(F, A)
    gE = solver.pd_gradient(prob, F, P)[prob.free]
    gb = solver.barrier_terms(prob, x, cs, kappa=1.0)[1][prob.free]
    ks = np.linspace(prob.kappa, 100 * prob.kappa, 100001)
    k_scan = ks[int(np.argmin([np.linalg.norm(gE + k * gb) for k in ks]))]
    assert prob.kappa < k_star < 100 * prob.kappa
    assert abs(k_star - k_scan) <= ks[1] - ks[0]


def test_adaptive_kappa_follows_its_rule_and_stays_fixed_without_contact():
    """Without pairs the stiffness stays kappa_0; from a pressed state with a
    soft kappa_0 it starts at the balanced value and doubles exactly at the
    iterations whose smallest squared distance falls below 1e-9 l^2 and
    below the previous one (at least once here)."""
    sc = mg.slabs(0, nx=4, ny=4, nz=2, gap=0.02)
    prob = solver.setup_scene(sc, kappa_adapt=True)
    A = fem.actuation_matrices(0.3 * sc.act_a, sc.act_R)
    r = solver.frame(prob, sc.X, A, iters=5)
    assert r.kappa == [prob.kappa] * 5
    sc, x = _pressed_slabs(9.5e-4, seed=3, kappa=0.01)
    prob = solver.setup_scene(sc, kappa_adapt=True)
    A = fem.actuation_matrices(sc.act_a, sc.act_R)
    r = solver.frame(prob, x, A, iters=10, trace=True)
    eps = 1e-9 * float(np.sum((prob.X.max(0) - prob.X.min(0)) ** 2))
    k0 = solver.balanced_kappa(prob, x, A, contact.constraint_set(x, prob.prox, prob.dhat))
    assert r.kappa[0] == k0 and k0 > prob.kappa
    d2 = [float(rec.cs.d2.min()) if rec.cs.size else np.inf for rec in r.trace]
    doublings = 0
    for k in range(1, len(r.kappa)):
        doubled = d2[k] < eps and d2[k] < d2[k - 1]
        expect = min(2 * r.kappa[k - 1], 100 * prob.kappa) if doubled else r.kappa[k - 1]
        assert r.kappa[k] == expect, (k, d2[k], r.kappa)
        assert r.trace[k].kappa == r.kappa[k]
        doublings += doubled
    assert doublings >= 1
    # with the stiffness fixed between doublings the total energy still
    # decreases at every accepted step
    for k in range(len(r.trace) - 1):
        if r.kappa[k + 1] == r.kappa[k]:
            e0 = _energy_at_kappa(prob, r.trace[k].x, A, r.kappa[k])
            e1 = _energy_at_kappa(prob, r.trace[k + 1].x, A, r.kappa[k])
            assert e1 <= e0 + 1e-12 * abs(e0)


def _energy_at_kappa(prob, x, A, kappa):
    F = local.deformation_gradients(x, prob.tets, prob.B)
    Ee = local.element_energies(F, A, prob.w)
    cs = contact.constraint_set(x, prob.prox, prob.dhat)
    return float(Ee.sum()) + kappa * float(barrier.barrier(np.sqrt(cs.d2), prob.dhat, prob.barrier_form).sum())


# --------------------------------------------------------------------------
# embedded proxy s = W x (Section 3.1)
# --------------------------------------------------------------------------
def _selection_embedding(sc):
    """The scene's own proxy written as an explicit selection W (one weight
    of 1 per row) with triangles over proxy vertex ids."""
    verts = np.unique(sc.surf_tris.reshape(-1))
    vmap = np.full(sc.n, -1)
    vmap[verts] = np.arange(verts.size)
    rowptr = np.arange(verts.size + 1, dtype=np.int32)
    return vmap[sc.surf_tris].astype(np.int32), (rowptr, verts.astype(np.int32), np.ones(verts.size))


def _pressed(sc, depth, seed=1, amp=5e-5):
    x = sc.X.copy()
    top = sc.X[:, 2].max()
    x[sc.X[:, 2] > 0.5 * top, 2] -= depth
    rng = np.random.default_rng(seed)
    x += rng.uniform(-amp, amp, x.shape) * (sc.dirichlet[:, None] == 0)
    return x


def test_selection_embedding_equals_the_plain_proxy():
    """W = an explicit selection reproduces the plain proxy's iteration and
    frame bit for bit."""
    sc = mg.slabs(0, nx=4, ny=4, nz=1, gap=1e-3)
    tris, W = _selection_embedding(sc)
    p0 = solver.setup_scene(sc)
    p1 = solver.setup(sc.X, sc.tets, sc.dirichlet, tris, sc.youngs, sc.poisson, sc.dhat, sc.kappa, W=W)
    x = _pressed(sc, 8e-4)
    A = fem.actuation_matrices(0.4 * sc.act_a, sc.act_R)
    x0, r0, _ = solver.iteration(p0, x, A)
    x1, r1, _ = solver.iteration(p1, x, A)
    assert r0.cs.size > 0 and r1.cs.size == r0.cs.size
    assert np.array_equal(r0.dx, r1.dx) and r0.alpha == r1.alpha and np.array_equal(x0, x1)
    assert np.array_equal(solver.affected_vertices(p0, r0.cs), solver.affected_vertices(p1, r1.cs))


def test_embedded_barrier_gradient_against_finite_differences():
    """With the refined proxy (edge midpoints interpolate two vertices), the
    barrier gradient over simulation DOFs equals central differences of
    kappa sum_k b(d_k(W x)) with the pair set held fixed."""
    sc = mg.refine_proxy(mg.slabs(0, nx=3, ny=3, nz=1, gap=1e-3))
    prob = solver.setup_scene(sc)
    x = _pressed(sc, 7e-4, seed=2)
    s = solver.proxy_positions(prob, x)
    cs = contact.constraint_set(s, prob.prox, prob.dhat)
    assert cs.size > 20
    E, g, Bm, _ = solver.barrier_terms(prob, x, cs)

    def energy(y):
        d2, _, _ = contact.pair_distances(prob.W @ y, prob.prox, cs.pt, cs.ee)
        return prob.kappa * barrier.barrier(np.sqrt(d2), prob.dhat).sum()
    assert np.isclose(E, energy(x), rtol=1e-12)
    rng = np.random.default_rng(4)
    moved = np.unique(prob.W[np.unique(contact.pair_vertices(prob.prox, cs.pt, cs.ee))].indices)
    for v in rng.choice(moved, 6, replace=False):
        for r in range(3):
            e = np.zeros_like(x)
            e[v, r] = 1e-9
            fd = (energy(x + e) - energy(x - e)) / 2e-9
            assert np.isclose(g[3 * v + r], fd, rtol=1e-4, atol=1e-6 * np.abs(g).max()), (v, r)
    # the projected Hessian is symmetric PSD over the simulation DOFs
    Bd = Bm.toarray()[np.ix_(prob.free, prob.free)]
    assert np.allclose(Bd, Bd.T, atol=1e-12 * np.abs(Bd).max())
    assert np.linalg.eigvalsh(Bd).min() >= -1e-9 * np.abs(Bd).max()


def test_embedded_frames_stay_intersection_free_and_energy_decreases():
    sc = mg.refine_proxy(mg.slabs(0, nx=3, ny=3, nz=1, gap=1e-3))
    prob = solver.setup_scene(sc)
    x = sc.X.copy()
    for t in (0.5, 1.0):
        A = fem.actuation_matrices(t * sc.act_a, sc.act_R)
        r = solver.frame(prob, x, A, iters=8, trace=True)

        def total(y):
            F = local.deformation_gradients(y, prob.tets, prob.B)
            s = solver.proxy_positions(prob, y)
            cs = contact.constraint_set(s, prob.prox, prob.dhat)
            return float(local.element_energies(F, A, prob.w).sum()) + \
                prob.kappa * float(barrier.barrier(np.sqrt(cs.d2), prob.dhat).sum())
        E = [total(rec.x) for rec in r.trace] + [total(r.x)]
        assert all(E[k + 1] <= E[k] + 1e-14 * abs(E[k]) for k in range(len(E) - 1)), E
        x = r.x
        assert contact.min_distance(solver.proxy_positions(prob, x), prob.prox) > 0
    assert max(r.n_pt) > 0
    # the contact set on the proxy reaches vertices that only the midpoints touch
    assert max(r.n_c) > 0
