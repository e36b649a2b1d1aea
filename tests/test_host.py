"""CPU tests of the library's host logic and its C ABI surface (no GPU)."""
import re
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import meshgen as mg
from oracle import solver as osolver

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib_or_skip():
    from paper_2312_02999_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libpdipc.so not built")
    return _lib


def test_library_exports_every_header_symbol():
    _lib = _lib_or_skip()
    L = _lib.lib()
    header = open(os.path.join(ROOT, "include", "pdipc.h")).read()
    names = set(re.findall(r"\b(pdipc_[a-z_]+)\s*\(", header))
    assert names, "no declarations parsed"
    for nm in sorted(names):
        assert hasattr(L, nm), nm
    assert set(_lib.EXPORTS) == names


def test_single_hip_runtime_in_process():
    _lib = _lib_or_skip()
    _lib.lib()
    assert len(_lib.hip_runtimes_loaded()) == 1, _lib.hip_runtimes_loaded()


def _scalar_split(sc):
    """Scalar PD matrix over free vertices in [x1, x2] order (from the oracle's H)."""
    prob = osolver.setup_scene(sc)
    Hs = prob.H.tocsr()[0::3, 0::3].tocsc()
    free = np.nonzero(sc.dirichlet == 0)[0]
    in2 = sc.region[free] == 1
    x1, x2 = free[~in2], free[in2]
    order = np.concatenate([x1, x2])
    Hf = Hs[order][:, order].tocsr()
    Hf.sort_indices()
    return Hf, x1, x2


@pytest.mark.parametrize("leaf", [8, 32, 96])
def test_host_factor_solves_pd_system_and_schur(leaf):
    from paper_2312_02999_amd import host_factor_solve
    _lib_or_skip()
    sc = mg.slabs(0, nx=6, ny=5, nz=3)
    Hf, x1, x2 = _scalar_split(sc)
    n1, n2 = len(x1), len(x2)
    b = np.random.default_rng(0).standard_normal(n1 + n2)
    x, sig, nnz = host_factor_solve(n1, n2, sc.X[x1], Hf.indptr, Hf.indices, Hf.data, b, leaf=leaf)
    ref = spla.spsolve(Hf.tocsc(), b)
    assert np.allclose(x, ref, rtol=1e-11, atol=1e-12 * np.abs(ref).max())
    H = Hf.toarray()
    S = H[n1:, n1:] - H[n1:, :n1] @ np.linalg.solve(H[:n1, :n1], H[:n1, n1:])
    assert np.allclose(sig, S, rtol=1e-11, atol=1e-11 * np.abs(S).max())
    assert nnz > 0


def test_host_factor_face_like_mesh():
    from paper_2312_02999_amd import host_factor_solve
    _lib_or_skip()
    sc = mg.face_like(14, 14, 3, seed=0, slits=(("mouth", 0.0, -0.35, 0.05),), region_radius=0.03)
    Hf, x1, x2 = _scalar_split(sc)
    n1, n2 = len(x1), len(x2)
    b = np.random.default_rng(1).standard_normal(n1 + n2)
    x, sig, _ = host_factor_solve(n1, n2, sc.X[x1], Hf.indptr, Hf.indices, Hf.data, b)
    ref = spla.spsolve(Hf.tocsc(), b)
    assert np.allclose(x, ref, rtol=1e-10, atol=1e-11 * np.abs(ref).max())


def test_host_factor_rejects_singular_matrix():
    from paper_2312_02999_amd import host_factor_solve, PdipcError
    _lib_or_skip()
    # graph Laplacian of a path (no fixed vertex): singular
    n = 20
    L = sp.diags([-np.ones(n - 1), np.r_[1, 2 * np.ones(n - 2), 1], -np.ones(n - 1)], [-1, 0, 1]).tocsr()
    L.sort_indices()
    coords = np.stack([np.arange(n), np.zeros(n), np.zeros(n)], axis=1).astype(float)
    with pytest.raises(PdipcError):
        host_factor_solve(n, 0, coords, L.indptr, L.indices, L.data, np.ones(n), leaf=8)
