"""Seeded synthetic scenes for the actuated PD+IPC solver.

This module only *describes inputs*: rest meshes, fixed vertices, the marked
collision region, the collision proxy (boundary triangles, embedded by
selection) and per-tet actuation parameters.  It holds none of the solver's
arithmetic; the solver library and the CPU oracle both consume what it makes.

The paper's own data (three facial sequences, face meshes and a neural
actuation model, Section 4) is not available, so these generators stand in for
it with matched scale:

* ``slabs``      two stacked 12x12x3-hex slabs ("lips") 1 mm apart.
* ``face_like``  a half-ellipsoidal shell with slot slits (mouth, eyelids).

Actuation follows the shape-targeting model of Eq. (1): each tet gets a scalar
strength ``a_i`` and a rotation ``R_i``; the symmetric target is
``R_i diag(1-a, 1+a/2, 1+a/2) R_i^T`` (built by the consumers, not here).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

__all__ = [
    "Scene", "hex_grid_tets", "boundary_faces", "unique_edges",
    "random_rotations", "slabs", "face_like", "ramp", "keyframe_sequence", "refine_proxy",
    "scene_by_name", "closed_slit_state",
]


@dataclass
class Scene:
    """A rest mesh plus everything a frame solve needs besides the state.

    Attributes (n vertices, m tets, F proxy triangles):
      X         (n,3) f64  rest positions [m]
      tets      (m,4) i32  positively oriented tetrahedra
      dirichlet (n,)  u8   1 = fixed at its rest position
      region    (n,)  u8   1 = collision-aware vertex (the x2 block)
      surf_tris (F,3) i32  proxy triangles, as simulation vertex ids (or, with
                           W, as proxy vertex ids: rows of W)
      act_a     (m,)  f64  actuation strength at full ramp
      act_R     (m,3,3) f64 actuation frame per tet (det +1)
    """
    name: str
    X: np.ndarray
    tets: np.ndarray
    dirichlet: np.ndarray
    region: np.ndarray
    surf_tris: np.ndarray
    act_a: np.ndarray
    act_R: np.ndarray
    youngs: float = 1.0e4
    poisson: float = 0.45
    dhat: float = 5.0e-4
    kappa: float = 1.0e3
    iters: int = 30
    frames: int = 5
    meta: dict = field(default_factory=dict)
    W: tuple | None = None      # proxy embedding s = W x as CSR (rowptr, col, val); None: selection

    @property
    def n(self) -> int:
        return int(self.X.shape[0])

    @property
    def m(self) -> int:
        return int(self.tets.shape[0])

    def proxy_vertices(self) -> np.ndarray:
        """Sorted simulation ids of the vertices used by proxy triangles."""
        return np.unique(self.surf_tris.reshape(-1)).astype(np.int32)

    def actuation_at(self, t: float) -> np.ndarray:
        """Strength field at ramp fraction t in [0, 1]."""
        return (float(t) * self.act_a).astype(np.float64)

    def sequence(self) -> list:
        """Per-frame strength fields of the scene's animation: from rest
        through its keyframe fields (piecewise linear, ``frames`` frames in
        all, spread evenly over the segments), or the plain ramp of ``act_a``
        when it has no keyframes."""
        keys = self.meta.get("keyframes") or []
        if not keys:
            return [self.actuation_at((t + 1) / self.frames) for t in range(self.frames)]
        fields = [np.zeros_like(self.act_a)] + list(keys)
        bounds = np.linspace(0, self.frames, len(fields)).round().astype(int)
        seq = []
        for k in range(len(fields) - 1):
            n_seg = bounds[k + 1] - bounds[k]
            for s in range(n_seg):
                w = (s + 1) / n_seg
                seq.append((1 - w) * fields[k] + w * fields[k + 1])
        return seq


# --------------------------------------------------------------------------
# structured hex grid -> conforming tets (Kuhn / Freudenthal split)
# --------------------------------------------------------------------------
_KUHN_PATHS = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]


def hex_grid_tets(ni: int, nj: int, nk: int, keep: np.ndarray | None = None) -> np.ndarray:
    """Split an ni x nj x nk hex grid into 6 tets per hex.

    Vertex (i, j, k) has id ``i + (ni+1) * (j + (nj+1) * k)``.  Every hex uses
    the same main diagonal (corner 000 to corner 111), which makes the split
    conforming across shared faces.  ``keep[i, j, k]`` (optional) drops hexes.
    Orientation is not fixed here; ``orient_tets`` does that from positions.
    """
    if keep is None:
        keep = np.ones((ni, nj, nk), dtype=bool)
    ii, jj, kk = np.nonzero(keep)
    nvi, nvj = ni + 1, nj + 1

    def vid(di, dj, dk):
        return (ii + di) + nvi * ((jj + dj) + nvj * (kk + dk))

    out = []
    for path in _KUHN_PATHS:
        corner = [0, 0, 0]
        verts = [vid(0, 0, 0)]
        for axis in path:
            corner[axis] = 1
            verts.append(vid(*corner))
        out.append(np.stack(verts, axis=1))
    return np.concatenate(out, axis=0).astype(np.int64)


def orient_tets(X: np.ndarray, tets: np.ndarray) -> np.ndarray:
    """Swap two vertices of every tet whose signed volume is negative."""
    t = tets.copy()
    e1 = X[t[:, 1]] - X[t[:, 0]]
    e2 = X[t[:, 2]] - X[t[:, 0]]
    e3 = X[t[:, 3]] - X[t[:, 0]]
    det = np.einsum("ij,ij->i", np.cross(e1, e2), e3)
    neg = det < 0
    t[neg, 2], t[neg, 3] = tets[neg, 3], tets[neg, 2]
    return t


def compact_vertices(X: np.ndarray, tets: np.ndarray):
    """Drop vertices no tet uses; return (X', tets', old_to_new)."""
    used = np.zeros(X.shape[0], dtype=bool)
    used[tets.reshape(-1)] = True
    old_to_new = -np.ones(X.shape[0], dtype=np.int64)
    old_to_new[used] = np.arange(int(used.sum()))
    return X[used], old_to_new[tets], old_to_new


def boundary_faces(tets: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Faces that belong to exactly one tet, with the owning tet index."""
    loc = np.array([[1, 2, 3], [0, 3, 2], [0, 1, 3], [0, 2, 1]])
    faces = tets[:, loc].reshape(-1, 3)
    owner = np.repeat(np.arange(tets.shape[0]), 4)
    key = np.sort(faces, axis=1)
    _, inv, cnt = np.unique(key, axis=0, return_inverse=True, return_counts=True)
    inv = inv.reshape(-1)
    single = cnt[inv] == 1
    return faces[single].astype(np.int64), owner[single]


def unique_edges(tris: np.ndarray) -> np.ndarray:
    """Sorted unique undirected edges (lo, hi) of a triangle list."""
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]], axis=0)
    e = np.sort(e, axis=1)
    return np.unique(e, axis=0)


def random_rotations(rng: np.random.Generator, count: int) -> np.ndarray:
    """Uniform random rotations from normalised Gaussian quaternions."""
    q = rng.standard_normal((count, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.empty((count, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - w * z)
    R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y)
    R[:, 2, 1] = 2 * (y * z + w * x)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


# --------------------------------------------------------------------------
# C1: two stacked slabs
# --------------------------------------------------------------------------
def slabs(seed: int = 0, nx: int = 12, ny: int = 12, nz: int = 3, h: float = 0.01,
          gap: float = 1.0e-3, a_max: float = 0.3, frames: int = 5, iters: int = 30,
          global_frame: bool = True) -> Scene:
    """Two slabs of nx*ny*nz hexes of edge h, the upper one ``gap`` above.

    Back faces (z = 0 and the top) are fixed.  The proxy is the pair of facing
    surfaces (lower slab top, upper slab bottom), embedded by selection; the
    collision-aware region is their vertices.  Actuation strengths are
    a_i ~ U[0, a_max].  With ``global_frame`` one seeded rotation, whose first
    axis lies in the xy-plane, is shared by all tets, so both slabs thicken
    toward the gap; otherwise every tet draws its own uniform rotation.
    """
    rng = np.random.default_rng(seed)
    nvx, nvy, nvz = nx + 1, ny + 1, nz + 1
    gi, gj, gk = np.meshgrid(np.arange(nvx), np.arange(nvy), np.arange(nvz), indexing="ij")
    # id = i + nvx*(j + nvy*k): flatten with k slowest
    P = np.stack([gi.transpose(2, 1, 0).reshape(-1), gj.transpose(2, 1, 0).reshape(-1),
                  gk.transpose(2, 1, 0).reshape(-1)], axis=1).astype(np.float64) * h
    T = hex_grid_tets(nx, ny, nz)
    nv = P.shape[0]
    Xl = P.copy()
    Xu = P.copy()
    Xu[:, 2] += nz * h + gap
    X = np.concatenate([Xl, Xu], axis=0)
    tets = np.concatenate([T, T + nv], axis=0)
    tets = orient_tets(X, tets)
    top = nz * h
    z = X[:, 2]
    dirichlet = (np.isclose(z, 0.0) | np.isclose(z, 2 * top + gap)).astype(np.uint8)
    faces, _ = boundary_faces(tets)
    fz = X[faces][:, :, 2]
    lower_top = np.all(np.isclose(fz, top), axis=1)
    upper_bot = np.all(np.isclose(fz, top + gap), axis=1)
    surf = faces[lower_top | upper_bot].astype(np.int32)
    region = np.zeros(X.shape[0], dtype=np.uint8)
    region[np.unique(surf)] = 1
    m = tets.shape[0]
    act_a = rng.uniform(0.0, a_max, size=m)
    if global_frame:
        phi = rng.uniform(0.0, 2 * np.pi)
        e1 = np.array([np.cos(phi), np.sin(phi), 0.0])
        e3 = np.array([0.0, 0.0, 1.0])
        e2 = np.cross(e3, e1)
        R0 = np.stack([e1, e2, e3], axis=1)
        act_R = np.broadcast_to(R0, (m, 3, 3)).copy()
    else:
        act_R = random_rotations(rng, m)
    return Scene(name=f"slabs_s{seed}", X=X, tets=tets.astype(np.int32),
                 dirichlet=dirichlet, region=region, surf_tris=surf,
                 act_a=act_a, act_R=act_R, frames=frames, iters=iters,
                 meta={"seed": seed, "h": h, "gap": gap})


# --------------------------------------------------------------------------
# C2/C3/C4/C5: face-like shell with slot slits
# --------------------------------------------------------------------------
def _ellipsoid_point(theta, phi, axes):
    a, b, c = axes
    return np.stack([a * np.sin(theta) * np.cos(phi), b * np.sin(phi),
                     c * np.cos(theta) * np.cos(phi)], axis=-1)


def _ellipsoid_normal(P, axes):
    a, b, c = axes
    n = np.stack([P[..., 0] / a ** 2, P[..., 1] / b ** 2, P[..., 2] / c ** 2], axis=-1)
    return n / np.linalg.norm(n, axis=-1, keepdims=True)


def graded_nodes(lo: float, hi: float, n: int, centers=(), ratio: float = 1.0, band: float = 1.0) -> np.ndarray:
    """n + 1 grid nodes on [lo, hi] whose spacing is ``ratio`` times finer
    near each of ``centers`` than far from them: node k sits where the
    integral of the density 1 + (ratio - 1) max_c exp(-((u - c) / band)^2)
    reaches k / n of its total.  ratio = 1 gives the uniform grid."""
    if ratio == 1.0 or not len(centers):
        return np.linspace(lo, hi, n + 1)
    u = np.linspace(lo, hi, 40001)
    bump = np.max([np.exp(-((u - c) / band) ** 2) for c in centers], axis=0)
    rho = 1.0 + (ratio - 1.0) * bump
    cum = np.concatenate([[0.0], np.cumsum(0.5 * (rho[1:] + rho[:-1]) * np.diff(u))])
    nodes = np.interp(np.linspace(0.0, cum[-1], n + 1), cum, u)
    nodes[0], nodes[-1] = lo, hi
    return nodes


def face_like(n_theta: int = 101, n_phi: int = 101, n_layers: int = 4, seed: int = 0,
              axes=(0.10, 0.12, 0.06), thickness: float = 0.02,
              theta_max: float = 1.2, phi_max: float = 1.2,
              slits=(("mouth", 0.0, -0.35, 0.06),), region_radius: float = 0.025,
              fix_radius: float = 0.03, n_bumps: int = 8, a_cap: float = 0.35,
              bump_height: float = 0.6, frames: int = 10, iters: int = 30,
              grade=(1.0, 1.0, 1.0, 1.0), keyframes: int = 0) -> Scene:
    """Half-ellipsoidal shell of n_theta x n_phi x n_layers hexes.

    The outer surface is the ellipsoid with semi-axes ``axes``; layers step
    inward along the outer normal to ``thickness``.  The (theta, phi) grid is
    graded toward the slits: ``grade = (ratio_theta, band_theta, ratio_phi,
    band_phi)`` makes cells ratio times finer within about band (radians) of
    the slit centres (see ``graded_nodes``).  Each slit
    (name, theta_c, phi_c, length) removes one row of hexes through the whole
    thickness over ``length`` of outer arc (the columns whose centres lie
    within length / 2 of the slit centre), leaving a slot of one cell height.
    ``keyframes`` > 0 adds that many further seeded strength fields (same
    bump recipe) to ``meta["keyframes"]`` for ``Scene.sequence``.
    Fixed vertices: the inner surface farther than ``fix_radius`` from every
    slit, plus the whole rim of the parameter domain.  The proxy is the
    boundary triangles of the tets whose centroid lies within
    ``region_radius`` of a slit; the collision-aware block x2 is the free
    vertices of those triangles (the vertices that embed the proxy).  Actuation: a sum of ``n_bumps`` Gaussian bumps per slit, capped at
    ``a_cap``, contracting along the local shell normal (so the skin grows
    in-plane and the slots close).
    """
    rng = np.random.default_rng(seed)
    nvt, nvp, nvl = n_theta + 1, n_phi + 1, n_layers + 1
    r_th, b_th, r_ph, b_ph = grade
    th = graded_nodes(-theta_max, theta_max, n_theta, [sl[1] for sl in slits], r_th, b_th)
    ph = graded_nodes(-phi_max, phi_max, n_phi, [sl[2] for sl in slits], r_ph, b_ph)
    # vertex (i, j, k): i along theta, j along phi, k through thickness
    TT, PP = np.meshgrid(th, ph, indexing="ij")          # (nvt, nvp)
    outer = _ellipsoid_point(TT, PP, axes)               # (nvt, nvp, 3)
    nrm = _ellipsoid_normal(outer, axes)
    depth = np.linspace(0.0, thickness, nvl)
    V = outer[:, :, None, :] - depth[None, None, :, None] * nrm[:, :, None, :]
    # ids i + nvt*(j + nvp*k)  ->  reorder to (k, j, i)
    X = V.transpose(2, 1, 0, 3).reshape(-1, 3)
    keep = np.ones((n_theta, n_phi, n_layers), dtype=bool)
    slit_info = []
    for name, th_c, ph_c, length in slits:
        jrow = int(np.argmin(np.abs(0.5 * (ph[:-1] + ph[1:]) - ph_c)))
        # outer arc length along theta at this latitude; columns whose centre
        # lies within length / 2 of the slit centre are removed
        phi_mid = 0.5 * (ph[jrow] + ph[jrow + 1])
        P = _ellipsoid_point(th, np.full_like(th, phi_mid), axes)
        arc = np.concatenate([[0.0], np.cumsum(np.linalg.norm(np.diff(P, axis=0), axis=1))])
        mid = 0.5 * (arc[1:] + arc[:-1])
        s_c = float(np.interp(th_c, th, arc))
        cols = np.nonzero(np.abs(mid - s_c) < 0.5 * length)[0]
        cols = cols[(cols >= 1) & (cols <= n_theta - 2)]
        if cols.size == 0:
            cols = np.array([int(np.argmin(np.abs(mid - s_c)))])
        i0, i1 = int(cols[0]), int(cols[-1]) + 1
        keep[i0:i1, jrow, :] = False
        a_pt = _ellipsoid_point(np.array(th[i0]), np.array(phi_mid), axes)
        b_pt = _ellipsoid_point(np.array(th[i1]), np.array(phi_mid), axes)
        slit_info.append({"name": name, "row": jrow, "cols": (i0, i1),
                          "a": a_pt, "b": b_pt})
    tets = hex_grid_tets(n_theta, n_phi, n_layers, keep)
    X, tets, _ = compact_vertices(X, tets)
    tets = orient_tets(X, tets)

    def dist_to_slits(P):
        d = np.full(P.shape[0], np.inf)
        for s in slit_info:
            a, b = s["a"], s["b"]
            ab = b - a
            t = np.clip(((P - a) @ ab) / (ab @ ab), 0.0, 1.0)
            q = a + t[:, None] * ab
            d = np.minimum(d, np.linalg.norm(P - q, axis=1))
        return d

    # parametric coordinates survive compaction through the vertex map
    full_ijk = np.stack(np.meshgrid(np.arange(nvt), np.arange(nvp), np.arange(nvl),
                                    indexing="ij"), axis=-1).transpose(2, 1, 0, 3).reshape(-1, 3)
    used = np.zeros(full_ijk.shape[0], dtype=bool)
    used[hex_grid_tets(n_theta, n_phi, n_layers, keep).reshape(-1)] = True
    ijk = full_ijk[used]
    # distances to a slit are lateral: measured from each vertex's counterpart
    # on the outer surface (layers step along the outer normal), so the whole
    # depth of a slit wall is as close to the slit as its outer edge
    Xo = outer[ijk[:, 0], ijk[:, 1]]
    dslit = dist_to_slits(Xo)
    inner = ijk[:, 2] == n_layers
    rim = (ijk[:, 0] == 0) | (ijk[:, 0] == n_theta) | (ijk[:, 1] == 0) | (ijk[:, 1] == n_phi)
    dirichlet = ((inner & (dslit > fix_radius)) | rim).astype(np.uint8)

    cent = X[tets].mean(axis=1)
    in_region = dist_to_slits(Xo[tets].mean(axis=1)) < region_radius
    faces, owner = boundary_faces(tets)
    surf = faces[in_region[owner]].astype(np.int32)
    # the collision-aware block x2: the free vertices that carry the proxy
    region = np.zeros(X.shape[0], dtype=np.uint8)
    region[np.unique(surf)] = 1
    region[dirichlet == 1] = 0

    # actuation: Gaussian bumps near each slit, contracting along the normal;
    # the scene's field and each keyframe field draw their own bumps
    m = tets.shape[0]

    def bump_field(g):
        act = np.zeros(m)
        for s in slit_info:
            mid = 0.5 * (s["a"] + s["b"])
            for _ in range(n_bumps):
                off = g.uniform(-1.0, 1.0, 3)
                off *= g.uniform(0.0, 0.04) / max(np.linalg.norm(off), 1e-12)
                mu = mid + off
                sig = g.uniform(0.01, 0.03)
                hgt = bump_height * g.uniform(0.5, 1.0)
                act += hgt * np.exp(-np.sum((cent - mu) ** 2, axis=1) / (2 * sig * sig))
        return np.minimum(a_cap, act)

    act_a = bump_field(rng)
    keys = [bump_field(np.random.default_rng([seed, 1000 + k])) for k in range(keyframes)]
    # local frame: first axis = outward shell normal at the tet centroid
    n_c = _ellipsoid_normal(cent * 0 + _project_to_outer(cent, axes), axes)
    up = np.where(np.abs(n_c[:, 1:2]) < 0.9, np.array([[0.0, 1.0, 0.0]]),
                  np.array([[1.0, 0.0, 0.0]]))
    t1 = np.cross(up, n_c)
    t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
    t2 = np.cross(n_c, t1)
    act_R = np.stack([n_c, t1, t2], axis=2)
    return Scene(name=f"face_{n_theta}x{n_phi}x{n_layers}_s{seed}", X=X,
                 tets=tets.astype(np.int32), dirichlet=dirichlet, region=region,
                 surf_tris=surf, act_a=act_a, act_R=act_R, frames=frames, iters=iters,
                 meta={"seed": seed, "slits": [(s["name"], s["row"], s["cols"]) for s in slit_info],
                       "ijk": ijk.astype(np.int32), "keyframes": keys})


def _project_to_outer(P, axes):
    """Radial projection of points onto the outer ellipsoid (for normals)."""
    a, b, c = axes
    s = np.sqrt((P[:, 0] / a) ** 2 + (P[:, 1] / b) ** 2 + (P[:, 2] / c) ** 2)
    return P / s[:, None]


def closed_slit_state(scene: Scene, gap: float, seed: int = 0, jitter: float = 0.0,
                      falloff_rows: int = 6) -> np.ndarray:
    """A contact state of a face-like scene made by moving material, not by
    solving: the upper wall of every slit is carried toward the lower wall
    until the walls are ``gap`` apart in the middle of the slit.

    For a vertex on grid row j >= row + 1 of a slit (row = the removed hex
    row) and on one of the slit's columns, the displacement is
    s(i) w(j) (1 - gap / h) (X(i, row, k) - X(i, row + 1, k)), with h the
    wall distance at that column and layer, s(i) a smooth bump that is 1 in the
    middle of the slit and 0 at its ends, and w(j) falling linearly from 1 on
    the wall to 0 ``falloff_rows`` rows above it.  Fixed vertices do not move.
    ``jitter`` adds a seeded uniform perturbation to the moved vertices.
    """
    ijk = scene.meta["ijk"]
    key = {tuple(v): q for q, v in enumerate(ijk.tolist())}
    x = scene.X.copy()
    rng = np.random.default_rng(seed)
    for _, row, (i0, i1) in scene.meta["slits"]:
        for q, (i, j, k) in enumerate(ijk.tolist()):
            if j < row + 1 or not (i0 <= i <= i1) or scene.dirichlet[q]:
                continue
            lo, up = key.get((i, row, k)), key.get((i, row + 1, k))
            if lo is None or up is None:
                continue
            d = scene.X[lo] - scene.X[up]
            h = float(np.linalg.norm(d))
            u = (i - i0) / max(i1 - i0, 1)
            s_i = np.sin(np.pi * u) ** 2
            w_j = max(0.0, 1.0 - (j - row - 1) / falloff_rows)
            x[q] += s_i * w_j * (1.0 - gap / h) * d
    if jitter > 0:
        moved = np.any(x != scene.X, axis=1)
        x[moved] += rng.uniform(-jitter, jitter, (int(moved.sum()), 3))
    return x


# --------------------------------------------------------------------------
# embedded collision proxy (Section 3.1: s = W x)
# --------------------------------------------------------------------------
def refine_proxy(scene: Scene) -> Scene:
    """The scene with a finer collision proxy embedded in its simulation
    surface: every proxy triangle is split into four at its edge midpoints.
    Proxy vertices are the original surface vertices (one weight of 1) and
    the edge midpoints (weights 1/2, 1/2), so each row of W interpolates the
    simulation vertices of one surface edge or vertex and sums to 1.
    ``W`` = (rowptr, col, val) is the n_s x n CSR of s = W x; the proxy
    triangles index proxy vertices (rows of W).  The collision-aware block
    is unchanged: the free simulation vertices that W touches."""
    tris = np.asarray(scene.surf_tris, dtype=np.int64)
    verts = np.unique(tris.reshape(-1))
    vmap = np.full(scene.n, -1, dtype=np.int64)
    vmap[verts] = np.arange(verts.size)
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]], axis=0)
    edges = np.unique(np.sort(e, axis=1), axis=0)
    eid = {(int(a), int(b)): verts.size + i for i, (a, b) in enumerate(edges)}

    def mid(a, b):
        return eid[(min(int(a), int(b)), max(int(a), int(b)))]

    new_tris = []
    for a, b, c in tris:
        A, B, Cc = vmap[a], vmap[b], vmap[c]
        ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
        new_tris += [(A, ab, ca), (ab, B, bc), (ca, bc, Cc), (ab, bc, ca)]
    ns = verts.size + edges.shape[0]
    rowptr = np.zeros(ns + 1, dtype=np.int32)
    rowptr[1:verts.size + 1] = 1
    rowptr[verts.size + 1:] = 2
    rowptr = np.cumsum(rowptr).astype(np.int32)
    col = np.concatenate([verts, edges.reshape(-1)]).astype(np.int32)
    val = np.concatenate([np.ones(verts.size), np.full(2 * edges.shape[0], 0.5)])
    out = Scene(name=scene.name + "_refined", X=scene.X, tets=scene.tets, dirichlet=scene.dirichlet,
                region=scene.region, surf_tris=np.asarray(new_tris, dtype=np.int32), act_a=scene.act_a,
                act_R=scene.act_R, frames=scene.frames, iters=scene.iters, youngs=scene.youngs,
                poisson=scene.poisson, dhat=scene.dhat, kappa=scene.kappa, meta=dict(scene.meta),
                W=(rowptr, col, val))
    return out


# --------------------------------------------------------------------------
# actuation sequences
# --------------------------------------------------------------------------
def ramp(scene: Scene, frames: int | None = None) -> list[np.ndarray]:
    """Linear ramp of the strength field over ``frames`` frames (t/T, t=1..T)."""
    T = scene.frames if frames is None else frames
    return [scene.actuation_at((t + 1) / T) for t in range(T)]


def keyframe_sequence(fields: list[np.ndarray], per_segment: int) -> list[np.ndarray]:
    """Piecewise-linear interpolation between keyframe strength fields."""
    seq = []
    for k in range(len(fields) - 1):
        for s in range(per_segment):
            w = (s + 1) / per_segment
            seq.append((1 - w) * fields[k] + w * fields[k + 1])
    return seq


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------
# Grading of the face-like grids toward the slits (cells 5x finer along the
# slit and 3x across it near the slit centres), and the number of layers
# through the 2 cm shell: together they put about 2% of the vertices on the
# slit walls of the 50k face, the contact level its workload calls for.
FACE_GRADE = (5.0, 0.3, 3.0, 0.2)
FACE_LAYERS = 10
# Peak bump height of the actuation fields (before the 0.35 cap), tuned once
# per workload so that the slits close; the values are frozen here.
FACE_BUMP = {"face5k": 0.6, "face20k": 0.6, "face50k": 0.6, "face100k": 0.6, "face250k": 0.6}
THREE_SLITS = (("mouth", 0.0, -0.35, 0.06), ("eye_l", -0.45, 0.35, 0.035), ("eye_r", 0.45, 0.35, 0.035))


def scene_by_name(name: str, seed: int = 0, bump_height: float | None = None) -> Scene:
    """Named workloads: 'slabs', 'tiny', 'face5k', 'face20k', 'face50k',
    'face100k', 'face250k'.

    face50k: 96 x 48 x 10 graded hexes (n = 52 283, m = 273 240), mouth slit,
    collision region within 3 cm of the slit (n2 = 3684 free proxy vertices),
    a 50-frame animation from rest through 4 keyframe fields, 30 iterations
    per frame.  face250k: 190 x 125 x 10 (n = 264 726), mouth and two eyelid
    slits, region within 1.2 cm (n2 = 12 096), 60 frames through 4 keyframes,
    40 iterations per frame.  face5k/20k/100k: the serving sizes, 10-frame
    ramps of one field.
    """
    if name == "slabs":
        return slabs(seed=seed)
    if name == "tiny":
        return slabs(seed=seed, nx=3, ny=3, nz=1, gap=1.0e-3, frames=3, iters=10)
    grids = {"face5k": (30, 14), "face20k": (60, 30), "face50k": (96, 48), "face100k": (136, 68),
             "face250k": (190, 125)}
    if name not in grids:
        raise KeyError(name)
    nt, nph = grids[name]
    h = FACE_BUMP[name] if bump_height is None else bump_height
    kw = dict(seed=seed, n_layers=FACE_LAYERS, grade=FACE_GRADE, region_radius=0.03, bump_height=h)
    if name == "face50k":
        kw.update(frames=50, keyframes=4)
    if name == "face250k":
        # region radius 1.2 cm keeps the dense inverse Schur complement at
        # n2 ~ 12k (1.2 GB)
        kw.update(iters=40, frames=60, keyframes=4, region_radius=0.012, slits=THREE_SLITS)
    return face_like(nt, nph, **kw)
