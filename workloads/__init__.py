"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests and
the benchmark: meshes, velocity-grid specifications and initial distributions.

This module holds none of the method's arithmetic (no moments, no equilibrium
solve, no FR operator).  It builds the *inputs* the method is applied to:

* hexahedral meshes in the layout of the C ABI (nodes, x-fastest element
  node lists, face neighbours / orientation codes / boundary tags);
* velocity-grid specifications ``{"n": (n,n,n), "umin": ..., "umax": ...}``;
* initial distributions f0 = Maxwellian sampled at every velocity node for a
  seeded macroscopic field (the paper initialises f as the equilibrium of a
  macroscopic state), evaluated with torch on the requested device.

The workloads stand in for the paper's capsule cases (whose mesh and data are
not available): periodic boxes at the paper's orders and velocity
resolutions, and an O-grid around a cylinder at Mach 8.
"""
from __future__ import annotations

import math

import numpy as np

SQRT_2_OVER_PI = math.sqrt(2.0 / math.pi)

# Face numbering: face = 2*d + side, side 0 at xi_d = -1, side 1 at xi_d = +1.
FACE_OPPOSITE = [1, 0, 3, 2, 5, 4]


def mu_ref_from_knudsen(kn: float) -> float:
    """Reference viscosity from a Knudsen number with unit length, density and
    temperature, through the mean free path lambda = (mu/rho) sqrt(pi/(2 theta))."""
    return kn * SQRT_2_OVER_PI


def box_mesh(N, length=1.0, periodic=True) -> dict:
    """Axis-aligned box [0,L]^3 of N[0] x N[1] x N[2] straight 8-node hexes.

    Element (ix,iy,iz) has id ix + N0 (iy + N1 iz).  With ``periodic`` every
    face has a neighbour (wrapping around), orientation code 0."""
    if np.isscalar(N):
        N = (int(N),) * 3
    N = tuple(int(v) for v in N)
    L = (length,) * 3 if np.isscalar(length) else tuple(length)
    nx, ny, nz = N
    gx = [np.linspace(0.0, L[d], N[d] + 1) for d in range(3)]
    nodes = np.stack(np.meshgrid(gx[0], gx[1], gx[2], indexing="ij"), axis=-1)
    nodes = nodes.transpose(2, 1, 0, 3).reshape(-1, 3)  # node id = i + (nx+1)(j + (ny+1) k)

    def nid(i, j, k):
        return i + (nx + 1) * (j + (ny + 1) * k)

    ne = nx * ny * nz
    en = np.zeros((ne, 8), np.int32)
    nbr = np.full((ne, 6), -1, np.int32)
    nbf = np.zeros((ne, 6), np.int8)
    bc = np.zeros((ne, 6), np.int8)
    for iz in range(nz):
        for iy in range(ny):
            for ix in range(nx):
                e = ix + nx * (iy + ny * iz)
                en[e] = [nid(ix + a, iy + b, iz + c) for c in (0, 1) for b in (0, 1) for a in (0, 1)]
                idx = [ix, iy, iz]
                for d in range(3):
                    for side in (0, 1):
                        f = 2 * d + side
                        j = list(idx)
                        j[d] += 1 if side else -1
                        if 0 <= j[d] < N[d] or periodic:
                            j[d] %= N[d]
                            nbr[e, f] = j[0] + nx * (j[1] + ny * j[2])
                            nbf[e, f] = FACE_OPPOSITE[f]
                        else:
                            bc[e, f] = 1
    return {"n_elem": ne, "n_nodes": nodes.shape[0], "geom_order": 1,
            "nodes": np.ascontiguousarray(nodes), "elem_nodes": en, "nbr_elem": nbr,
            "nbr_face": nbf, "nbr_orient": np.zeros((ne, 6), np.int8), "bc": bc,
            "N": N, "length": L}


def cylinder_mesh(n_theta=48, n_r=24, n_z=2, r0=0.5, r1=6.0, stretch=1.15, lz=0.25, half=False) -> dict:
    """O-grid of 27-node (quadratic) hexes around a cylinder of radius r0 with
    axis z: xi_0 radial (element widths growing by ``stretch`` from the wall
    to r1), xi_1 azimuthal (mid-edge nodes on the arcs, so the faces are
    curved), xi_2 spanwise over [0, lz] (periodic).  Element (i, j, k) has id
    i + n_r (j + n_theta k).  Inner faces: diffuse wall (bc 2); outer faces:
    farfield (bc 1).  ``half``: only the upper half (0 <= angle <= pi) with
    specular symmetry walls (bc 3) on the cut y = 0."""
    g = stretch ** np.arange(n_r)
    edges = r0 + (r1 - r0) * np.concatenate([[0.0], np.cumsum(g)]) / g.sum()
    radii = np.empty(2 * n_r + 1)
    radii[0::2] = edges
    radii[1::2] = 0.5 * (edges[:-1] + edges[1:])
    NR, NT, NZ = 2 * n_r + 1, 2 * n_theta + (1 if half else 0), 2 * n_z + 1
    th = (np.pi * np.arange(NT) / (NT - 1)) if half else (2 * np.pi * np.arange(NT) / NT)
    zz = lz * np.arange(NZ) / (NZ - 1)
    R, T, Z = np.meshgrid(radii, th, zz, indexing="ij")
    nodes = np.stack([R * np.cos(T), R * np.sin(T), Z], -1).transpose(2, 1, 0, 3).reshape(-1, 3)

    def nid(a, b, c):
        return a + NR * ((b % NT) + NT * c)

    ne = n_r * n_theta * n_z
    en = np.zeros((ne, 27), np.int32)
    nbr = np.full((ne, 6), -1, np.int32)
    nbf = np.zeros((ne, 6), np.int8)
    bc = np.zeros((ne, 6), np.int8)
    for k in range(n_z):
        for j in range(n_theta):
            for i in range(n_r):
                e = i + n_r * (j + n_theta * k)
                en[e] = [nid(2 * i + a, 2 * j + b, 2 * k + c) for c in range(3) for b in range(3) for a in range(3)]
                if i > 0:
                    nbr[e, 0] = e - 1
                else:
                    bc[e, 0] = 2
                if i < n_r - 1:
                    nbr[e, 1] = e + 1
                else:
                    bc[e, 1] = 1
                if half and j == 0:
                    bc[e, 2] = 3
                else:
                    nbr[e, 2] = i + n_r * ((j - 1) % n_theta + n_theta * k)
                if half and j == n_theta - 1:
                    bc[e, 3] = 3
                else:
                    nbr[e, 3] = i + n_r * ((j + 1) % n_theta + n_theta * k)
                nbr[e, 4] = i + n_r * (j + n_theta * ((k - 1) % n_z))
                nbr[e, 5] = i + n_r * (j + n_theta * ((k + 1) % n_z))
                for f in range(6):
                    if nbr[e, f] >= 0:
                        nbf[e, f] = FACE_OPPOSITE[f]
    return {"n_elem": ne, "n_nodes": nodes.shape[0], "geom_order": 2,
            "nodes": np.ascontiguousarray(nodes), "elem_nodes": en, "nbr_elem": nbr,
            "nbr_face": nbf, "nbr_orient": np.zeros((ne, 6), np.int8), "bc": bc,
            "r0": r0, "r1": r1, "lz": lz}


def quadratic_map_mesh(N, eps=0.15, bc_all=1) -> dict:
    """Non-periodic box [0,1]^3 of N^3 27-node hexes whose nodes are moved by
    the global quadratic map x -> x + eps (x_1^2, x_2^2, x_0^2); every element
    is then an exact quadratic image of a cube.  Every boundary face carries
    bc ``bc_all``."""
    if np.isscalar(N):
        N = (int(N),) * 3
    base = box_mesh(N, periodic=False)
    nx, ny, nz = N
    M = [2 * v + 1 for v in N]
    gx = [np.linspace(0.0, 1.0, m) for m in M]
    X = np.stack(np.meshgrid(gx[0], gx[1], gx[2], indexing="ij"), -1).transpose(2, 1, 0, 3).reshape(-1, 3)
    X = X + eps * np.stack([X[:, 1] ** 2, X[:, 2] ** 2, X[:, 0] ** 2], -1)
    ne = nx * ny * nz
    en = np.zeros((ne, 27), np.int32)
    for iz in range(nz):
        for iy in range(ny):
            for ix in range(nx):
                e = ix + nx * (iy + ny * iz)
                en[e] = [(2 * ix + a) + M[0] * ((2 * iy + b) + M[1] * (2 * iz + c))
                         for c in range(3) for b in range(3) for a in range(3)]
    bc = np.where(base["nbr_elem"] < 0, bc_all, 0).astype(np.int8)
    return {**base, "n_nodes": X.shape[0], "geom_order": 2, "nodes": np.ascontiguousarray(X),
            "elem_nodes": en, "bc": bc, "eps": eps}


def _signed_perms():
    import itertools
    out = []
    for perm in itertools.permutations(range(3)):
        for flips in itertools.product((0, 1), repeat=3):
            M = np.zeros((3, 3))
            for d in range(3):
                M[d, perm[d]] = -1.0 if flips[d] else 1.0
            if np.linalg.det(M) > 0:
                out.append((perm, flips))
    return out


def _orient_code(n, pairs):
    """Orientation code (bit0 swap, bit1 reverse first, bit2 reverse second)
    reproducing the face-point map pairs[(a, b)] = (pa, pb)."""
    for o in range(8):
        ok = True
        for (a, b), (pa, pb) in pairs.items():
            x, y = (b, a) if o & 1 else (a, b)
            if o & 2:
                x = n - 1 - x
            if o & 4:
                y = n - 1 - y
            ok = ok and (x, y) == (pa, pb)
        if ok:
            return o
    raise ValueError("no orientation code")


def reorient_elements(mesh: dict, seed: int = 0):
    """Give every element of a mesh built in one global frame (all faces
    orientation 0, neighbour across face f on its face f^1, 8-node elements)
    a random orientation-preserving local frame.  Returns (mesh, frames); the
    frame of element e is (perm, flips): new axis d runs along old axis
    perm[d], reversed if flips[d].  ``reindex_points`` maps per-element
    arrays of tensor points between the frames."""
    assert mesh["geom_order"] == 1
    rng = np.random.default_rng(seed)
    sp = _signed_perms()
    ne = mesh["n_elem"]
    frames = [sp[rng.integers(len(sp))] for _ in range(ne)]

    def old_index(fr, I, n):
        perm, flips = fr
        J = [0, 0, 0]
        for d in range(3):
            J[perm[d]] = n - 1 - I[d] if flips[d] else I[d]
        return J

    def new_index(fr, J, n):
        perm, flips = fr
        return [n - 1 - J[perm[d]] if flips[d] else J[perm[d]] for d in range(3)]

    en_old = mesh["elem_nodes"]
    en = np.zeros_like(en_old)
    for e in range(ne):
        for c in range(2):
            for b in range(2):
                for a in range(2):
                    J = old_index(frames[e], [a, b, c], 2)
                    en[e, a + 2 * (b + 2 * c)] = en_old[e, J[0] + 2 * (J[1] + 2 * J[2])]
    nbr = np.full((ne, 6), -1, np.int32)
    nbf = np.zeros((ne, 6), np.int8)
    nor = np.zeros((ne, 6), np.int8)
    bc = np.zeros((ne, 6), np.int8)
    n = 3  # face-point maps are independent of n; 3 points tell every code apart
    for e in range(ne):
        perm, flips = frames[e]
        for f in range(6):
            d, s = divmod(f, 2)
            g = 2 * perm[d] + (s ^ flips[d])
            nb = mesh["nbr_elem"][e, g]
            if nb < 0:
                bc[e, f] = mesh["bc"][e, g]
                continue
            t = [x for x in range(3) if x != d]
            pairs = {}
            nf_new = None
            for bb in range(n):
                for aa in range(n):
                    I = [0, 0, 0]
                    I[d] = s * (n - 1)
                    I[t[0]], I[t[1]] = aa, bb
                    J = old_index(frames[e], I, n)
                    J[perm[d]] = n - 1 - J[perm[d]]
                    K = new_index(frames[nb], J, n)
                    pn, fn = frames[nb]
                    dn = pn.index(perm[d])
                    sn = (1 if J[perm[d]] == n - 1 else 0)
                    sn_new = sn ^ fn[dn]
                    nf_new = 2 * dn + sn_new
                    tn = [x for x in range(3) if x != dn]
                    pairs[(aa, bb)] = (K[tn[0]], K[tn[1]])
            nbr[e, f] = nb
            nbf[e, f] = nf_new
            nor[e, f] = _orient_code(n, pairs)
    out = {**mesh, "elem_nodes": en, "nbr_elem": nbr, "nbr_face": nbf, "nbr_orient": nor, "bc": bc}
    return out, frames


def reindex_points(a: np.ndarray, frames, p: int, to_new: bool = True) -> np.ndarray:
    """Reorder axis 1 (the (p+1)^3 tensor points, x-fastest) of a per-element
    array between the global frame and the frames of ``reorient_elements``."""
    n = p + 1
    out = np.empty_like(a)
    for e, (perm, flips) in enumerate(frames):
        for c in range(n):
            for b in range(n):
                for q in range(n):
                    I = [q, b, c]
                    J = [0, 0, 0]
                    for d in range(3):
                        J[perm[d]] = n - 1 - I[d] if flips[d] else I[d]
                    sn = q + n * (b + n * c)
                    so = J[0] + n * (J[1] + n * J[2])
                    if to_new:
                        out[e, sn] = a[e, so]
                    else:
                        out[e, so] = a[e, sn]
    return out


def gauss_points(p: int) -> np.ndarray:
    return np.polynomial.legendre.leggauss(p + 1)[0]


def box_solution_points(mesh: dict, p: int) -> np.ndarray:
    """Physical coordinates [ne][ns][3] of the Gauss solution points of an
    axis-aligned box mesh (solution index i + n (j + n l), x fastest)."""
    xi = gauss_points(p)
    n = p + 1
    nodes, en = mesh["nodes"], mesh["elem_nodes"]
    lo = nodes[en[:, 0]]
    hi = nodes[en[:, 7]]
    r = (xi + 1.0) / 2.0
    rx, ry, rz = np.meshgrid(r, r, r, indexing="ij")
    ref = np.stack([rx, ry, rz], -1).transpose(2, 1, 0, 3).reshape(n ** 3, 3)
    return lo[:, None, :] + ref[None, :, :] * (hi - lo)[:, None, :]


# ---- mixed meshes: hexahedra, prisms, tetrahedra (straight elements) ----
# Element types and vertex orders of the C ABI.  Hexahedron: 8 vertices,
# x-fastest (reference [-1,1]^3).  Prism: the triangle (v0, v1, v2) at
# reference zeta = -1 and (v3, v4, v5) over it at zeta = +1, reference
# triangle (-1,-1), (1,-1), (-1,1).  Tetrahedron: reference vertices
# (-1,-1,-1), (1,-1,-1), (-1,1,-1), (-1,-1,1).  Faces are numbered as in
# MIXED_FACE_VERTS.
HEX, PRISM, TET = 0, 1, 2
MIXED_FACE_VERTS = {
    HEX: [[0, 2, 4, 6], [1, 3, 5, 7], [0, 1, 4, 5], [2, 3, 6, 7], [0, 1, 2, 3], [4, 5, 6, 7]],
    PRISM: [[0, 1, 2], [3, 4, 5], [0, 1, 4, 3], [1, 2, 5, 4], [2, 0, 3, 5]],
    TET: [[0, 1, 2], [0, 1, 3], [1, 2, 3], [0, 2, 3]],
}
MIXED_NVERT = {HEX: 8, PRISM: 6, TET: 4}
# the vertices whose offsets from v0 span the affine map of each type
_AFFINE_AXES = {HEX: (1, 2, 4), PRISM: (1, 2, 3), TET: (1, 2, 3)}


def mixed_box_mesh(N: int = 3, length: float = 1.0) -> dict:
    """Periodic box [0, L]^3 of N^3 cells: the centre cell (b, b, b), b = N // 2,
    split into the six Kuhn tetrahedra around its main diagonal; the other
    cells of the x row through it (j = k = b) split into two prisms extruded
    along x whose triangles halve the (y, z) square along its (min, min) -
    (max, max) diagonal, likewise the y and z rows; every other cell a
    hexahedron.  Every face is met by a face of the same shape and vertices
    (the Kuhn split halves each face of the centre cell along the same
    diagonal as the prisms).  Neighbours (element, face) are found by
    matching face vertices modulo the period."""
    import itertools
    assert N >= 3
    b = N // 2
    h = length / N
    n1 = N + 1
    g = np.arange(n1) * h
    nodes = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).transpose(2, 1, 0, 3).reshape(-1, 3)
    types, gverts = [], []  # gverts: integer grid coordinates of each vertex
    for k in range(N):
        for j in range(N):
            for i in range(N):
                o = np.array([i, j, k])
                if (i, j, k) == (b, b, b):
                    for perm in itertools.permutations(range(3)):
                        P = [o.copy()]
                        for d in perm:
                            q = P[-1].copy()
                            q[d] += 1
                            P.append(q)
                        e1, e2, e3 = P[1] - P[0], P[2] - P[0], P[3] - P[0]
                        if np.dot(np.cross(e1, e2), e3) < 0:
                            P[1], P[2] = P[2], P[1]
                        types.append(TET)
                        gverts.append(P)
                    continue
                axis = 0 if (j == b and k == b) else 1 if (i == b and k == b) else 2 if (i == b and j == b) else -1
                if axis < 0:
                    types.append(HEX)
                    gverts.append([o + np.array([a, bb, cc]) for cc in (0, 1) for bb in (0, 1) for a in (0, 1)])
                    continue
                d1, d2 = (axis + 1) % 3, (axis + 2) % 3
                for tri in (((0, 0), (1, 0), (1, 1)), ((0, 0), (1, 1), (0, 1))):
                    P = []
                    for end in (0, 1):
                        for (a1, a2) in tri:
                            q = o.copy()
                            q[d1] += a1
                            q[d2] += a2
                            q[axis] += end
                            P.append(q)
                    types.append(PRISM)
                    gverts.append(P)
    return _mixed_from_cells(N, length, nodes, types, gverts)


def prism_tet_box_mesh(N: int, length: float = 1.0) -> dict:
    """Periodic box [0, L]^3 of N^3 cells standing in for the paper's capsule
    mesh of prisms and tetrahedra: the lower N // 2 layers of cells each split
    into two prisms extruded along z (triangles halving the (x, y) square
    along its (min, min) - (max, max) diagonal, a boundary-layer stand-in),
    the upper layers each into the six Kuhn tetrahedra of its main diagonal.
    The Kuhn split halves every face of a cell along the same diagonal as the
    prisms, so all faces conform (triangles meet triangles, quadrilaterals
    quadrilaterals).  N >= 3 (with 2 cells per period distinct faces would
    have the same vertices modulo the period)."""
    import itertools
    assert N >= 3
    n1 = N + 1
    h = length / N
    g = np.arange(n1) * h
    nodes = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).transpose(2, 1, 0, 3).reshape(-1, 3)
    types, gverts = [], []
    for k in range(N):
        for j in range(N):
            for i in range(N):
                o = np.array([i, j, k])
                if k < N // 2:
                    for tri in (((0, 0), (1, 0), (1, 1)), ((0, 0), (1, 1), (0, 1))):
                        types.append(PRISM)
                        gverts.append([o + np.array([a, b, end]) for end in (0, 1) for (a, b) in tri])
                else:
                    for perm in itertools.permutations(range(3)):
                        P = [o.copy()]
                        for d in perm:
                            q = P[-1].copy()
                            q[d] += 1
                            P.append(q)
                        if np.dot(np.cross(P[1] - P[0], P[2] - P[0]), P[3] - P[0]) < 0:
                            P[1], P[2] = P[2], P[1]
                        types.append(TET)
                        gverts.append(P)
    return _mixed_from_cells(N, length, nodes, types, gverts)


def _mixed_from_cells(N, length, nodes, types, gverts) -> dict:
    """Mesh dictionary of elements given by integer grid vertices: element
    node lists and face neighbours found by matching face vertices modulo the
    period."""
    n1 = N + 1
    ne = len(types)
    en = np.full((ne, 8), -1, np.int32)
    for e, P in enumerate(gverts):
        en[e, :len(P)] = [int(c[0] + n1 * (c[1] + n1 * c[2])) for c in P]
    nbr = np.full((ne, 6), -1, np.int32)
    nbf = np.full((ne, 6), -1, np.int8)
    seen = {}
    for e, (t, P) in enumerate(zip(types, gverts)):
        for f, fv in enumerate(MIXED_FACE_VERTS[t]):
            key = frozenset(tuple(int(x) % N for x in P[v]) for v in fv)
            if key in seen:
                e2, f2 = seen.pop(key)
                nbr[e, f], nbf[e, f] = e2, f2
                nbr[e2, f2], nbf[e2, f2] = e, f
            else:
                seen[key] = (e, f)
    assert not seen, "unmatched faces"
    return {"n_elem": ne, "n_nodes": nodes.shape[0], "nodes": np.ascontiguousarray(nodes),
            "elem_type": np.asarray(types, np.int8), "elem_nodes": en, "nbr_elem": nbr, "nbr_face": nbf,
            "period": (length,) * 3, "N": N}


def gll_points(p: int) -> np.ndarray:
    """Gauss-Lobatto points on [-1, 1]: the ends and the roots of P_p'."""
    if p == 1:
        return np.array([-1.0, 1.0])
    inner = np.polynomial.legendre.Legendre.basis(p).deriv().roots()
    return np.concatenate([[-1.0], np.sort(inner.real), [1.0]])


def _simplex_points(p: int, dim: int) -> np.ndarray:
    """Solution points of the reference triangle (dim 2) or tetrahedron
    (dim 3) for p <= 3, in the ABI's order (barycentric indices (i, j[, k])
    with i + j [+ k] <= p, the last index outermost): the equispaced points
    with every point on an edge moved to the Gauss-Lobatto position along
    that edge (the alpha-optimised warp & blend points reduce to this for
    p <= 3)."""
    assert 1 <= p <= 3
    X = np.array([[-1, -1, -1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], float)[:dim + 1, :dim]
    gl = gll_points(p)
    pts = []
    rng = range(p + 1)
    idx = [(i, j, 0) for j in rng for i in rng if i + j <= p] if dim == 2 else \
          [(i, j, k) for k in rng for j in rng for i in rng if i + j + k <= p]
    for (i, j, k) in idx:
        lam = np.array([p - i - j - k, i, j, k][:dim + 1], float) / p
        nz = np.nonzero(lam)[0]
        if len(nz) == 2:
            a, c = nz
            m = int(round(lam[c] * p))
            lam[c] = (1.0 + gl[m]) / 2.0
            lam[a] = 1.0 - lam[c]
        pts.append(lam @ X)
    return np.array(pts)


def mixed_reference_points(etype: int, p: int) -> np.ndarray:
    """Reference coordinates [ns][3] of the solution points of an element
    type, in the ABI's order: hexahedron Gauss-Lobatto tensor points
    i + n (j + n l); prism triangle point t + n_tri l over the Gauss-Lobatto
    points l of the extrusion coordinate; tetrahedron as _simplex_points."""
    gl = gll_points(p)
    if etype == HEX:
        r = np.meshgrid(gl, gl, gl, indexing="ij")
        return np.stack(r, -1).transpose(2, 1, 0, 3).reshape(-1, 3)
    if etype == PRISM:
        tri = _simplex_points(p, 2)
        return np.array([[a, b_, z] for z in gl for (a, b_) in tri])
    return _simplex_points(p, 3)


def mixed_solution_points(mesh: dict, p: int) -> np.ndarray:
    """Physical coordinates [npts][3] of the solution points of a mixed mesh,
    element after element (straight elements: affine maps)."""
    out = []
    for e in range(mesh["n_elem"]):
        t = int(mesh["elem_type"][e])
        V = mesh["nodes"][mesh["elem_nodes"][e, :MIXED_NVERT[t]]]
        A = np.stack([V[a] - V[0] for a in _AFFINE_AXES[t]], 1)
        ref = mixed_reference_points(t, p)
        out.append(V[0] + (ref + 1.0) / 2.0 @ A.T)
    return np.concatenate(out, 0)


def velocity_axes(grid: dict):
    out = []
    for d in range(3):
        n = int(grid["n"][d])
        if n == 1:
            out.append(np.array([float(grid["umin"][d])]))
        else:
            out.append(np.linspace(float(grid["umin"][d]), float(grid["umax"][d]), n))
    return out


def grid_spec(n, umax, umin=None) -> dict:
    n = (int(n),) * 3 if np.isscalar(n) else tuple(int(v) for v in n)
    umax = (float(umax),) * 3 if np.isscalar(umax) else tuple(float(v) for v in umax)
    umin = tuple(-v for v in umax) if umin is None else (
        (float(umin),) * 3 if np.isscalar(umin) else tuple(float(v) for v in umin))
    return {"n": n, "umin": umin, "umax": umax}


# --------------------------------------------------------------------------
# Macroscopic initial fields
# --------------------------------------------------------------------------

def _wavevectors(kmin=1.0, kmax=2.0):
    ks = []
    for a in range(-2, 3):
        for b in range(-2, 3):
            for c in range(-2, 3):
                k = np.array([a, b, c], float)
                nk = np.linalg.norm(k)
                if nk < kmin - 1e-12 or nk > kmax + 1e-12:
                    continue
                nz = k[np.nonzero(k)[0][0]]
                if nz > 0:  # half-space representative
                    ks.append(k)
    return np.array(ks)


def divergence_free_field(xs: np.ndarray, seed: int, amp: float) -> np.ndarray:
    """Sum of Fourier modes with 1 <= |k| <= 2 whose amplitudes are projected
    perpendicular to k (divergence free), scaled to max |U| = amp."""
    rng = np.random.default_rng(seed)
    ks = _wavevectors()
    U = np.zeros(xs.shape)
    for k in ks:
        a, b = rng.standard_normal(3), rng.standard_normal(3)
        kh = k / np.linalg.norm(k)
        a -= kh * (a @ kh)
        b -= kh * (b @ kh)
        ph = 2 * np.pi * (xs @ k)
        U += np.cos(ph)[..., None] * a + np.sin(ph)[..., None] * b
    m = np.linalg.norm(U, axis=-1).max()
    return U * (amp / m)


def prim_random_modes(xs: np.ndarray, seed: int = 1, U_amp: float = 0.2) -> np.ndarray:
    """Config-1 field: rho = 1 + 0.1 sin sin sin, U = random divergence-free
    modes (|k| in [1,2]) with max |U| = U_amp, theta = 1 + 0.05 cos(2 pi k*.x + phi)."""
    rng = np.random.default_rng(seed + 1000)
    x, y, z = xs[..., 0], xs[..., 1], xs[..., 2]
    rho = 1.0 + 0.1 * np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y) * np.sin(2 * np.pi * z)
    U = divergence_free_field(xs, seed, U_amp)
    ks = _wavevectors()
    kst = ks[rng.integers(len(ks))]
    phi = rng.uniform(0, 2 * np.pi)
    theta = 1.0 + 0.05 * np.cos(2 * np.pi * (xs @ kst) + phi)
    return np.concatenate([rho[..., None], U, theta[..., None]], -1)


def prim_taylor_green(xs: np.ndarray, U0: float, pert: float = 0.0, seed: int = 5) -> np.ndarray:
    """Taylor-Green vortex on the unit box, rho = theta = 1, plus an optional
    seeded divergence-free perturbation of amplitude pert * U0."""
    x, y, z = xs[..., 0], xs[..., 1], xs[..., 2]
    s2 = 2 * np.pi
    U = np.stack([U0 * np.sin(s2 * x) * np.cos(s2 * y) * np.cos(s2 * z),
                  -U0 * np.cos(s2 * x) * np.sin(s2 * y) * np.cos(s2 * z),
                  np.zeros_like(x)], -1)
    if pert > 0:
        U = U + divergence_free_field(xs, seed, pert * U0)
    one = np.ones(x.shape + (1,))
    return np.concatenate([one, U, one], -1)


def maxwellian(prim, grid: dict, dtype=None, device="cpu", chunk_pts: int = 1 << 14):
    """f[..., k] = rho (2 pi theta)^(-3/2) exp(-|u_k - U|^2 / (2 theta)) at every
    node k = i + n0 (j + n1 l) of the velocity grid, computed in FP64 with torch
    and cast to ``dtype``.  prim[..., 5] = (rho, Ux, Uy, Uz, theta)."""
    import torch
    dtype = dtype or torch.float64
    prim = torch.as_tensor(np.asarray(prim), dtype=torch.float64)
    lead = prim.shape[:-1]
    pr = prim.reshape(-1, 5)
    ax = [torch.as_tensor(a, dtype=torch.float64, device=device) for a in velocity_axes(grid)]
    n0, n1, n2 = (len(a) for a in ax)
    out = torch.empty((pr.shape[0], n0 * n1 * n2), dtype=dtype, device=device)
    for s in range(0, pr.shape[0], chunk_pts):
        p = pr[s:s + chunk_pts].to(device)
        rho, U, th = p[:, 0:1], p[:, 1:4], p[:, 4:5]
        ex = torch.exp(-(ax[0][None, :] - U[:, 0:1]) ** 2 / (2 * th))
        ey = torch.exp(-(ax[1][None, :] - U[:, 1:2]) ** 2 / (2 * th))
        ez = torch.exp(-(ax[2][None, :] - U[:, 2:3]) ** 2 / (2 * th))
        c = rho * (2 * math.pi * th) ** -1.5
        f = (c[:, :, None, None] * ez[:, :, None, None] * ey[:, None, :, None]
             * ex[:, None, None, :])
        out[s:s + chunk_pts] = f.reshape(p.shape[0], -1).to(dtype)
    return out.reshape(tuple(lead) + (n0 * n1 * n2,))


# --------------------------------------------------------------------------
# Macroscopic states for the learned Newton guess
# --------------------------------------------------------------------------

def lattice_min_variance(U: np.ndarray, umax: float, nv: int) -> np.ndarray:
    """Smallest sum over axes of the variance a non-negative distribution on
    the closed uniform grid [-umax, umax] can have at mean velocity U: all
    mass on the two nodes bracketing U_d, i.e. (U_d - u_i)(u_{i+1} - U_d)."""
    du = 2 * umax / (nv - 1)
    i = np.clip(np.floor((U + umax) / du), 0, nv - 2)
    lo = -umax + i * du
    return ((U - lo) * (lo + du - U)).sum(-1)


def sample_states(n: int, seed: int = 4, umax_choices=(6.0, 10.0, 14.0), nv: int = 32, margin: float = 1.05):
    """Seeded macroscopic states: rho log-normal (sigma 1), |U| uniform up to
    0.8 u_max with a uniform direction, theta log-uniform on [0.1, 4], u_max
    drawn from umax_choices.  States whose temperature is within `margin` of
    the lattice bound 3 theta > min variance (not attainable by any positive
    distribution on the grid) are rejected and redrawn.
    Returns dict of arrays rho[n], U[n,3], theta[n], umax[n], and the
    rejection rate."""
    rng = np.random.default_rng(seed)
    out = {"rho": [], "U": [], "theta": [], "umax": []}
    drawn = kept = n_ok = 0
    while kept < n:
        m = 2 * (n - kept) + 16
        rho = np.exp(rng.standard_normal(m))
        d = rng.standard_normal((m, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        um = rng.choice(np.asarray(umax_choices, float), m)
        U = d * (rng.uniform(0, 0.8, m) * um)[:, None]
        th = np.exp(rng.uniform(np.log(0.1), np.log(4.0), m))
        ok = np.array([3 * th[i] > margin * lattice_min_variance(U[i], um[i], nv) for i in range(m)])
        drawn += m
        n_ok += int(ok.sum())
        take = np.nonzero(ok)[0][: n - kept]
        for k, v in (("rho", rho), ("U", U), ("theta", th), ("umax", um)):
            out[k].append(v[take])
        kept += len(take)
    res = {k: np.concatenate(v) for k, v in out.items()}
    res["reject_rate"] = 1.0 - n_ok / drawn
    return res


def state_moments(rho, U, theta):
    """Q = (rho, rho U, rho |U|^2 / 2 + 3/2 rho theta) of the continuous state."""
    rho = np.asarray(rho)
    U = np.asarray(U)
    th = np.asarray(theta)
    E = 0.5 * rho * (U * U).sum(-1) + 1.5 * rho * th
    return np.concatenate([rho[:, None], rho[:, None] * U, E[:, None]], 1)


# --------------------------------------------------------------------------
# Named workloads (the shapes of the paper's runs, scaled to one GPU)
# --------------------------------------------------------------------------

OMEGA_POWER_LAW = 0.81


def workload(name: str) -> dict:
    """Definition of a named workload: mesh builder args, order, grid, physics."""
    W = {
        # 4^3 periodic box, p=1, 8^3 grid on [-6,6]^3, BGK, Kn=0.05, 10 SSP-RK3 steps
        "box4_p1_v8": dict(N=4, p=1, grid=grid_spec(8, 6.0), model=0, prandtl=1.0,
                           kn=0.05, ic="modes", seed=1, steps=10, rk=0, precision=0),
        # 16^3 periodic box, p=3, 16^3 grid on [-6,6]^3, BGK, Kn=1e-3, Taylor-Green U0=0.3
        "box16_p3_v16": dict(N=16, p=3, grid=grid_spec(16, 6.0), model=0, prandtl=1.0,
                             kn=1e-3, ic="tgv", U0=0.3, pert=0.0, seed=2, steps=100, rk=0,
                             precision=0),
        # 24^3 periodic box, p=3, 20^3 grid on [-8,8]^3, ES-BGK Pr=0.71, Kn=2e-4,
        # Taylor-Green U0=0.5 with a 1% seeded perturbation
        "box24_p3_v20_es": dict(N=24, p=3, grid=grid_spec(20, 8.0), model=1, prandtl=0.71,
                                kn=2e-4, ic="tgv", U0=0.5, pert=0.01, seed=5, steps=200,
                                rk=1, precision=2),
        # O-grid around the cylinder of diameter 1: 24 radial (growth 1.15) x 48 azimuthal
        # x 2 spanwise quadratic hexes, p=2, 24^3 grid on [-14,14]^3, ES-BGK Pr=2/3,
        # Kn=0.01, uniform Mach-8 inflow at theta=1 (1% seeded density noise),
        # diffuse wall at theta_w=2, farfield outside
        # prisms + tetrahedra standing in for the paper's capsule mesh: 12^3 cells,
        # lower half prisms, upper half Kuhn tetrahedra (1728 prisms, 5184
        # tetrahedra, 172800 solution points), p=3, 24^3 grid on [-8,8]^3 (the
        # paper's velocity resolution), ES-BGK Pr=2/3, Kn=1e-3, Taylor-Green U0=0.3
        "ptbox12_p3_v24_es": dict(mesh="prism_tet", N=12, p=3, grid=grid_spec(24, 8.0), model=1,
                                  prandtl=2.0 / 3.0, kn=1e-3, ic="tgv", U0=0.3, pert=0.01, seed=7,
                                  steps=50, rk=1, precision=1),
        "cyl48x24x2_p2_v24_es": dict(mesh="cylinder", p=2, grid=grid_spec(24, 14.0), model=1,
                                     prandtl=2.0 / 3.0, kn=0.01, ic="uniform", mach=8.0, noise=0.01,
                                     theta_wall=2.0, seed=31, steps=2000, rk=1, precision=1, positivity=1),
    }
    w = dict(W[name])
    w["name"] = name
    w["mu_ref"] = mu_ref_from_knudsen(w["kn"])
    if w.get("ic") == "uniform":
        w["farfield"] = [1.0, w["mach"] * math.sqrt(5.0 / 3.0), 0.0, 0.0, 1.0]
    return w


def paper_freestream(mach: float, reynolds: float, alpha_deg: float = 0.0, t_inf_kelvin: float = 203.0,
                     gamma: float = 5.0 / 3.0) -> dict:
    """Physics parameters in the paper's freestream units (unit density and
    speed, P = 1/(gamma M^2), mu_ref = 1/Re at theta_ref = P, Sutherland
    temperature 110.4 K scaled by the freestream temperature, wall at the
    freestream temperature, farfield = the freestream Maxwellian)."""
    th = 1.0 / (gamma * mach * mach)
    a = math.radians(alpha_deg)
    return {"mu_ref": 1.0 / reynolds, "theta_ref": th, "visc_law": 1, "theta_s": th * 110.4 / t_inf_kelvin,
            "farfield": [1.0, math.cos(a), math.sin(a), 0.0, th], "theta_wall": th}


def workload_mesh(w: dict) -> dict:
    if w.get("mesh") == "cylinder":
        return cylinder_mesh()
    if w.get("mesh") == "prism_tet":
        return prism_tet_box_mesh(w["N"])
    return box_mesh(w["N"])


def initial_prim(mesh: dict, p: int, w: dict) -> np.ndarray:
    if w["ic"] == "uniform":
        # the farfield state everywhere, density with seeded uniform noise
        ns = (p + 1) ** 3
        rng = np.random.default_rng(w["seed"])
        prim = np.tile(np.asarray(w["farfield"], dtype=float), (mesh["n_elem"], ns, 1))
        prim[..., 0] *= 1.0 + w["noise"] * rng.uniform(-1.0, 1.0, size=(mesh["n_elem"], ns))
        return prim
    # mixed meshes: [points][5] (the library's point-per-element view)
    xs = mixed_solution_points(mesh, p)[:, None, :] if "elem_type" in mesh else box_solution_points(mesh, p)
    if w["ic"] == "modes":
        return prim_random_modes(xs, seed=w["seed"])
    if w["ic"] == "tgv":
        return prim_taylor_green(xs, w["U0"], w.get("pert", 0.0), w.get("seed", 5))
    raise ValueError(w["ic"])


def physics_params(w: dict) -> dict:
    par = {"model": w["model"], "prandtl": w["prandtl"], "mu_ref": w["mu_ref"],
           "theta_ref": 1.0, "omega": OMEGA_POWER_LAW, "visc_law": 0, "theta_s": 0.0,
           "newton_tol": 1e-13, "newton_max_iter": 50}
    if "farfield" in w:
        par["farfield"] = list(w["farfield"])
        par["theta_wall"] = w["theta_wall"]
    # the positivity-preserving scheme: on where a wall meets an impulsive
    # start (the smooth periodic boxes keep f positive without it)
    par["positivity"] = int(w.get("positivity", 0))
    return par
