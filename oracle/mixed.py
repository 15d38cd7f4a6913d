"""FP64 CPU oracle of the FR residual on mixed meshes of straight hexahedra,
prisms and tetrahedra (the paper's element types, Section "Implementation &
problem setup": prisms and tetrahedra, alpha-optimised points on simplices,
Gauss-Lobatto points on tensor-product elements).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import it.  It shares no code with the
HIP library and never imports it.

What it computes (Section "Numerical method", eq. transport: every velocity
node u is advected by its own FR scheme; upwind interface flux; the
correction that recovers the DG scheme): on each element, with the solution
polynomial f_h interpolating the nodal values,

    R_i = - u . grad f_h (x_i)
          - sum_faces (|J_face| / |J|) sum_j LIFT_f[i, j] min(u.n, 0) (f_nb,j - f_j)

where LIFT_f = M^-1 E_f is the DG-recovering correction of a unit jump at
face point j (M the element mass matrix, E_f[i, j] the integral over the
face of l_i l_j), f_j the element's own value at face point j and f_nb,j the
neighbour's value at the same physical point.  For the point sets used here
the face (flux) points are the solution points lying on the face, so the
traces need no interpolation.  Reading (p <= 3): the alpha-optimised warp &
blend points of Hesthaven & Warburton reduce, for any alpha, to the vertices,
the Gauss-Lobatto points along every edge and the face / cell centroids
(``warp_blend_tri`` and ``warp_blend_tet`` construct them from the published
algorithm for the tests to check this); prisms take the triangle points times
the Gauss-Lobatto points of the extrusion coordinate.

Derivation (independent of the library's): Lagrange bases through a monomial
Vandermonde matrix; volume integrals of monomials exactly in rational
arithmetic; face integrals with a Duffy-collapsed (triangles) or tensor
(quadrilaterals) Gauss-Legendre rule of more than enough points.  The
collision source, moments and totals reuse the point-wise FP64 oracle.
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction

import numpy as np

HEX, PRISM, TET = 0, 1, 2
NVERT = {HEX: 8, PRISM: 6, TET: 4}
# reference vertices of each type (the ABI's vertex order)
REF_VERTS = {
    HEX: np.array([[a, b, c] for c in (-1, 1) for b in (-1, 1) for a in (-1, 1)], float),
    PRISM: np.array([[-1, -1, -1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1], [1, -1, 1], [-1, 1, 1]], float),
    TET: np.array([[-1, -1, -1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], float),
}
FACE_VERTS = {
    HEX: [[0, 2, 4, 6], [1, 3, 5, 7], [0, 1, 4, 5], [2, 3, 6, 7], [0, 1, 2, 3], [4, 5, 6, 7]],
    PRISM: [[0, 1, 2], [3, 4, 5], [0, 1, 4, 3], [1, 2, 5, 4], [2, 0, 3, 5]],
    TET: [[0, 1, 2], [0, 1, 3], [1, 2, 3], [0, 2, 3]],
}
# vertices whose offsets from vertex 0 give the columns of the affine map
AXES = {HEX: (1, 2, 4), PRISM: (1, 2, 3), TET: (1, 2, 3)}


# ---------------------------------------------------------------- points --

def gauss_lobatto_points(p: int) -> np.ndarray:
    """-1, the roots of P_p' (Legendre), 1 (ascending)."""
    if p == 1:
        return np.array([-1.0, 1.0])
    c = np.zeros(p + 1)
    c[p] = 1.0
    r = np.polynomial.legendre.legroots(np.polynomial.legendre.legder(c))
    return np.concatenate([[-1.0], np.sort(r), [1.0]])


def _simplex_index(p: int, dim: int):
    r = range(p + 1)
    if dim == 2:
        return [(i, j) for j in r for i in r if i + j <= p]
    return [(i, j, k) for k in r for j in r for i in r if i + j + k <= p]


def simplex_points(p: int, dim: int) -> np.ndarray:
    """Reference points of the triangle / tetrahedron for p <= 3: barycentric
    index (i, j[, k]) / p, and every point with exactly two nonzero
    barycentric coordinates moved along its edge to the Gauss-Lobatto
    position."""
    if not 1 <= p <= 3:
        raise ValueError("p <= 3")
    V = REF_VERTS[TET][:dim + 1, :dim]
    gl = gauss_lobatto_points(p)
    out = []
    for idx in _simplex_index(p, dim):
        lam = np.array([p - sum(idx)] + list(idx), float) / p
        nz = [a for a in range(dim + 1) if lam[a] > 0]
        if len(nz) == 2:
            a, b = nz
            m = int(round(lam[b] * p))
            lam[b] = 0.5 * (1.0 + gl[m])
            lam[a] = 1.0 - lam[b]
        out.append(lam @ V)
    return np.array(out)


def reference_points(etype: int, p: int) -> np.ndarray:
    gl = gauss_lobatto_points(p)
    if etype == HEX:
        return np.array([[a, b, c] for c in gl for b in gl for a in gl])
    if etype == PRISM:
        tri = simplex_points(p, 2)
        return np.array([[a, b, c] for c in gl for (a, b) in tri])
    return simplex_points(p, 3)


# Warp & blend construction (Hesthaven & Warburton, "Nodal Discontinuous
# Galerkin Methods", Sections 6.1 and 10.1), written from the published
# description, for the tests that check the closed form above against it.
# alpha tables of that reference (index N - 1).
ALPHA_TRI = [0.0000, 0.0000, 1.4152, 0.1001, 0.2751, 0.9800, 1.0999, 1.2832, 1.3648, 1.4773, 1.4959, 1.5743,
             1.5770, 1.6223, 1.6258]
ALPHA_TET = [0.0, 0.0, 0.0, 0.1002, 1.1332, 1.5608, 1.3413, 1.2577, 1.1603, 1.10153, 0.6080, 0.4523, 0.8856,
             0.8717, 0.9655]


def _warp1d(p: int, r: np.ndarray) -> np.ndarray:
    """Interpolant through the equispaced points of the displacement to the
    Gauss-Lobatto points, evaluated at r, divided by 1 - r^2 (the edge warp
    without its end zeros)."""
    req = np.linspace(-1.0, 1.0, p + 1)
    gl = gauss_lobatto_points(p)
    w = np.zeros_like(r)
    for i in range(p + 1):
        li = np.ones_like(r)
        for j in range(p + 1):
            if j != i:
                li *= (r - req[j]) / (req[i] - req[j])
        w += (gl[i] - req[i]) * li
    interior = np.abs(r) < 1.0 - 1e-10
    out = np.zeros_like(r)
    out[interior] = w[interior] / (1.0 - r[interior] ** 2)
    return out


def warp_blend_tri(p: int, alpha: float | None = None) -> np.ndarray:
    """Points of the equilateral triangle (-1, -1/sqrt3), (1, -1/sqrt3),
    (0, 2/sqrt3), returned as barycentric coordinates [n][3]."""
    if alpha is None:
        alpha = ALPHA_TRI[p - 1]
    idx = _simplex_index(p, 2)
    L2 = np.array([i for i, j in idx], float) / p
    L3 = np.array([j for i, j in idx], float) / p
    L1 = 1.0 - L2 - L3
    x = -L2 + L3
    y = (-L2 - L3 + 2.0 * L1) / math.sqrt(3.0)
    b1, b2, b3 = 4 * L2 * L3, 4 * L1 * L3, 4 * L1 * L2
    w1, w2, w3 = _warp1d(p, L3 - L2), _warp1d(p, L1 - L3), _warp1d(p, L2 - L1)
    w1 = b1 * w1 * (1 + (alpha * L1) ** 2)
    w2 = b2 * w2 * (1 + (alpha * L2) ** 2)
    w3 = b3 * w3 * (1 + (alpha * L3) ** 2)
    X = x + w1 + math.cos(2 * math.pi / 3) * w2 + math.cos(4 * math.pi / 3) * w3
    Y = y + math.sin(2 * math.pi / 3) * w2 + math.sin(4 * math.pi / 3) * w3
    # back to barycentric coordinates of the equilateral triangle
    V = np.array([[-1.0, -1.0 / math.sqrt(3)], [1.0, -1.0 / math.sqrt(3)], [0.0, 2.0 / math.sqrt(3)]])
    T = np.array([[V[1, 0] - V[0, 0], V[2, 0] - V[0, 0]], [V[1, 1] - V[0, 1], V[2, 1] - V[0, 1]]])
    lam = np.linalg.solve(T, np.stack([X - V[0, 0], Y - V[0, 1]]))
    return np.stack([1 - lam[0] - lam[1], lam[0], lam[1]], 1)


def _eval_shift(p, alpha, L1, L2, L3):
    """Warp shift (2-D) of the face blend of the tetrahedron construction."""
    w1, w2, w3 = _warp1d(p, L3 - L2), _warp1d(p, L1 - L3), _warp1d(p, L2 - L1)
    b1, b2, b3 = 4 * L2 * L3, 4 * L1 * L3, 4 * L1 * L2
    w1 = b1 * w1 * (1 + (alpha * L1) ** 2)
    w2 = b2 * w2 * (1 + (alpha * L2) ** 2)
    w3 = b3 * w3 * (1 + (alpha * L3) ** 2)
    dx = w1 + math.cos(2 * math.pi / 3) * w2 + math.cos(4 * math.pi / 3) * w3
    dy = math.sin(2 * math.pi / 3) * w2 + math.sin(4 * math.pi / 3) * w3
    return dx, dy


def warp_blend_tet(p: int, alpha: float | None = None) -> np.ndarray:
    """Points of the regular tetrahedron by warp & blend, returned as
    barycentric coordinates [n][4] (vertex order of the reference tet)."""
    if alpha is None:
        alpha = ALPHA_TET[p - 1]
    idx = _simplex_index(p, 3)
    lam = np.array([[p - sum(t)] + list(t) for t in idx], float) / p  # L1..L4 <-> vertices 0..3
    v = np.array([[-1, -1 / math.sqrt(3), -1 / math.sqrt(6)], [1, -1 / math.sqrt(3), -1 / math.sqrt(6)],
                  [0, 2 / math.sqrt(3), -1 / math.sqrt(6)], [0, 0, 3 / math.sqrt(6)]])
    X = lam @ v
    shift = np.zeros_like(X)
    tol = 1e-10
    # (a, b, c, d): the face lam_a = 0 and its points' barycentric
    # coordinates (b, c, d) in the order of the triangle construction (its
    # x axis runs from vertex c to vertex d, its y axis towards vertex b)
    faces = [(3, 2, 0, 1), (2, 3, 0, 1), (0, 3, 1, 2), (1, 3, 0, 2)]
    for a, b, c, d in faces:
        La, Lb, Lc, Ld = lam[:, a], lam[:, b], lam[:, c], lam[:, d]
        dx, dy = _eval_shift(p, alpha, Lb, Lc, Ld)
        blend = Lb * Lc * Ld
        denom = (Lb + 0.5 * La) * (Lc + 0.5 * La) * (Ld + 0.5 * La)
        ids = denom > tol
        blend_f = blend.copy()
        blend_f[ids] = (1 + (alpha * La[ids]) ** 2) * blend[ids] / denom[ids]
        t1 = v[d] - v[c]
        t2 = v[b] - 0.5 * (v[c] + v[d])
        t1 = t1 / np.linalg.norm(t1)
        t2 = t2 / np.linalg.norm(t2)
        shift += (blend_f * dx)[:, None] * t1[None] + (blend_f * dy)[:, None] * t2[None]
        # points on an edge of this face take its warp alone
        onface = (La < tol) & ((Lb > tol).astype(int) + (Lc > tol) + (Ld > tol) < 3)
        shift[onface] = dx[onface, None] * t1[None] + dy[onface, None] * t2[None]
    X = X + shift
    T = np.stack([v[1] - v[0], v[2] - v[0], v[3] - v[0]], 1)
    l = np.linalg.solve(T, (X - v[0]).T).T
    return np.concatenate([1 - l.sum(1, keepdims=True), l], 1)


# ------------------------------------------------------------ operators --

def exponents(etype: int, p: int):
    r = range(p + 1)
    if etype == HEX:
        return [(a, b, c) for c in r for b in r for a in r]
    if etype == PRISM:
        return [(a, b, c) for c in r for b in r for a in r if a + b <= p]
    return [(a, b, c) for c in r for b in r for a in r if a + b + c <= p]


def _shift_binomial(a):
    """Coefficients of r^a with r = 2x - 1 as a polynomial in x."""
    return [(k, Fraction(math.comb(a, k) * 2 ** k * (-1) ** (a - k))) for k in range(a + 1)]


def mono_integral(etype: int, a: int, b: int, c: int) -> Fraction:
    """Exact integral of r^a s^t t^c over the reference element."""
    if etype == HEX:
        one = lambda n: Fraction(2, n + 1) if n % 2 == 0 else Fraction(0)
        return one(a) * one(b) * one(c)
    if etype == PRISM:
        # triangle (r, s): r = 2x - 1, s = 2y - 1 on the unit triangle (Jacobian 4)
        tri = Fraction(0)
        for k, ck in _shift_binomial(a):
            for l, cl in _shift_binomial(b):
                tri += ck * cl * Fraction(math.factorial(k) * math.factorial(l), math.factorial(k + l + 2))
        line = Fraction(2, c + 1) if c % 2 == 0 else Fraction(0)
        return 4 * tri * line
    tot = Fraction(0)
    for k, ck in _shift_binomial(a):
        for l, cl in _shift_binomial(b):
            for m, cm in _shift_binomial(c):
                tot += ck * cl * cm * Fraction(math.factorial(k) * math.factorial(l) * math.factorial(m),
                                               math.factorial(k + l + m + 3))
    return 8 * tot


def _vander(pts, ex):
    return np.array([[x ** a * y ** b * z ** c for (a, b, c) in ex] for (x, y, z) in pts])


def _quad_edges(verts: np.ndarray):
    """First vertex and the two edge vectors from it of a parallelogram
    given by its 4 vertices in any order (the farthest one is opposite)."""
    A = verts[0]
    far = int(np.argmax([np.linalg.norm(v - A) for v in verts[1:]])) + 1
    B, D = [verts[i] for i in range(1, 4) if i != far]
    return A, B - A, D - A


def _face_rule(verts: np.ndarray, n: int):
    """Quadrature points and weights (reference surface measure) on a planar
    reference face with 3 or 4 vertices (the quadrilaterals here are
    parallelograms)."""
    g, w = np.polynomial.legendre.leggauss(n)
    g, w = 0.5 * (g + 1.0), 0.5 * w
    A = verts[0]
    if len(verts) == 3:
        B, Cc = verts[1], verts[2]
        area2 = np.linalg.norm(np.cross(B - A, Cc - A))
        pts, wts = [], []
        for i in range(n):
            for j in range(n):
                u, v = g[i], g[j] * (1.0 - g[i])
                pts.append(A + u * (B - A) + v * (Cc - A))
                wts.append(w[i] * w[j] * (1.0 - g[i]) * area2)
        return np.array(pts), np.array(wts)
    A, eB, eD = _quad_edges(verts)
    area = np.linalg.norm(np.cross(eB, eD))
    pts = np.array([A + g[i] * eB + g[j] * eD for i in range(n) for j in range(n)])
    wts = np.array([w[i] * w[j] * area for i in range(n) for j in range(n)])
    return pts, wts


class RefElement:
    """Nodal operators of one reference element type at order p.  The
    monomial Vandermonde matrix is inverted and the operators formed in
    32-digit arithmetic (mpmath) and rounded to FP64 once, so that the
    conditioning of the monomial basis (about 1e4 at p = 3) costs no FP64
    digits."""

    def __init__(self, etype: int, p: int):
        import mpmath as mp
        mp.mp.dps = 32
        self.etype, self.p = etype, p
        self.x = reference_points(etype, p)
        self.ns = len(self.x)
        ex = exponents(etype, p)
        assert len(ex) == self.ns
        self.ex = ex
        X = [[mp.mpf(float(v)) for v in row] for row in self.x]
        V = mp.matrix([[x ** a * y ** b * z ** c for (a, b, c) in ex] for (x, y, z) in X])
        Cm = V ** -1  # column i: monomial coefficients of l_i
        self.C = np.array(Cm.tolist(), dtype=float)

        def dvander(d):
            rows = []
            for pt in X:
                row = []
                for e in ex:
                    if e[d] == 0:
                        row.append(mp.mpf(0))
                    else:
                        e2 = list(e)
                        e2[d] -= 1
                        row.append(e[d] * pt[0] ** e2[0] * pt[1] ** e2[1] * pt[2] ** e2[2])
                rows.append(row)
            return mp.matrix(rows)

        self.D = [np.array((dvander(d) * Cm).tolist(), dtype=float) for d in range(3)]
        Mm = mp.matrix([[mp.mpf(mono_integral(etype, a1 + a2, b1 + b2, c1 + c2).numerator) /
                         mono_integral(etype, a1 + a2, b1 + b2, c1 + c2).denominator for (a2, b2, c2) in ex]
                        for (a1, b1, c1) in ex])
        Mmp = Cm.T * Mm * Cm
        self.M = np.array(Mmp.tolist(), dtype=float)
        self.Minv = np.array((Mmp ** -1).tolist(), dtype=float)
        self.W = np.array([float(mp.fsum(Mmp[i, j] for j in range(self.ns))) for i in range(self.ns)])
        self.faces = []
        for fv in FACE_VERTS[etype]:
            verts = REF_VERTS[etype][fv]
            nrm = np.cross(verts[1] - verts[0], verts[2] - verts[0])
            nrm /= np.linalg.norm(nrm)
            on = [i for i in range(self.ns) if abs((self.x[i] - verts[0]) @ nrm) < 1e-12]
            q, wq = _face_rule(verts, p + 3)
            L = _vander(q, ex) @ self.C[:, on]  # face points' Lagrange functions at the face rule
            E = (L * wq[:, None]).T @ L
            area = wq.sum()
            self.faces.append({"verts": fv, "nodes": np.array(on), "lift": self.Minv[:, on] @ E, "area": area})

    def basis(self, pts: np.ndarray) -> np.ndarray:
        """Lagrange basis functions at reference points [m][3] -> [m][ns]."""
        return _vander(np.asarray(pts, float), self.ex) @ self.C


_REF_CACHE = {}


def ref_element(etype: int, p: int) -> RefElement:
    key = (int(etype), int(p))
    if key not in _REF_CACHE:
        _REF_CACHE[key] = RefElement(*key)
    return _REF_CACHE[key]


# ----------------------------------------------------------------- mesh --

class MixedMesh:
    """Geometry, face-point matching and per-face scalings of a mesh of
    straight elements (affine maps x = x0 + A (xi + 1))."""

    def __init__(self, mesh: dict, p: int):
        self.p = p
        self.ne = int(mesh["n_elem"])
        self.types = np.asarray(mesh["elem_type"], int)
        self.ref = {t: ref_element(t, p) for t in set(self.types.tolist())}
        X = np.asarray(mesh["nodes"], float)
        en = np.asarray(mesh["elem_nodes"])
        per = np.asarray(mesh.get("period", (0.0, 0.0, 0.0)), float)
        self.off = np.zeros(self.ne + 1, int)
        for e in range(self.ne):
            self.off[e + 1] = self.off[e] + self.ref[self.types[e]].ns
        self.npts = int(self.off[-1])
        self.A, self.Ainv, self.detJ, self.xs = [], [], np.zeros(self.ne), np.zeros((self.npts, 3))
        self.fnorm, self.fscale, self.fpts = [], [], []
        self.vol = np.zeros(self.ne)
        self.hmin = np.inf
        for e in range(self.ne):
            t = self.types[e]
            R = self.ref[t]
            Vx = X[en[e, :NVERT[t]]]
            A = np.stack([(Vx[a] - Vx[0]) / 2.0 for a in AXES[t]], 1)
            # the straight element must be the affine image of the reference one
            img = Vx[0] + (REF_VERTS[t] + 1.0) @ A.T
            if np.abs(img - Vx).max() > 1e-12 * (1 + np.abs(Vx).max()):
                raise ValueError(f"element {e} is not affine")
            dj = np.linalg.det(A)
            if dj <= 0:
                raise ValueError(f"element {e}: non-positive Jacobian")
            self.A.append(A)
            self.Ainv.append(np.linalg.inv(A))
            self.detJ[e] = dj
            self.xs[self.off[e]:self.off[e + 1]] = Vx[0] + (R.x + 1.0) @ A.T
            cen = Vx.mean(0)
            nrms, scales, pts = [], [], []
            amax = 0.0
            for fc in R.faces:
                fvx = Vx[fc["verts"]]
                nrm = np.cross(fvx[1] - fvx[0], fvx[2] - fvx[0])
                area = 0.5 * np.linalg.norm(nrm) if len(fvx) == 3 else np.linalg.norm(np.cross(*_quad_edges(fvx)[1:]))
                nrm /= np.linalg.norm(nrm)
                if (fvx.mean(0) - cen) @ nrm < 0:
                    nrm = -nrm
                nrms.append(nrm)
                scales.append(area / fc["area"] / dj)  # |J_face| / |J|
                pts.append(self.xs[self.off[e] + fc["nodes"]])
                amax = max(amax, area)
            self.vol[e] = dj * R.W.sum()
            self.hmin = min(self.hmin, self.vol[e] / amax)
            self.fnorm.append(nrms)
            self.fscale.append(scales)
            self.fpts.append(pts)
        # neighbour's point (global index) at every face point
        nbr, nbf = np.asarray(mesh["nbr_elem"]), np.asarray(mesh["nbr_face"])
        self.fmatch = []
        for e in range(self.ne):
            R = self.ref[self.types[e]]
            ms = []
            for f, fc in enumerate(R.faces):
                n2, f2 = int(nbr[e, f]), int(nbf[e, f])
                if n2 < 0:
                    raise ValueError("mixed oracle: periodic / closed meshes only")
                mine, theirs = self.fpts[e][f], self.fpts[n2][f2]
                shift = mine.mean(0) - theirs.mean(0)
                shift = np.where(per > 0, per * np.round(shift / np.where(per > 0, per, 1.0)), 0.0)
                R2 = self.ref[self.types[n2]]
                idx = []
                for x in mine:
                    d = np.linalg.norm(theirs + shift - x, axis=1)
                    k = int(np.argmin(d))
                    if d[k] > 1e-9:
                        raise ValueError(f"face points of element {e} face {f} do not match")
                    idx.append(self.off[n2] + R2.faces[f2]["nodes"][k])
                ms.append(np.array(idx))
            self.fmatch.append(ms)


# ------------------------------------------------------------- problem --

class MixedProblem:
    """Mixed mesh + order + velocity grid + physics parameters."""

    def __init__(self, mesh: dict, p: int, grid: dict, params: dict):
        import oracle as O
        self.mm = MixedMesh(mesh, p)
        self.p = p
        self.u, self.w = O.vgrid(grid["n"], grid["umin"], grid["umax"])
        self.nu = self.u.shape[0]
        self.params = dict(params)
        self._pts = O.Problem.points_only(grid, params) if "mu_ref" in params else None

    @property
    def shape(self):
        return (self.mm.npts, self.nu)

    def residual(self, f):
        """df/dt of the transport alone, [npts][nu]."""
        mm = self.mm
        f = np.asarray(f, float).reshape(self.shape)
        R = np.zeros_like(f)
        for e in range(mm.ne):
            Rf = mm.ref[mm.types[e]]
            sl = slice(mm.off[e], mm.off[e + 1])
            fe = f[sl]
            c = self.u @ mm.Ainv[e].T  # c[k, a] = sum_d u_kd dxi_a/dx_d
            r = np.zeros_like(fe)
            for a in range(3):
                r -= (Rf.D[a] @ fe) * c[None, :, a]
            for fidx, fc in enumerate(Rf.faces):
                un = self.u @ mm.fnorm[e][fidx]
                jump = np.minimum(un, 0.0)[None, :] * (f[mm.fmatch[e][fidx]] - fe[fc["nodes"]])
                r -= mm.fscale[e][fidx] * (fc["lift"] @ jump)
            R[sl] = r
        return R

    def collide(self, f):
        S = self._pts.collide(np.asarray(f, float).reshape(self.shape))[0]
        return S

    def rhs(self, f):
        return self.residual(f) + self.collide(f)

    def rk_step(self, f, dt, scheme=0, nsteps=1):
        """SSP-RK3 (Shu-Osher) or Williamson's three-stage low-storage scheme."""
        f = np.asarray(f, float).reshape(self.shape).copy()
        for _ in range(nsteps):
            if scheme == 0:
                f1 = f + dt * self.rhs(f)
                f2 = 0.75 * f + 0.25 * (f1 + dt * self.rhs(f1))
                f = f / 3.0 + 2.0 / 3.0 * (f2 + dt * self.rhs(f2))
            else:
                A = (0.0, -5.0 / 9.0, -153.0 / 128.0)
                B = (1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0)
                dF = np.zeros_like(f)
                for k in range(3):
                    dF = A[k] * dF + dt * self.rhs(f)
                    f = f + B[k] * dF
        return f

    def moments(self, f):
        """(rho, rho U, E) per point."""
        import oracle as O
        return O.moments(np.asarray(f, float).reshape(self.shape), self.u, self.w)

    def point_weights(self):
        """Integral of each solution point's Lagrange function over its element."""
        mm = self.mm
        return np.concatenate([mm.ref[mm.types[e]].W * mm.detJ[e] for e in range(mm.ne)])

    def totals(self, f):
        Q = self.moments(f)
        return (self.point_weights()[:, None] * Q).sum(0)

    def dt(self, cfl):
        """cfl h_min / ((2p + 1) max_k sum_d |u_kd|), h = element volume over
        its largest face area (the edge length of a cube)."""
        return cfl * self.mm.hmin / ((2 * self.p + 1) * np.abs(self.u).sum(1).max())
