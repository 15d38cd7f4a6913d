"""FP64 CPU oracle of the FR x conservative-DVM Boltzmann step.

TEST INFRASTRUCTURE.  This package is the plain, slow definition that the GPU
library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import it.  It shares no code with
the HIP library (``paper_2312_06567_amd``) and never imports it.

The arithmetic lives in ``frdvm_oracle.c`` (plain C, long-double velocity
sums, OpenMP over elements / points); this module only marshals numpy arrays
through ctypes.  Section and equation citations are in the C source.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "frdvm_oracle.c")
_LIB = os.path.join(_HERE, "libfrdvm_oracle.so")
_lib = None

NEWTON_OK, NEWTON_FALLBACK, NEWTON_NONREAL, NEWTON_ESGUARD = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile the oracle shared library (gcc, OpenMP, IEEE FP64: no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               _SRC, "-lm", "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_bp = C.POINTER(C.c_int8)


class _Problem(C.Structure):
    _fields_ = [("ne", C.c_int32), ("p", C.c_int32), ("nu", C.c_int32),
                ("u", _dp), ("w", _dp), ("detJ", _dp), ("S", _dp), ("nf", _dp),
                ("nbr_elem", _ip), ("nbr_face", _bp), ("nbr_orient", _bp), ("bc", _bp),
                ("f_inf", _dp), ("theta_w", C.c_double),
                ("model", C.c_int32), ("Pr", C.c_double), ("mu_ref", C.c_double),
                ("theta_ref", C.c_double), ("omega", C.c_double),
                ("visc_law", C.c_int32), ("theta_s", C.c_double),
                ("newton_tol", C.c_double), ("newton_max_iter", C.c_int32), ("nv", C.c_int32 * 3),
                ("nodes", C.c_int32), ("delta", C.c_double), ("ncomp", C.c_int32),
                ("positivity", C.c_int32)]


def _declare(L):
    L.orc_gauss_legendre.argtypes = [C.c_int, _dp, _dp]
    L.orc_fr_ops.argtypes = [C.c_int, _dp, _dp, _dp, _dp, _dp, _dp]
    L.orc_fr_ops_set.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp, _dp, _dp, _dp]
    L.orc_gauss_lobatto.argtypes = [C.c_int, _dp, _dp]
    L.orc_geometry_set.argtypes = [C.c_int, C.c_int, _dp, _ip, C.c_int, C.c_int, _dp, _dp, _dp, _dp]
    L.orc_geometry.argtypes = [C.c_int, C.c_int, _dp, _ip, C.c_int, _dp, _dp, _dp, _dp]
    L.orc_vgrid.argtypes = [_ip, _dp, _dp, _dp, _dp]
    L.orc_moments.argtypes = [C.c_int64, C.c_int, _dp, _dp, _dp, _dp]
    L.orc_pressure_tensor.argtypes = [C.c_int64, C.c_int, _dp, _dp, _dp, _dp]
    L.orc_viscosity.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, C.c_int, C.c_double]
    L.orc_viscosity.restype = C.c_double
    P = C.POINTER(_Problem)
    L.orc_residual.argtypes = [P, _dp, _dp]
    L.orc_collide.argtypes = [P, C.c_int64, _dp, _dp, _dp, _dp, _ip, _ip]
    L.orc_rhs.argtypes = [P, _dp, _dp]
    L.orc_rk_step.argtypes = [P, _dp, C.c_double, C.c_int, C.c_int]
    L.orc_positivity.argtypes = [P, _dp]
    L.orc_totals.argtypes = [P, _dp, _dp]
    L.orc_state_moments.argtypes = [P, C.c_int64, _dp, _dp]
    L.orc_kn_gll.argtypes = [P, _dp, _dp]
    L.orc_dt.argtypes = [P, C.c_double]
    L.orc_dt.restype = C.c_double
    L.orc_num_threads.restype = C.c_int


def _d(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def gauss_legendre(n: int):
    xi, w = np.zeros(n), np.zeros(n)
    assert lib().orc_gauss_legendre(n, _d(xi), _d(w)) == 0
    return xi, w


def gauss_lobatto(n: int):
    xi, w = np.zeros(n), np.zeros(n)
    assert lib().orc_gauss_lobatto(n, _d(xi), _d(w)) == 0
    return xi, w


def fr_ops(p: int, nodes: int = 0) -> dict:
    """1-D FR operators on Gauss-Legendre (nodes 0) or Gauss-Lobatto (1) points."""
    n = p + 1
    o = {k: np.zeros(n) for k in ("xi", "lamL", "lamR", "cM", "cP")}
    o["D"] = np.zeros((n, n))
    assert lib().orc_fr_ops_set(p, nodes, _d(o["xi"]), _d(o["D"]), _d(o["lamL"]), _d(o["lamR"]),
                                _d(o["cM"]), _d(o["cP"])) == 0
    return o


def vgrid(n, umin, umax):
    n = np.ascontiguousarray(n, dtype=np.int32)
    umin, umax = _f64(umin), _f64(umax)
    nu = int(np.prod(n))
    u, w = np.zeros((nu, 3)), np.zeros(nu)
    assert lib().orc_vgrid(n.ctypes.data_as(_ip), _d(umin), _d(umax), _d(u), _d(w)) == 0
    return u, w


def geometry(mesh: dict, p: int, nodes: int = 0) -> dict:
    ne = int(mesh["n_elem"])
    n = p + 1
    ns = n ** 3
    X = _f64(mesh["nodes"])
    en = np.ascontiguousarray(mesh["elem_nodes"], dtype=np.int32)
    g = {"xs": np.zeros((ne, ns, 3)), "detJ": np.zeros((ne, ns)),
         "S": np.zeros((ne, ns, 3, 3)), "nf": np.zeros((ne, 6, n * n, 3))}
    rc = lib().orc_geometry_set(ne, int(mesh["geom_order"]), _d(X), en.ctypes.data_as(_ip), p, int(nodes),
                                _d(g["xs"]), _d(g["detJ"]), _d(g["S"]), _d(g["nf"]))
    if rc != 0:
        raise ValueError("oracle geometry: non-positive Jacobian")
    return g


def moments(f, u, w):
    f = _f64(f)
    nu = f.shape[-1]
    npts = f.size // nu
    Q = np.zeros((npts, 5))
    lib().orc_moments(npts, nu, _d(_f64(u)), _d(_f64(w)), _d(f), _d(Q))
    return Q.reshape(f.shape[:-1] + (5,))


def pressure_tensor(f, u, w):
    f = _f64(f)
    nu = f.shape[-1]
    npts = f.size // nu
    Pi = np.zeros((npts, 6))
    lib().orc_pressure_tensor(npts, nu, _d(_f64(u)), _d(_f64(w)), _d(f), _d(Pi))
    return Pi.reshape(f.shape[:-1] + (6,))


def viscosity(theta, mu_ref, theta_ref=1.0, omega=0.81, law=0, theta_s=0.0):
    return lib().orc_viscosity(theta, mu_ref, theta_ref, omega, law, theta_s)


class Problem:
    """Mesh + order + velocity grid + physics parameters, as plain arrays."""

    @classmethod
    def points_only(cls, grid: dict, params: dict) -> "Problem":
        """A problem on a single periodic p=0 element, for point-wise calls
        (moments, collision) on arbitrary arrays of distributions."""
        import workloads
        return cls(workloads.box_mesh(1), 0, grid, params)

    def __init__(self, mesh: dict, p: int, grid: dict, params: dict):
        self.p = p
        self.n = p + 1
        self.ns = self.n ** 3
        self.ne = int(mesh["n_elem"])
        self.u, self.w = vgrid(grid["n"], grid["umin"], grid["umax"])
        self.nu = self.u.shape[0]
        self.delta = float(params.get("delta", 0.0))
        self.ncomp = 2 if self.delta > 0 else 1
        self.nodes = int(params.get("nodes", 0))
        self.geo = geometry(mesh, p, self.nodes)
        self.nbr_elem = np.ascontiguousarray(mesh["nbr_elem"], dtype=np.int32)
        self.nbr_face = np.ascontiguousarray(mesh["nbr_face"], dtype=np.int8)
        self.nbr_orient = np.ascontiguousarray(mesh["nbr_orient"], dtype=np.int8)
        self.bc = np.ascontiguousarray(mesh["bc"], dtype=np.int8)
        self.params = dict(params)
        fi = params.get("f_inf")
        self.f_inf = _f64(fi) if fi is not None else np.zeros(self.nu * self.ncomp)
        assert self.f_inf.size == self.nu * self.ncomp
        s = _Problem()
        s.ne, s.p, s.nu = self.ne, p, self.nu
        s.u, s.w = _d(self.u), _d(self.w)
        s.detJ, s.S, s.nf = _d(self.geo["detJ"]), _d(self.geo["S"]), _d(self.geo["nf"])
        s.nbr_elem = self.nbr_elem.ctypes.data_as(_ip)
        s.nbr_face = self.nbr_face.ctypes.data_as(_bp)
        s.nbr_orient = self.nbr_orient.ctypes.data_as(_bp)
        s.bc = self.bc.ctypes.data_as(_bp)
        s.f_inf = _d(self.f_inf)
        s.theta_w = float(params.get("theta_wall", 1.0))
        s.model = int(params.get("model", 0))
        s.Pr = float(params.get("prandtl", 1.0))
        s.mu_ref = float(params["mu_ref"])
        s.theta_ref = float(params.get("theta_ref", 1.0))
        s.omega = float(params.get("omega", 0.81))
        s.visc_law = int(params.get("visc_law", 0))
        s.theta_s = float(params.get("theta_s", 0.0))
        s.newton_tol = float(params.get("newton_tol", 1e-13))
        s.newton_max_iter = int(params.get("newton_max_iter", 50))
        for d in range(3):
            s.nv[d] = int(grid["n"][d])
        s.nodes = self.nodes
        s.delta = self.delta
        s.ncomp = self.ncomp
        s.positivity = int(params.get("positivity", 0))
        self._s = s

    @property
    def shape(self):
        return (self.ne, self.ns, self.nu * self.ncomp)

    def residual(self, f):
        f = _f64(f).reshape(self.shape)
        R = np.zeros(self.shape)
        rc = lib().orc_residual(C.byref(self._s), _d(f), _d(R))
        if rc != 0:
            raise ValueError("oracle residual: bad boundary tag")
        return R

    def collide(self, f):
        """Collision source at every point of f[..., nu] (any leading shape).
        Returns S, prim' = (rho', U', theta'), z, status, iterations."""
        f = _f64(f)
        sh = f.shape[:-1]
        nut = self.nu * self.ncomp
        assert f.shape[-1] == nut
        npts = f.size // nut
        S = np.zeros(f.shape)
        prim, z = np.zeros((npts, 5)), np.zeros((npts, 5))
        st, it = np.zeros(npts, np.int32), np.zeros(npts, np.int32)
        lib().orc_collide(C.byref(self._s), npts, _d(f), _d(S), _d(prim), _d(z),
                          st.ctypes.data_as(_ip), it.ctypes.data_as(_ip))
        return S, prim.reshape(sh + (5,)), z.reshape(sh + (5,)), st.reshape(sh), it.reshape(sh)

    def rhs(self, f):
        f = _f64(f).reshape(self.shape)
        L = np.zeros(self.shape)
        lib().orc_rhs(C.byref(self._s), _d(f), _d(L))
        return L

    def rk_step(self, f, dt, scheme=0, nsteps=1):
        f = _f64(f).reshape(self.shape).copy()
        rc = lib().orc_rk_step(C.byref(self._s), _d(f), float(dt), int(scheme), int(nsteps))
        if rc != 0:
            raise RuntimeError(f"oracle rk_step rc={rc}")
        return f

    def positivity(self, f):
        """The positivity limiter applied to a copy of f (every element, every
        state value): nonnegative at solution and flux points, element means
        kept."""
        f = _f64(f).reshape(self.shape).copy()
        if lib().orc_positivity(C.byref(self._s), _d(f)) != 0:
            raise RuntimeError("oracle positivity")
        return f

    def moments(self, f):
        """(rho, rho U, E) per point; E includes the integral of G for the
        reduced pair."""
        f = _f64(f).reshape(self.shape)
        Q = np.zeros(self.shape[:2] + (5,))
        lib().orc_state_moments(C.byref(self._s), self.ne * self.ns, _d(f), _d(Q))
        return Q

    def kn_gll(self, f):
        """Density gradient-length local Knudsen number at every solution
        point, [ne][ns] (Section "Results")."""
        f = _f64(f).reshape(self.shape)
        kn = np.zeros((self.ne, self.ns))
        if lib().orc_kn_gll(C.byref(self._s), _d(f), _d(kn)) != 0:
            raise RuntimeError("oracle kn_gll")
        return kn

    def totals(self, f):
        f = _f64(f).reshape(self.shape)
        t = np.zeros(5)
        lib().orc_totals(C.byref(self._s), _d(f), _d(t))
        return t

    def dt(self, cfl):
        return float(lib().orc_dt(C.byref(self._s), float(cfl)))
