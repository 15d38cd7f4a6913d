"""Python binding of libfrdvm (include/fr_dvm.h): argument marshalling only.

Every computation runs in the HIP kernels of ``libfrdvm.so``; torch tensors
are used only as device memory (their ``data_ptr``) and streams.  There is
no CPU fallback: if the library is missing, importing the binding raises.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfrdvm.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "fr_dvm.h")

BGK, ESBGK, FREE = 0, 1, 2
E_SCRATCH = -5  # FR_DVM_ESCRATCH of fr_dvm.h
MLP_NOALLOC_FLOATS = 1 << 22  # FR_MLP_NOALLOC_FLOATS of fr_dvm_mlp.h
FP64, FP32, FP32_DEV = 0, 1, 2
GUESS_COLD, GUESS_WARM, GUESS_MLP, GUESS_MLP_WARM = 0, 1, 2, 3
MLP_INPUTS = 13  # FR_MLP_INPUTS of fr_dvm_mlp.h
SSPRK3, LSRK3_2N = 0, 1
NEWTON_OK, NEWTON_FALLBACK, NEWTON_NONREAL, NEWTON_ESGUARD = 0, 1, 2, 3


class FrDvmError(RuntimeError):
    pass


class _Mesh(C.Structure):
    _fields_ = [("n_elem", C.c_int32), ("n_nodes", C.c_int32), ("geom_order", C.c_int32),
                ("nodes", C.POINTER(C.c_double)), ("elem_nodes", C.POINTER(C.c_int32)),
                ("nbr_elem", C.POINTER(C.c_int32)), ("nbr_face", C.POINTER(C.c_int8)),
                ("nbr_orient", C.POINTER(C.c_int8)), ("bc", C.POINTER(C.c_int8))]


class _MixedMesh(C.Structure):
    _fields_ = [("n_elem", C.c_int32), ("n_nodes", C.c_int32), ("nodes", C.POINTER(C.c_double)),
                ("elem_type", C.POINTER(C.c_int8)), ("elem_nodes", C.POINTER(C.c_int32)),
                ("nbr_elem", C.POINTER(C.c_int32)), ("nbr_face", C.POINTER(C.c_int8)),
                ("period", C.c_double * 3)]


class _VGrid(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("umin", C.c_double * 3), ("umax", C.c_double * 3)]


class _Params(C.Structure):
    _fields_ = [("model", C.c_int32), ("prandtl", C.c_double), ("mu_ref", C.c_double),
                ("theta_ref", C.c_double), ("omega", C.c_double), ("visc_law", C.c_int32),
                ("theta_s", C.c_double), ("precision", C.c_int32), ("newton_tol", C.c_double),
                ("newton_max_iter", C.c_int32), ("guess", C.c_int32), ("rk", C.c_int32),
                ("farfield", C.c_double * 5), ("theta_wall", C.c_double), ("overlap", C.c_int32),
                ("positivity", C.c_int32)]


_lib = None


def lib():
    """Load the in-tree libfrdvm.so (built by ``paper_2312_06567_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2312_06567_amd.build` "
                              "(there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        vp, dp, i64p = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)
        L.fr_dvm_default_params.argtypes = [C.POINTER(_Params)]
        L.fr_dvm_create.argtypes = [C.POINTER(_Mesh), C.c_int, C.POINTER(_VGrid), C.POINTER(vp)]
        L.fr_dvm_create_nodes.argtypes = [C.POINTER(_Mesh), C.c_int, C.c_int, C.POINTER(_VGrid), C.POINTER(vp)]
        L.fr_dvm_create_gas.argtypes = [C.POINTER(_Mesh), C.c_int, C.c_int, C.c_double, C.POINTER(_VGrid),
                                        C.POINTER(vp)]
        L.fr_dvm_create_mixed.argtypes = [C.POINTER(_MixedMesh), C.c_int, C.POINTER(_VGrid), C.POINTER(vp)]
        L.fr_dvm_set_params.argtypes = [vp, C.POINTER(_Params)]
        L.fr_dvm_set_stream.argtypes = [vp, vp]
        L.fr_dvm_sizes.argtypes = [vp, i64p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                   C.POINTER(C.c_int32), C.POINTER(C.c_size_t)]
        L.fr_dvm_velocity_nodes.argtypes = [vp, dp, dp]
        L.fr_dvm_dt.argtypes = [vp, C.c_double, dp]
        L.fr_dvm_residual.argtypes = [vp, vp, vp]
        L.fr_dvm_collide.argtypes = [vp, vp, vp, vp, C.c_int]
        L.fr_dvm_moments.argtypes = [vp, vp, vp, dp]
        L.fr_dvm_kn_gll.argtypes = [vp, vp, vp]
        L.fr_dvm_rk_step.argtypes = [vp, vp, C.c_double]
        L.fr_dvm_rk_steps.argtypes = [vp, vp, C.c_double, C.c_int]
        L.fr_dvm_newton_stats.argtypes = [vp, i64p, i64p, i64p, i64p, dp, C.c_int]
        L.fr_dvm_newton_points.argtypes = [vp, vp, vp, vp]
        L.fr_dvm_mlp_set_weights.argtypes = [vp, C.POINTER(C.c_float), C.c_size_t]
        L.fr_dvm_equilibrium.argtypes = [vp, vp, C.c_int64, C.c_int, vp, vp, vp, vp, vp]
        L.fr_mlp_param_count.argtypes = [C.c_int]
        L.fr_mlp_param_count.restype = C.c_size_t
        L.fr_mlp_workspace_floats.argtypes = [C.c_int, C.c_int64]
        L.fr_mlp_workspace_floats.restype = C.c_size_t
        L.fr_mlp_forward.argtypes = [C.c_int, vp, vp, C.c_int64, vp, vp, vp]
        L.fr_mlp_forward_noalloc.argtypes = [C.c_int, vp, vp, C.c_int64, vp, vp]
        L.fr_mlp_grad.argtypes = [C.c_int, vp, vp, vp, C.c_int64, vp, vp, vp, vp]
        L.fr_mlp_adam.argtypes = [C.c_int, vp, vp, vp, vp, C.c_int, C.c_float, vp]
        L.fr_dvm_hbm_copy.argtypes = [vp, vp, C.c_size_t, vp]
        L.fr_dvm_profile.argtypes = [vp, C.c_int]
        L.fr_dvm_profile_read.argtypes = [vp, dp, i64p, C.c_int]
        L.fr_dvm_last_error.argtypes = [vp]
        L.fr_dvm_last_error.restype = C.c_char_p
        L.fr_dvm_destroy.argtypes = [vp]
        L.fr_dvm_destroy.restype = None
        _lib = L
    return _lib


HEADERS = [HEADER, os.path.join(os.path.dirname(_HERE), "include", "fr_dvm_mlp.h")]


def header_functions() -> list[str]:
    """Names of the functions declared in include/*.h."""
    names = set()
    for h in HEADERS:
        names |= set(re.findall(r"\b(fr_(?:dvm|mlp)_[a-z0-9_]+)\s*\(", open(h).read()))
    return sorted(names)


def hbm_copy(dst, src, nbytes, stream=None):
    """Plain device-to-device copy kernel of the library (bandwidth probe)."""
    s = getattr(stream, "cuda_stream", stream) or 0
    rc = lib().fr_dvm_hbm_copy(_ptr(dst), _ptr(src), int(nbytes), C.c_void_p(int(s)))
    if rc != 0:
        raise FrDvmError(f"fr_dvm_hbm_copy failed ({rc})")


class Mlp:
    """The learned-guess network's GPU kernels (include/fr_dvm_mlp.h)."""

    def __init__(self, H: int = 64):
        self.H = int(H)
        self.n = int(lib().fr_mlp_param_count(self.H))

    def workspace(self, B: int):
        import torch
        return torch.empty(int(lib().fr_mlp_workspace_floats(self.H, int(B))), dtype=torch.float32, device="cuda")

    def forward(self, w, X, out=None, work=None):
        import torch
        if X.dim() != 2 or X.shape[1] != MLP_INPUTS:
            raise FrDvmError(f"features must be [B, {MLP_INPUTS}]")
        B = X.shape[0]
        out = torch.empty((B, 5), dtype=torch.float32, device="cuda") if out is None else out
        work = self.workspace(B) if work is None else work
        rc = lib().fr_mlp_forward(self.H, _ptr(w), _ptr(X), B, _ptr(out), _ptr(work), None)
        if rc != 0:
            raise FrDvmError(f"fr_mlp_forward failed ({rc})")
        return out

    def forward_noalloc(self, w, X, out, stream=None):
        """Forward pass on the library's fixed per-GPU scratch (no allocation,
        no workspace); ``out`` [B, 5] float32 must be given."""
        if X.dim() != 2 or X.shape[1] != MLP_INPUTS:
            raise FrDvmError(f"features must be [B, {MLP_INPUTS}]")
        s = getattr(stream, "cuda_stream", stream) or 0
        rc = lib().fr_mlp_forward_noalloc(self.H, _ptr(w), _ptr(X), X.shape[0], _ptr(out), C.c_void_p(int(s)))
        if rc != 0:
            raise FrDvmError(f"fr_mlp_forward_noalloc failed ({rc})")
        return out

    def grad(self, w, X, T, grad=None, loss=None, work=None):
        import torch
        if X.dim() != 2 or X.shape[1] != MLP_INPUTS:
            raise FrDvmError(f"features must be [B, {MLP_INPUTS}]")
        B = X.shape[0]
        grad = torch.empty(self.n, dtype=torch.float32, device="cuda") if grad is None else grad
        loss = torch.empty(1, dtype=torch.float32, device="cuda") if loss is None else loss
        work = self.workspace(B) if work is None else work
        rc = lib().fr_mlp_grad(self.H, _ptr(w), _ptr(X), _ptr(T), B, _ptr(grad), _ptr(loss), _ptr(work), None)
        if rc != 0:
            raise FrDvmError(f"fr_mlp_grad failed ({rc})")
        return grad, loss

    def adam(self, w, g, m, v, step, lr):
        rc = lib().fr_mlp_adam(self.H, _ptr(w), _ptr(g), _ptr(m), _ptr(v), int(step), float(lr), None)
        if rc != 0:
            raise FrDvmError(f"fr_mlp_adam failed ({rc})")


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


class FrDvm:
    """One handle of the library: a mesh, an FR order and a velocity grid."""

    def __init__(self, mesh: dict, order: int, grid: dict, params: dict | None = None, nodes: int = 0,
                 delta: float = 0.0):
        """nodes: solution points per axis, 0 Gauss-Legendre, 1 Gauss-Lobatto;
        delta > 0: a gas with delta internal degrees of freedom, state (F, G).
        A mesh with "elem_type" is a mixed mesh (fr_dvm_create_mixed): the
        handle's state is [points][nu] (ne = points, ns = 1)."""
        L = lib()
        g = _VGrid()
        for d in range(3):
            g.n[d] = int(grid["n"][d])
            g.umin[d] = float(grid["umin"][d])
            g.umax[d] = float(grid["umax"][d])
        if "elem_type" in mesh:
            self._keep = {
                "nodes": np.ascontiguousarray(mesh["nodes"], np.float64),
                "elem_type": np.ascontiguousarray(mesh["elem_type"], np.int8),
                "elem_nodes": np.ascontiguousarray(mesh["elem_nodes"], np.int32),
                "nbr_elem": np.ascontiguousarray(mesh["nbr_elem"], np.int32),
                "nbr_face": np.ascontiguousarray(mesh["nbr_face"], np.int8),
            }
            k = self._keep
            m = _MixedMesh(int(mesh["n_elem"]), int(k["nodes"].shape[0]),
                           k["nodes"].ctypes.data_as(C.POINTER(C.c_double)),
                           k["elem_type"].ctypes.data_as(C.POINTER(C.c_int8)),
                           k["elem_nodes"].ctypes.data_as(C.POINTER(C.c_int32)),
                           k["nbr_elem"].ctypes.data_as(C.POINTER(C.c_int32)),
                           k["nbr_face"].ctypes.data_as(C.POINTER(C.c_int8)),
                           (C.c_double * 3)(*[float(x) for x in mesh.get("period", (0.0, 0.0, 0.0))]))
            h = C.c_void_p()
            rc = L.fr_dvm_create_mixed(C.byref(m), int(order), C.byref(g), C.byref(h))
            self._finish(h, rc, order, 1, 0.0, params)
            return
        self._keep = {
            "nodes": np.ascontiguousarray(mesh["nodes"], np.float64),
            "elem_nodes": np.ascontiguousarray(mesh["elem_nodes"], np.int32),
            "nbr_elem": np.ascontiguousarray(mesh["nbr_elem"], np.int32),
            "nbr_face": np.ascontiguousarray(mesh["nbr_face"], np.int8),
            "nbr_orient": np.ascontiguousarray(mesh["nbr_orient"], np.int8),
            "bc": np.ascontiguousarray(mesh["bc"], np.int8),
        }
        k = self._keep
        m = _Mesh(int(mesh["n_elem"]), int(k["nodes"].shape[0]), int(mesh["geom_order"]),
                  k["nodes"].ctypes.data_as(C.POINTER(C.c_double)),
                  k["elem_nodes"].ctypes.data_as(C.POINTER(C.c_int32)),
                  k["nbr_elem"].ctypes.data_as(C.POINTER(C.c_int32)),
                  k["nbr_face"].ctypes.data_as(C.POINTER(C.c_int8)),
                  k["nbr_orient"].ctypes.data_as(C.POINTER(C.c_int8)),
                  k["bc"].ctypes.data_as(C.POINTER(C.c_int8)))
        h = C.c_void_p()
        rc = L.fr_dvm_create_gas(C.byref(m), int(order), int(nodes), float(delta), C.byref(g), C.byref(h))
        self._finish(h, rc, order, nodes, delta, params)

    def _finish(self, h, rc, order, nodes, delta, params):
        L = lib()
        self._h = h
        if rc != 0:
            msg = self.last_error() if h.value else "invalid argument"
            self.destroy()
            raise FrDvmError(f"fr_dvm_create failed ({rc}): {msg}")
        ne, ns, nf, nu = C.c_int64(), C.c_int32(), C.c_int32(), C.c_int32()
        L.fr_dvm_sizes(h, C.byref(ne), C.byref(ns), C.byref(nf), C.byref(nu), None)
        self.ne, self.ns, self.nf, self.nu = ne.value, ns.value, nf.value, nu.value
        self.order = int(order)
        self.nodes = int(nodes)
        self.ncomp = 2 if delta > 0 else 1
        self.precision = FP64
        if params is not None:
            self.set_params(**params)

    # -- plumbing --------------------------------------------------------
    def _check(self, rc, what):
        if rc != 0:
            raise FrDvmError(f"{what} failed ({rc}): {self.last_error()}")

    def last_error(self) -> str:
        if not self._h or not self._h.value:
            return ""
        return lib().fr_dvm_last_error(self._h).decode()

    def destroy(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().fr_dvm_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    @property
    def shape(self):
        return (self.ne, self.ns, self.ncomp * self.nu)

    @property
    def dtype(self):
        import torch
        return torch.float64 if self.precision == FP64 else torch.float32

    def _check_f(self, t, name):
        import torch
        if t is None:
            raise FrDvmError(f"{name} is None")
        if not t.is_cuda or t.dtype != self.dtype or not t.is_contiguous() or t.numel() != self.ne * self.ns * self.ncomp * self.nu:
            raise FrDvmError(f"{name} must be a contiguous {self.dtype} CUDA tensor with {self.shape} elements")

    def _check_d(self, t, n, name):
        import torch
        if t is not None and (not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous() or t.numel() != n):
            raise FrDvmError(f"{name} must be a contiguous float64 CUDA tensor of {n} elements")

    # -- ABI -------------------------------------------------------------
    def set_params(self, **kw):
        p = _Params()
        lib().fr_dvm_default_params(C.byref(p))
        alias = {"prandtl": "prandtl", "Pr": "prandtl"}
        for key, val in kw.items():
            key = alias.get(key, key)
            if key == "farfield":
                for i, v in enumerate(val):
                    p.farfield[i] = float(v)
            elif key in dict(_Params._fields_):
                setattr(p, key, type(getattr(p, key))(val))
            else:
                raise FrDvmError(f"unknown parameter {key}")
        self._check(lib().fr_dvm_set_params(self._h, C.byref(p)), "fr_dvm_set_params")
        self.precision = int(p.precision)
        self.params = {f: (list(getattr(p, f)) if f == "farfield" else getattr(p, f)) for f, _ in _Params._fields_}
        return self

    def set_stream(self, stream):
        s = getattr(stream, "cuda_stream", stream)
        self._check(lib().fr_dvm_set_stream(self._h, C.c_void_p(int(s) if s else 0)), "fr_dvm_set_stream")

    def sizes(self):
        ne, ns, nf, nu, ws = C.c_int64(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_size_t()
        self._check(lib().fr_dvm_sizes(self._h, C.byref(ne), C.byref(ns), C.byref(nf), C.byref(nu),
                                       C.byref(ws)), "fr_dvm_sizes")
        return {"n_elem": ne.value, "ns": ns.value, "nf": nf.value, "nu": nu.value, "workspace_bytes": ws.value}

    def velocity_nodes(self):
        u, w = np.zeros((self.nu, 3)), np.zeros(self.nu)
        self._check(lib().fr_dvm_velocity_nodes(self._h, u.ctypes.data_as(C.POINTER(C.c_double)),
                                                w.ctypes.data_as(C.POINTER(C.c_double))), "velocity_nodes")
        return u, w

    def dt(self, cfl: float) -> float:
        out = C.c_double()
        self._check(lib().fr_dvm_dt(self._h, float(cfl), C.byref(out)), "fr_dvm_dt")
        return out.value

    def residual(self, f, R):
        self._check_f(f, "f")
        self._check_f(R, "R")
        self._check(lib().fr_dvm_residual(self._h, _ptr(f), _ptr(R)), "fr_dvm_residual")
        return R

    def collide(self, f, S, Qp=None, accumulate=False):
        self._check_f(f, "f")
        self._check_f(S, "S")
        self._check_d(Qp, self.ne * self.ns * 5, "Qp")
        self._check(lib().fr_dvm_collide(self._h, _ptr(f), _ptr(S), _ptr(Qp), int(bool(accumulate))),
                    "fr_dvm_collide")
        return S

    def moments(self, f, Q=None, totals=False):
        self._check_f(f, "f")
        self._check_d(Q, self.ne * self.ns * 5, "Q")
        tot = np.zeros(5) if totals else None
        tp = tot.ctypes.data_as(C.POINTER(C.c_double)) if totals else None
        self._check(lib().fr_dvm_moments(self._h, _ptr(f), _ptr(Q), tp), "fr_dvm_moments")
        return tot

    def kn_gll(self, f, kn):
        """Gradient-length local Knudsen number per solution point into kn [e][s] (float64)."""
        self._check_f(f, "f")
        self._check_d(kn, self.ne * self.ns, "kn")
        if kn is None:
            raise FrDvmError("kn must be given")
        self._check(lib().fr_dvm_kn_gll(self._h, _ptr(f), _ptr(kn)), "fr_dvm_kn_gll")
        return kn

    def rk_step(self, f, dt):
        self._check_f(f, "f")
        self._check(lib().fr_dvm_rk_step(self._h, _ptr(f), float(dt)), "fr_dvm_rk_step")
        return f

    def rk_steps(self, f, dt, nsteps):
        self._check_f(f, "f")
        self._check(lib().fr_dvm_rk_steps(self._h, _ptr(f), float(dt), int(nsteps)), "fr_dvm_rk_steps")
        return f

    def newton_stats(self, reset=False):
        hist = np.zeros(64, np.int64)
        nf, ng, ne, mr = C.c_int64(), C.c_int64(), C.c_int64(), C.c_double()
        self._check(lib().fr_dvm_newton_stats(self._h, hist.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(nf),
                                              C.byref(ng), C.byref(ne), C.byref(mr), int(bool(reset))),
                    "fr_dvm_newton_stats")
        return {"hist": hist, "n_fallback": nf.value, "n_guard": ng.value, "n_evals": ne.value,
                "max_resid": mr.value}

    def newton_points(self):
        """Per-point outcome of the most recent Newton solve: status, linear
        solves and final scaled residual, device tensors [n_elem, ns]."""
        import torch
        n = self.ne * self.ns
        st = torch.empty(n, dtype=torch.int32, device="cuda")
        it = torch.empty(n, dtype=torch.int32, device="cuda")
        res = torch.empty(n, dtype=torch.float64, device="cuda")
        self._check(lib().fr_dvm_newton_points(self._h, _ptr(st), _ptr(it), _ptr(res)), "fr_dvm_newton_points")
        return st.view(self.ne, self.ns), it.view(self.ne, self.ns), res.view(self.ne, self.ns)

    def equilibrium(self, Q, guess=GUESS_COLD):
        """FP64 Newton for the conservative equilibria of moment vectors Q[n][5]
        (device float64) on this handle's grid: returns z[n][5], iterations
        (linear solves), evaluations (sum passes), status and final scaled
        residuals (device tensors)."""
        import torch
        n = Q.shape[0]
        self._check_d(Q, n * 5, "Q")
        z = torch.empty((n, 5), dtype=torch.float64, device="cuda")
        it = torch.empty(n, dtype=torch.int32, device="cuda")
        ev = torch.empty(n, dtype=torch.int32, device="cuda")
        st = torch.empty(n, dtype=torch.int32, device="cuda")
        res = torch.empty(n, dtype=torch.float64, device="cuda")
        self._check(lib().fr_dvm_equilibrium(self._h, _ptr(Q), n, int(guess), _ptr(z), _ptr(it), _ptr(ev), _ptr(st),
                                             _ptr(res)), "fr_dvm_equilibrium")
        return z, it, ev, st, res

    def profile(self, enable=True):
        self._check(lib().fr_dvm_profile(self._h, int(bool(enable))), "fr_dvm_profile")

    def profile_read(self, reset=False):
        """Summed HIP-event milliseconds and launch counts per kernel kind:
        stage (fused FR stage), newton, prime, other."""
        ms, n = np.zeros(4), np.zeros(4, np.int64)
        self._check(lib().fr_dvm_profile_read(self._h, ms.ctypes.data_as(C.POINTER(C.c_double)),
                                              n.ctypes.data_as(C.POINTER(C.c_int64)), int(bool(reset))),
                    "fr_dvm_profile_read")
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(("stage", "newton", "prime", "other"))}

    def mlp_set_weights(self, w):
        w = np.ascontiguousarray(w, np.float32)
        self._check(lib().fr_dvm_mlp_set_weights(self._h, w.ctypes.data_as(C.POINTER(C.c_float)), w.size),
                    "fr_dvm_mlp_set_weights")
