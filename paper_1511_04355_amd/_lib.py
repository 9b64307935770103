"""ctypes binding of libafsbem.so.  Argument marshalling only.

Device buffers are torch tensors on the current HIP device; complex arrays are
complex128 (interleaved re, im doubles) unless stated otherwise.  Calls are
enqueued on ``torch.cuda.current_stream()``.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "libafsbem.so")
_lib = None

OK, EINVAL, ENOMEM, EDEVICE, ENOCONV, EBREAKDOWN, ENAN = 0, -1, -2, -3, -4, -5, -6
FMT_C128, FMT_SPLIT = 0, 1
PREC_FP64, PREC_MIXED = 0, 1
WARM_NONE, WARM_PREV, WARM_USER, WARM_LEARNED = 0, 1, 2, 3


class AfsbemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"afsbem error {code}: {msg}")
        self.code = code


class _Material(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_double), ("nu", ctypes.c_double), ("rho", ctypes.c_double)]


class _Policy(ctypes.Structure):
    _fields_ = [("far_ratio", ctypes.c_double), ("max_subdiv", ctypes.c_int32),
                ("self_n_theta", ctypes.c_int32), ("self_n_rho", ctypes.c_int32)]


class _Opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("warm_start", ctypes.c_int32), ("inner_tol", ctypes.c_double),
                ("batch", ctypes.c_int32), ("fault_inject", ctypes.c_uint32), ("profile", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("refine_steps", ctypes.c_int32), ("fallback", ctypes.c_int32),
                ("status", ctypes.c_int32), ("rel_res_fp64", ctypes.c_double), ("t_assemble_ms", ctypes.c_double),
                ("t_solve_ms", ctypes.c_double), ("bytes", ctypes.c_double), ("gemv_ms", ctypes.c_double),
                ("gemv64_ms", ctypes.c_double), ("gemv_count", ctypes.c_int32), ("gemv64_count", ctypes.c_int32)]


def lib_path() -> str:
    return _LIBPATH


def lib():
    """Load libafsbem.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBPATH):
            raise RuntimeError(f"{_LIBPATH} is missing: build it with `python -m paper_1511_04355_amd.build`")
        L = ctypes.CDLL(_LIBPATH)
        P, i64, i32, d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.afsbem_last_error.restype = ctypes.c_char_p
        L.afsbem_version.argtypes = [P, P]
        L.afsbem_mesh_create.argtypes = [P, i64, P, i64, P]
        L.afsbem_mesh_destroy.argtypes = [P]
        L.afsbem_problem_create.argtypes = [P, P, P, P, P]
        L.afsbem_problem_destroy.argtypes = [P]
        L.afsbem_problem_info.argtypes = [P, P, P, P, P]
        L.afsbem_assemble_device.argtypes = [P, d, d, P, ctypes.c_int, P, P, P, P, P]
        L.afsbem_matvec_device.argtypes = [P, ctypes.c_int, ctypes.c_int, P, P, P, P, P]
        L.afsbem_solve_opts_default.argtypes = [P]
        L.afsbem_solve_device.argtypes = [P, i32, P, P, P, P, P, P, P, P, P]
        _lib = L
    return _lib


def _check(rc, allow=()):
    if rc != OK and rc not in allow:
        raise AfsbemError(rc, lib().afsbem_last_error().decode())
    return rc


def version():
    a, b = ctypes.c_int(), ctypes.c_int()
    _check(lib().afsbem_version(ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def lda_of(N: int) -> int:
    return (N + 63) // 64 * 64


@dataclass
class SolveOptions:
    tol: float = 1e-6
    restart: int = 50
    max_iter: int = 1000
    precision: int = PREC_FP64
    warm_start: int = WARM_NONE
    inner_tol: float = 0.0
    batch: int = 0
    fault_inject: int = 0
    profile: int = 0

    def _c(self):
        return _Opts(self.tol, self.restart, self.max_iter, self.precision, self.warm_start, self.inner_tol,
                     self.batch, self.fault_inject, self.profile)


class Problem:
    """Mesh + material + boundary-condition kinds + quadrature policy, with the
    s-independent plan uploaded to the current device."""

    def __init__(self, xyz, tri, bc_kind, material=(1.0, 0.25, 1.0), policy=(2.0, 8, 16, 16)):
        L = lib()
        xyz = np.ascontiguousarray(xyz, np.float64)
        tri = np.ascontiguousarray(tri, np.int32)
        kind = np.ascontiguousarray(bc_kind, np.int8)
        self.n_tri = int(tri.shape[0])
        self.N = 3 * self.n_tri
        self.lda = lda_of(self.N)
        mesh = ctypes.c_void_p()
        _check(L.afsbem_mesh_create(xyz.ctypes.data, xyz.shape[0], tri.ctypes.data, tri.shape[0],
                                    ctypes.byref(mesh)))
        try:
            mat = _Material(*material)
            pol = None if policy is None else _Policy(float(policy[0]), int(policy[1]), int(policy[2]),
                                                      int(policy[3]))
            h = ctypes.c_void_p()
            _check(L.afsbem_problem_create(mesh, ctypes.byref(mat), kind.ctypes.data,
                                           None if pol is None else ctypes.byref(pol), ctypes.byref(h)))
            self._h = h
        finally:
            L.afsbem_mesh_destroy(mesh)

    @classmethod
    def from_mesh(cls, mesh, material=(1.0, 0.25, 1.0), policy=(2.0, 8, 16, 16)):
        return cls(mesh.xyz, mesh.tri, mesh.bc_kind, material, policy)

    def close(self):
        if getattr(self, "_h", None):
            lib().afsbem_problem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        v = [ctypes.c_int64() for _ in range(4)]
        _check(lib().afsbem_problem_info(self._h, *[ctypes.byref(x) for x in v]))
        return {"n_tri": v[0].value, "n_near_pairs": v[1].value, "n_leaves": v[2].value,
                "self_nodes_per_element": v[3].value}

    # ---------------------------------------------------------- step level
    def alloc_matrix(self, fmt=FMT_C128):
        import torch
        if fmt == FMT_C128:
            return torch.empty((self.N, self.lda), dtype=torch.complex128, device="cuda"), None
        hi = torch.empty((self.N, self.lda), dtype=torch.complex64, device="cuda")
        lo = torch.empty((self.N, self.lda), dtype=torch.complex64, device="cuda")
        return hi, lo

    def assemble(self, s, bc_val, fmt=FMT_C128, A=None, A_lo=None, with_precond=False):
        """A(s), b(s) on the device.  bc_val: complex128 cuda tensor [n_tri, 3].
        Returns (A, A_lo, b, precond); A is [N cols, lda] (column-major)."""
        import torch
        if A is None:
            A, A_lo = self.alloc_matrix(fmt)
        b = torch.empty(self.N, dtype=torch.complex128, device="cuda")
        pc = torch.empty((self.n_tri, 3, 3), dtype=torch.complex128, device="cuda") if with_precond else None
        bc = bc_val.contiguous()
        assert bc.dtype == torch.complex128 and bc.numel() == self.N and bc.is_cuda
        _check(lib().afsbem_assemble_device(self._h, float(np.real(s)), float(np.imag(s)), _ptr(bc), int(fmt),
                                            _ptr(A), _ptr(A_lo), _ptr(b), _ptr(pc), _stream()))
        return A, A_lo, b, pc

    def matvec(self, A, A_lo, x, fmt=FMT_C128, precision=0):
        import torch
        x = x.contiguous()
        assert x.dtype == torch.complex128 and x.numel() == self.N and x.is_cuda
        y = torch.empty(self.N, dtype=torch.complex128, device="cuda")
        _check(lib().afsbem_matvec_device(self._h, int(fmt), int(precision), _ptr(A), _ptr(A_lo), _ptr(x), _ptr(y),
                                          _stream()))
        return y

    # --------------------------------------------------------------- solve
    def solve(self, s_list, bc_val, opts: SolveOptions | None = None, x0=None, want_ut=True, out=None):
        """Solve at every s in s_list.  bc_val: complex128 cuda [n_s, n_tri, 3].
        Returns dict(a, u, t, stats, status)."""
        import torch
        opts = opts or SolveOptions()
        s_arr = np.ascontiguousarray(np.stack([np.real(s_list), np.imag(s_list)], axis=1), np.float64)
        ns = s_arr.shape[0]
        bc = bc_val.contiguous()
        assert bc.dtype == torch.complex128 and bc.numel() == ns * self.N and bc.is_cuda
        if out is None:
            out = {"a": torch.empty((ns, self.N), dtype=torch.complex128, device="cuda")}
            if want_ut:
                out["u"] = torch.empty((ns, self.n_tri, 3), dtype=torch.complex128, device="cuda")
                out["t"] = torch.empty((ns, self.n_tri, 3), dtype=torch.complex128, device="cuda")
        stats = (_Stats * max(ns, 1))()
        c = opts._c()
        rc = lib().afsbem_solve_device(self._h, ns, s_arr.ctypes.data, _ptr(bc), _ptr(x0), _ptr(out.get("a")),
                                       _ptr(out.get("u")), _ptr(out.get("t")), ctypes.byref(c), stats, _stream())
        _check(rc, allow=(ENOCONV,))
        out["status"] = rc
        out["stats"] = [{f: getattr(stats[k], f) for f, _ in _Stats._fields_} for k in range(ns)]
        return out
