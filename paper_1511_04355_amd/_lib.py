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
WARM_NONE, WARM_PREV, WARM_USER, WARM_LEARNED, WARM_MODEL, WARM_EXTRAP, WARM_USER_AUG = 0, 1, 2, 3, 4, 5, 6


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
                ("batch", ctypes.c_int32), ("fault_inject", ctypes.c_uint32), ("profile", ctypes.c_int32),
                ("learn_steps", ctypes.c_int32), ("precond", ctypes.c_int32), ("matrix_free", ctypes.c_int32),
                ("no_graph", ctypes.c_int32), ("hmat_eps", ctypes.c_double), ("hmat_eta", ctypes.c_double),
                ("learn_aug", ctypes.c_int32), ("no_recycle", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("refine_steps", ctypes.c_int32), ("fallback", ctypes.c_int32),
                ("status", ctypes.c_int32), ("rel_res_fp64", ctypes.c_double), ("t_assemble_ms", ctypes.c_double),
                ("t_solve_ms", ctypes.c_double), ("bytes", ctypes.c_double), ("gemv_ms", ctypes.c_double),
                ("gemv64_ms", ctypes.c_double), ("gemv_count", ctypes.c_int32), ("gemv64_count", ctypes.c_int32),
                ("rel_res_start", ctypes.c_double), ("used_net", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("t_far_ms", ctypes.c_double)]


class _AfsParams(ctypes.Structure):
    _fields_ = [("T", ctypes.c_double), ("eta", ctypes.c_double), ("Ns", ctypes.c_int32), ("J0", ctypes.c_int32),
                ("alpha_H", ctypes.c_double), ("alpha_L", ctypes.c_double), ("E1_bar", ctypes.c_double),
                ("E2_bar", ctypes.c_double), ("Jc", ctypes.c_int32), ("max_Nc", ctypes.c_int32),
                ("grid_pts", ctypes.c_int32), ("n_iter", ctypes.c_int32), ("q", ctypes.c_int32)]


_RESPONSE_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                ctypes.POINTER(ctypes.c_double), ctypes.c_void_p)


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
        L.afsbem_mesh_create_quadratic.argtypes = [P, i64, P, i64, P]
        L.afsbem_problem_points.argtypes = [P, P]
        L.afsbem_problem_create.argtypes = [P, P, P, P, P]
        L.afsbem_problem_destroy.argtypes = [P]
        L.afsbem_problem_info.argtypes = [P, P, P, P, P]
        L.afsbem_assemble_device.argtypes = [P, d, d, P, ctypes.c_int, P, P, P, P, P]
        L.afsbem_matvec_device.argtypes = [P, ctypes.c_int, ctypes.c_int, P, P, P, P, P]
        L.afsbem_matvec_device_noalloc.argtypes = [P, ctypes.c_int, ctypes.c_int, P, P, P, P, P]
        L.afsbem_autotune_set.argtypes = [ctypes.c_int]
        L.afsbem_autotune_report.argtypes = [P, i64, P]
        L.afsbem_matvec_free_device.argtypes = [P, d, d, ctypes.c_int, P, P, P, P, P]
        L.afsbem_hmat_matvec_device.argtypes = [P, d, d, d, d, P, P, P, P, P, P]
        L.afsbem_hmat_partition_info.argtypes = [P, P, P, d, P]
        L.afsbem_plan_info.argtypes = [P, P, P, P]
        L.afsbem_solve_opts_default.argtypes = [P]
        L.afsbem_problem_clusters.argtypes = [P, P, P, P]
        L.afsbem_precond_apply_device.argtypes = [P, ctypes.c_int, P, P, P, P, P]
        L.afsbem_solve_device.argtypes = [P, i32, P, P, P, P, P, P, P, P, P]
        L.afsbem_solve.argtypes = [P, i32, P, P, P, P, P, P, P, P]
        L.afsbem_solve_batched_device.argtypes = [i32, P, P, P, P, P, P, P, P, P, P]
        L.afsbem_mlp_n_params.argtypes = [i32, i32, i32, P]
        L.afsbem_mlp_forward.argtypes = [i32, i32, i32, i32, P, P, P, ctypes.c_int, P]
        L.afsbem_mlp_loss_grad.argtypes = [i32, i32, i32, i32, P, P, P, P, P, ctypes.c_int, P]
        L.afsbem_mlp_adam.argtypes = [i64, P, P, P, P, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                      ctypes.c_float, P]
        L.afsbem_mlp_train_step.argtypes = [i32, i32, i32, i32, P, P, P, P, P, i32, ctypes.c_float,
                                            ctypes.c_float, ctypes.c_float, ctypes.c_float, P, P]
        L.afsbem_fsm_grid.argtypes = [d, d, i32, P]
        L.afsbem_fsm_invert.argtypes = [d, d, i32, ctypes.c_int, i64, P, P]
        L.afsbem_vf_fit.argtypes = [i32, P, i32, P, i32, P, i32, d, P, P, P]
        L.afsbem_vf_residues.argtypes = [i32, P, i64, P, i32, P, P]
        L.afsbem_vf_eval.argtypes = [i32, P, i64, P, i32, P, P]
        L.afsbem_vf_eval_time.argtypes = [i32, P, i64, P, i32, P, P]
        L.afsbem_afs_params_default.argtypes = [P]
        L.afsbem_afs_run.argtypes = [P, i32, i32, _RESPONSE_FN, P, P]
        L.afsbem_afs_run_problem.argtypes = [P, P, P, ctypes.c_int, P, i32, i32, P, P]
        L.afsbem_afs_result_info.argtypes = [P, P, P, P, P]
        L.afsbem_afs_result_get.argtypes = [P, P, P, P, P, P, P]
        L.afsbem_afs_result_destroy.argtypes = [P]
        L.afsbem_afs_result_work.argtypes = [P, P]
        L.afsbem_afs_result_status.argtypes = [P, P, P, P]
        L.afsbem_time_synthesis_device.argtypes = [i32, P, i32, P, i64, P, i32, P, P, P]
        L.afsbem_model_sample_device.argtypes = [i32, P, i32, P, i64, P, i32, P, P, P]
        L.afsbem_fsm_invert_device.argtypes = [d, d, i32, ctypes.c_int, i64, P, P, P]
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
    learn_steps: int = 0
    precond: int = 0
    matrix_free: int = 0
    no_graph: int = 0
    hmat_eps: float = 0.0
    hmat_eta: float = 0.0
    learn_aug: int = 0
    no_recycle: int = 0

    def _c(self):
        return _Opts(self.tol, self.restart, self.max_iter, self.precision, self.warm_start, self.inner_tol,
                     self.batch, self.fault_inject, self.profile, self.learn_steps, self.precond, self.matrix_free,
                     self.no_graph, self.hmat_eps, self.hmat_eta, self.learn_aug, self.no_recycle)


class Problem:
    """Mesh + material + boundary-condition kinds + quadrature policy, with the
    s-independent plan uploaded to the current device."""

    def __init__(self, xyz, tri, bc_kind, material=(1.0, 0.25, 1.0), policy=(2.0, 8, 16, 16)):
        L = lib()
        xyz = np.ascontiguousarray(xyz, np.float64)
        tri = np.ascontiguousarray(tri, np.int32)
        kind = np.ascontiguousarray(bc_kind, np.int8)
        # six nodes per element: the Nystrom discretisation, six collocation points per element
        self.quadratic = tri.shape[1] == 6
        self.n_el = int(tri.shape[0])
        self.n_tri = 6 * self.n_el if self.quadratic else self.n_el
        self.N = 3 * self.n_tri
        self.lda = lda_of(self.N)
        mesh = ctypes.c_void_p()
        create = L.afsbem_mesh_create_quadratic if self.quadratic else L.afsbem_mesh_create
        _check(create(xyz.ctypes.data, xyz.shape[0], tri.ctypes.data, tri.shape[0], ctypes.byref(mesh)))
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
        tri = mesh.tri6 if hasattr(mesh, "tri6") else mesh.tri
        return cls(mesh.xyz, tri, mesh.bc_kind, material, policy)

    def points(self):
        """Collocation points (n_tri, 3), unit normals (n_tri, 3), weights (n_tri,)
        (element areas, or w_q J_q of the Nystrom points) and kinds (n_tri,)."""
        out = np.zeros((self.n_tri, 8))
        _check(lib().afsbem_problem_points(self._h, out.ctypes.data))
        return out[:, 0:3], out[:, 3:6], out[:, 6], out[:, 7].astype(np.int8)

    def close(self):
        if getattr(self, "_h", None):
            lib().afsbem_problem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def afs(self, params, bc_shape, dof_idx, K, load_kind=0, opts: "SolveOptions | None" = None):
        """Adaptive frequency sampling driving this problem's GPU solve."""
        bc = np.ascontiguousarray(bc_shape, np.float64)
        idx = np.ascontiguousarray(dof_idx, np.int64)
        c = (opts or SolveOptions())._c()
        r = ctypes.c_void_p()
        _check(lib().afsbem_afs_run_problem(self._h, ctypes.byref(params), bc.ctypes.data, int(load_kind),
                                            idx.ctypes.data, int(K), int(idx.shape[0]), ctypes.byref(c),
                                            ctypes.byref(r)))
        return _afs_result(r, int(idx.shape[0]))

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

    def matvec_noalloc(self, A, A_lo, x, y, fmt=FMT_C128, precision=0):
        """y = A x through afsbem_matvec_device_noalloc (the library allocates
        nothing; the caller passes the output buffer y)."""
        import torch
        x = x.contiguous()
        assert x.dtype == torch.complex128 and x.numel() == self.N and x.is_cuda
        assert y.dtype == torch.complex128 and y.numel() == self.N and y.is_cuda and y.is_contiguous()
        _check(lib().afsbem_matvec_device_noalloc(self._h, int(fmt), int(precision), _ptr(A), _ptr(A_lo), _ptr(x),
                                                  _ptr(y), _stream()))
        return y

    def solve_host(self, s_list, bc_val, opts: SolveOptions | None = None, x0=None):
        """Host-array solve (numpy in, numpy out) through afsbem_solve."""
        opts = opts or SolveOptions()
        s_arr = np.ascontiguousarray(np.stack([np.real(s_list), np.imag(s_list)], axis=1), np.float64)
        ns = s_arr.shape[0]
        bc = np.ascontiguousarray(np.asarray(bc_val, np.complex128).reshape(ns, self.n_tri, 3))
        x0a = None if x0 is None else np.ascontiguousarray(np.asarray(x0, np.complex128).reshape(ns, self.N))
        a = np.zeros((ns, self.N), np.complex128)
        u = np.zeros((ns, self.n_tri, 3), np.complex128)
        t = np.zeros((ns, self.n_tri, 3), np.complex128)
        stats = (_Stats * max(ns, 1))()
        c = opts._c()
        rc = lib().afsbem_solve(self._h, ns, s_arr.ctypes.data, bc.ctypes.data,
                                None if x0a is None else x0a.ctypes.data, a.ctypes.data, u.ctypes.data,
                                t.ctypes.data, ctypes.byref(c), stats)
        _check(rc, allow=(ENOCONV,))
        return {"a": a, "u": u, "t": t, "status": rc,
                "stats": [{f: getattr(stats[k], f) for f, _ in _Stats._fields_} for k in range(ns)]}

    def matvec_free(self, s, x=None, bc_val=None, precision=0):
        """Matrix-free product y = A(s) x and/or b(s) (bc_val given).  Returns (y, b)."""
        import torch
        y = b = None
        if x is not None:
            x = x.contiguous()
            assert x.dtype == torch.complex128 and x.numel() == self.N and x.is_cuda
            y = torch.empty(self.N, dtype=torch.complex128, device="cuda")
        if bc_val is not None:
            bc_val = bc_val.contiguous()
            assert bc_val.dtype == torch.complex128 and bc_val.numel() == self.N and bc_val.is_cuda
            b = torch.empty(self.N, dtype=torch.complex128, device="cuda")
        s = complex(s)
        _check(lib().afsbem_matvec_free_device(self._h, s.real, s.imag, int(precision), _ptr(bc_val), _ptr(x),
                                               _ptr(y), _ptr(b), _stream()))
        return y, b

    def hmat_matvec(self, s, x, eps=1e-5, eta=1.0):
        """y = A_H(s) x with the hierarchical (low-rank far field) form of the
        matrix-free operator.  Returns (y, info) with info = dict(max_rank,
        n_lowrank, n_dense, converged)."""
        import torch
        x = x.contiguous()
        assert x.dtype == torch.complex128 and x.numel() == self.N and x.is_cuda
        y = torch.empty(self.N, dtype=torch.complex128, device="cuda")
        mr, nl, nd = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
        s = complex(s)
        rc = lib().afsbem_hmat_matvec_device(self._h, s.real, s.imag, float(eps), float(eta), _ptr(x), _ptr(y),
                                             ctypes.byref(mr), ctypes.byref(nl), ctypes.byref(nd), _stream())
        _check(rc, allow=(ENOCONV,))
        return y, {"max_rank": mr.value, "n_lowrank": nl.value, "n_dense": nd.value, "converged": rc == 0}

    def clusters(self):
        n = ctypes.c_int64()
        _check(lib().afsbem_problem_clusters(self._h, ctypes.byref(n), None, None))
        ptr = np.zeros(n.value + 1, np.int64)
        elem = np.zeros(self.n_tri, np.int32)
        _check(lib().afsbem_problem_clusters(self._h, ctypes.byref(n), ptr.ctypes.data, elem.ctypes.data))
        return ptr, elem

    def precond_apply(self, A, A_lo, v, fmt=FMT_C128):
        import torch
        v = v.contiguous()
        z = torch.empty_like(v)
        _check(lib().afsbem_precond_apply_device(self._h, int(fmt), _ptr(A), _ptr(A_lo), _ptr(v), _ptr(z), _stream()))
        return z

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


def plan_info(mesh, policy=(2.0, 8, 16, 16)):
    """Sizes of the quadrature plan for a flat or six-node mesh, built on the
    host (no device): points, near pairs, subdivision leaves, clusters."""
    L = lib()
    xyz = np.ascontiguousarray(mesh.xyz, np.float64)
    six = hasattr(mesh, "tri6")
    tri = np.ascontiguousarray(mesh.tri6 if six else mesh.tri, np.int32)
    kind = np.ascontiguousarray(mesh.bc_kind, np.int8)
    m = ctypes.c_void_p()
    create = L.afsbem_mesh_create_quadratic if six else L.afsbem_mesh_create
    _check(create(xyz.ctypes.data, xyz.shape[0], tri.ctypes.data, tri.shape[0], ctypes.byref(m)))
    try:
        out = np.zeros(4, np.int64)
        pol = _Policy(float(policy[0]), int(policy[1]), int(policy[2]), int(policy[3]))
        _check(L.afsbem_plan_info(m, kind.ctypes.data, ctypes.byref(pol), out.ctypes.data))
    finally:
        L.afsbem_mesh_destroy(m)
    return dict(zip(["points", "near_pairs", "leaves", "clusters"], (int(v) for v in out)))


def hmat_partition_info(mesh, eta=1.0, policy=(2.0, 8, 16, 16)):
    """Block partition of the hierarchical operator for a flat mesh, built on
    the host (no device): dict of counts (see afsbem_hmat_partition_info)."""
    L = lib()
    xyz = np.ascontiguousarray(mesh.xyz, np.float64)
    tri = np.ascontiguousarray(mesh.tri, np.int32)
    kind = np.ascontiguousarray(mesh.bc_kind, np.int8)
    m = ctypes.c_void_p()
    _check(L.afsbem_mesh_create(xyz.ctypes.data, xyz.shape[0], tri.ctypes.data, tri.shape[0], ctypes.byref(m)))
    try:
        out = np.zeros(8, np.int64)
        pol = _Policy(float(policy[0]), int(policy[1]), int(policy[2]), int(policy[3]))
        _check(L.afsbem_hmat_partition_info(m, kind.ctypes.data, ctypes.byref(pol), float(eta), out.ctypes.data))
    finally:
        L.afsbem_mesh_destroy(m)
    keys = ["n", "n_dense", "n_lowrank", "pairs_covered", "near_pairs_in_lowrank", "largest_lowrank_side",
            "leaf_elements", "leaf_list_entries"]
    return dict(zip(keys, (int(v) for v in out)))


def solve_batched(problems, s_lists, bc_vals, opts: SolveOptions | None = None, want_ut=False):
    """Lockstep solve of every frequency of every problem (meshes may differ
    in size).  problems: list of Problem; s_lists[p]: its frequencies;
    bc_vals[p]: complex128 cuda [n_s_p, n_tri_p, 3].  Returns a list of dicts
    (a, u, t, stats) per problem and the return code."""
    import torch
    opts = opts or SolveOptions()
    n = len(problems)
    handles = (ctypes.c_void_p * max(n, 1))(*[p._h for p in problems])
    ns = np.array([len(s) for s in s_lists], np.int32)
    s_all = np.concatenate([np.asarray(s, np.complex128).reshape(-1) for s in s_lists]) if n else np.zeros(0)
    s_arr = np.ascontiguousarray(np.stack([s_all.real, s_all.imag], axis=1), np.float64)
    outs, keep = [], []
    for p, s, bc in zip(problems, s_lists, bc_vals):
        bc = bc.contiguous()
        assert bc.dtype == torch.complex128 and bc.numel() == len(s) * p.N and bc.is_cuda
        o = {"a": torch.empty((len(s), p.N), dtype=torch.complex128, device="cuda"), "bc": bc}
        if want_ut:
            o["u"] = torch.empty((len(s), p.n_tri, 3), dtype=torch.complex128, device="cuda")
            o["t"] = torch.empty((len(s), p.n_tri, 3), dtype=torch.complex128, device="cuda")
        outs.append(o)

    def arr(key):
        return (ctypes.c_void_p * max(n, 1))(*[_ptr(o.get(key)) for o in outs])

    total = int(ns.sum())
    stats = (_Stats * max(total, 1))()
    c = opts._c()
    rc = lib().afsbem_solve_batched_device(n, handles, ns.ctypes.data, s_arr.ctypes.data, arr("bc"), arr("a"),
                                           arr("u") if want_ut else None, arr("t") if want_ut else None,
                                           ctypes.byref(c), stats, _stream())
    _check(rc, allow=(ENOCONV,))
    k = 0
    for o, m in zip(outs, ns):
        o.pop("bc")
        o["stats"] = [{f: getattr(stats[k + q], f) for f, _ in _Stats._fields_} for q in range(int(m))]
        k += int(m)
    return outs, rc


def autotune_set(enabled: bool):
    _check(lib().afsbem_autotune_set(int(bool(enabled))))


def autotune_report() -> str:
    n = ctypes.c_int64()
    _check(lib().afsbem_autotune_report(None, 0, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value + 1)
    _check(lib().afsbem_autotune_report(buf, n.value + 1, ctypes.byref(n)))
    return buf.value.decode()


# ------------------------------------------------------------------- drivers
def _c128(a):
    return np.ascontiguousarray(np.asarray(a, np.complex128))


def fsm_grid(P, eta, Ns):
    out = np.zeros(Ns // 2 + 1, np.complex128)
    _check(lib().afsbem_fsm_grid(float(P), float(eta), int(Ns), out.ctypes.data))
    return out


def fsm_invert(P, eta, Ns, H, window=False):
    """H: [n_sig, Ns/2+1] complex -> h: [n_sig, Ns] real at t_n = n P / Ns."""
    H = _c128(np.atleast_2d(H))
    assert H.shape[1] == Ns // 2 + 1
    out = np.zeros((H.shape[0], Ns))
    _check(lib().afsbem_fsm_invert(float(P), float(eta), int(Ns), int(bool(window)), H.shape[0], H.ctypes.data,
                                   out.ctypes.data))
    return out


def vf_fit(s, F, M, n_iter=10, init_poles=None, omega_max=0.0):
    s = _c128(s)
    F = _c128(np.atleast_2d(F))
    K, J = F.shape
    poles = np.zeros(M, np.complex128)
    res = np.zeros((K, M), np.complex128)
    rms = ctypes.c_double()
    ip = None if init_poles is None else _c128(init_poles)
    _check(lib().afsbem_vf_fit(J, s.ctypes.data, K, F.ctypes.data, M, None if ip is None else ip.ctypes.data,
                               int(n_iter), float(omega_max), poles.ctypes.data, res.ctypes.data, ctypes.byref(rms)))
    return poles, res, rms.value


def vf_residues(s, F, poles):
    s, F, poles = _c128(s), _c128(np.atleast_2d(F)), _c128(poles)
    res = np.zeros((F.shape[0], poles.shape[0]), np.complex128)
    _check(lib().afsbem_vf_residues(s.shape[0], s.ctypes.data, F.shape[0], F.ctypes.data, poles.shape[0],
                                    poles.ctypes.data, res.ctypes.data))
    return res


def vf_eval(poles, res, s):
    poles, res, s = _c128(poles), _c128(np.atleast_2d(res)), _c128(s)
    out = np.zeros((res.shape[0], s.shape[0]), np.complex128)
    _check(lib().afsbem_vf_eval(poles.shape[0], poles.ctypes.data, res.shape[0], res.ctypes.data, s.shape[0],
                                s.ctypes.data, out.ctypes.data))
    return out


def vf_eval_time(poles, res, t):
    poles, res = _c128(poles), _c128(np.atleast_2d(res))
    t = np.ascontiguousarray(t, np.float64)
    out = np.zeros((res.shape[0], t.shape[0]))
    _check(lib().afsbem_vf_eval_time(poles.shape[0], poles.ctypes.data, res.shape[0], res.ctypes.data, t.shape[0],
                                     t.ctypes.data, out.ctypes.data))
    return out


def time_synthesis(poles, s, X, t):
    """Time responses h [N, Nt] (float64 cuda) of every column of X [J, N]
    (complex128 cuda samples at s) with the given common poles."""
    import torch
    poles, s = _c128(poles), _c128(s)
    t = np.ascontiguousarray(t, np.float64)
    X = X.contiguous()
    assert X.dtype == torch.complex128 and X.is_cuda and X.shape[0] == s.shape[0]
    N = X.shape[1]
    h = torch.empty((N, t.shape[0]), dtype=torch.float64, device="cuda")
    _check(lib().afsbem_time_synthesis_device(poles.shape[0], poles.ctypes.data, s.shape[0], s.ctypes.data, N,
                                              _ptr(X), t.shape[0], t.ctypes.data, _ptr(h), _stream()))
    return h


def model_sample(poles, s, X, z):
    """Values H [N, n_z] (complex128 cuda) at the complex frequencies z of the
    model of every column of X [J, N] (complex128 cuda samples at s) with the
    given common poles."""
    import torch
    poles, s, z = _c128(poles), _c128(s), _c128(z)
    X = X.contiguous()
    assert X.dtype == torch.complex128 and X.is_cuda and X.shape[0] == s.shape[0]
    N = X.shape[1]
    H = torch.empty((N, z.shape[0]), dtype=torch.complex128, device="cuda")
    _check(lib().afsbem_model_sample_device(poles.shape[0], poles.ctypes.data, s.shape[0], s.ctypes.data, N,
                                            _ptr(X), z.shape[0], z.ctypes.data, _ptr(H), _stream()))
    return H


def fsm_invert_device(P, eta, Ns, H, window=False):
    """H: [n_sig, Ns/2+1] complex128 cuda -> h: [n_sig, Ns] float64 cuda at
    t_n = n P / Ns (the same inversion as fsm_invert, on the GPU)."""
    import torch
    H = H.contiguous()
    assert H.dtype == torch.complex128 and H.is_cuda and H.dim() == 2 and H.shape[1] == Ns // 2 + 1
    h = torch.empty((H.shape[0], Ns), dtype=torch.float64, device="cuda")
    _check(lib().afsbem_fsm_invert_device(float(P), float(eta), int(Ns), int(bool(window)), H.shape[0], _ptr(H),
                                          _ptr(h), _stream()))
    return h


def afs_params(T, eta, Ns, **kw):
    p = _AfsParams()
    _check(lib().afsbem_afs_params_default(ctypes.byref(p)))
    p.T, p.eta, p.Ns = float(T), float(eta), int(Ns)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _afs_result(r, Kt):
    L = lib()
    nc, m, ns, conv = (ctypes.c_int32() for _ in range(4))
    _check(L.afsbem_afs_result_info(r, ctypes.byref(nc), ctypes.byref(m), ctypes.byref(ns), ctypes.byref(conv)))
    s = np.zeros(nc.value, np.complex128)
    F = np.zeros((nc.value, Kt), np.complex128)
    poles = np.zeros(m.value, np.complex128)
    res = np.zeros((Kt, m.value), np.complex128)
    E1 = np.zeros(ns.value)
    E2 = np.zeros(ns.value)
    _check(L.afsbem_afs_result_get(r, s.ctypes.data, F.ctypes.data, poles.ctypes.data, res.ctypes.data,
                                   E1.ctypes.data, E2.ctypes.data))
    mv = ctypes.c_int64()
    _check(L.afsbem_afs_result_work(r, ctypes.byref(mv)))
    capped, unconv, worst = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    _check(L.afsbem_afs_result_status(r, ctypes.byref(capped), ctypes.byref(unconv), ctypes.byref(worst)))
    L.afsbem_afs_result_destroy(r)
    return {"s": s, "F": F, "poles": poles, "residues": res, "E1": E1, "E2": E2, "Nc": nc.value,
            "converged": bool(conv.value), "capped": bool(capped.value), "matvecs": mv.value,
            "unconverged_solves": unconv.value, "worst_rel_res": worst.value}


def afs_run(response, K, Kt, params):
    """AFS with a Python response(s: complex array) -> [len(s), Kt] complex."""
    err = []

    def cb(n, sp, kt, fp, user):
        try:
            sv = np.ctypeslib.as_array(sp, shape=(2 * n,)).view(np.complex128)
            f = np.asarray(response(sv.copy()), np.complex128).reshape(n, kt)
            np.ctypeslib.as_array(fp, shape=(2 * n * kt,))[:] = f.reshape(-1).view(np.float64)
            return 0
        except Exception as e:  # reported through the status code
            err.append(e)
            return 1

    fn = _RESPONSE_FN(cb)
    r = ctypes.c_void_p()
    rc = lib().afsbem_afs_run(ctypes.byref(params), int(K), int(Kt), fn, None, ctypes.byref(r))
    if err:
        raise err[0]
    _check(rc)
    return _afs_result(r, Kt)


# ----------------------------------------------------------------------- MLP
def mlp_n_params(d_in, hidden, d_out):
    n = ctypes.c_int64()
    _check(lib().afsbem_mlp_n_params(d_in, hidden, d_out, ctypes.byref(n)))
    return n.value


def mlp_forward(params, X, d_in, hidden, d_out, mode=1):
    """params: float32 cuda [n_params]; X: float32 cuda [n, d_in] -> Y [n, d_out]."""
    import torch
    X = X.contiguous()
    Y = torch.empty((X.shape[0], d_out), dtype=torch.float32, device="cuda")
    _check(lib().afsbem_mlp_forward(d_in, hidden, d_out, X.shape[0], _ptr(params), _ptr(X), _ptr(Y), int(mode),
                                    _stream()))
    return Y


def mlp_loss_grad(params, X, T, d_in, hidden, d_out, mode=1):
    import torch
    X, T = X.contiguous(), T.contiguous()
    G = torch.empty_like(params)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    _check(lib().afsbem_mlp_loss_grad(d_in, hidden, d_out, X.shape[0], _ptr(params), _ptr(X), _ptr(T), _ptr(G),
                                      _ptr(loss), int(mode), _stream()))
    return loss, G


def mlp_train_step(params, X, T, m, v, t, d_in, hidden, d_out, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One bf16 matrix-core training step (loss, gradient, Adam) in place on
    params, m, v.  Returns the loss before the step (cuda scalar)."""
    import torch
    X, T = X.contiguous(), T.contiguous()
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    _check(lib().afsbem_mlp_train_step(d_in, hidden, d_out, X.shape[0], _ptr(params), _ptr(X), _ptr(T), _ptr(m),
                                       _ptr(v), int(t), lr, beta1, beta2, eps, _ptr(loss), _stream()))
    return loss


def mlp_adam(params, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    _check(lib().afsbem_mlp_adam(params.numel(), _ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(t), lr, beta1,
                                 beta2, eps, _stream()))
