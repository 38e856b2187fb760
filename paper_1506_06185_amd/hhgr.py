"""Python binding of libhhgr.so (the C ABI in include/hhgr.h).

Argument marshalling only: every numerical step runs in the library's HIP
kernels.  PyTorch provides the device memory (the workspace and all vectors)
and the stream; tensors must be CUDA (HIP) tensors of dtype float64.

``lib()`` returns the ctypes library whose functions carry the C names
(``hhgr_create``, ``hhgr_vcycle``, ...); ``Context`` wraps one solver context
with methods named after the C calls without the prefix.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhhgr.so")

HHGR_OK, HHGR_EINVAL, HHGR_ENOMEM, HHGR_EHIP, HHGR_ESTATE, HHGR_ENOCONV = 0, -1, -2, -3, -4, -5
HHGR_FP64, HHGR_MIXED = 0, 1
HHGR_RHS_LOAD, HHGR_RHS_NODAL_F, HHGR_RHS_DIRICHLET = 0, 1, 2
_CODES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ESTATE", -5: "ENOCONV"}


class HHGRError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"hhgr error {_CODES.get(code, code)}: {msg}")
        self.code = code


class Desc(C.Structure):
    _fields_ = [("n_sub", C.c_int), ("level", C.c_int), ("coarse_level", C.c_int), ("nu_pre", C.c_int),
                ("nu_post", C.c_int), ("omega", C.c_double), ("precision", C.c_int),
                ("variable_coeff", C.c_int), ("max_faults", C.c_int), ("general_geometry", C.c_int)]


class Report(C.Structure):
    _fields_ = [("cycles", C.c_int), ("rel_res", C.c_double), ("history", C.POINTER(C.c_double)),
                ("history_cap", C.c_int)]


_lib = None
_vp, _dp, _ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int)


def lib():
    """Load the in-tree library; fails loudly when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1506_06185_amd/build.py "
                          "(or __graft_entry__.build())")
    L = C.CDLL(LIB_PATH)
    sig = {
        "hhgr_desc_default": (None, [C.POINTER(Desc)]),
        "hhgr_workspace_bytes": (C.c_int, [C.POINTER(Desc), C.POINTER(C.c_size_t)]),
        "hhgr_create": (C.c_int, [C.POINTER(Desc), _vp, C.c_size_t, _vp, C.POINTER(_vp)]),
        "hhgr_mesh_workspace_bytes": (C.c_int, [C.POINTER(Desc), C.c_int, _vp, C.c_int, _vp,
                                                C.POINTER(C.c_size_t)]),
        "hhgr_set_fused_sweeps": (C.c_int, [_vp, C.c_int, C.c_int]),
        "hhgr_mesh_boundary": (C.c_int, [_vp, C.POINTER(C.c_longlong), _vp]),
        "hhgr_mesh_set_coeff": (C.c_int, [_vp, _vp]),
        "hhgr_create_mesh": (C.c_int, [C.POINTER(Desc), C.c_int, _vp, C.c_int, _vp, _vp, C.c_size_t, _vp,
                                       C.POINTER(_vp)]),
        "hhgr_destroy": (None, [_vp]),
        "hhgr_sizes": (C.c_int, [_vp, C.POINTER(C.c_longlong), C.POINTER(C.c_int), C.POINTER(C.c_longlong)]),
        "hhgr_set_rhs": (C.c_int, [_vp, _vp, C.c_int]),
        "hhgr_set_coeff": (C.c_int, [_vp, _vp]),
        "hhgr_set_geometry": (C.c_int, [_vp, _dp]),
        "hhgr_set_solution": (C.c_int, [_vp, _vp]),
        "hhgr_get_solution": (C.c_int, [_vp, _vp]),
        "hhgr_vcycle": (C.c_int, [_vp, C.c_int, _dp]),
        "hhgr_solve": (C.c_int, [_vp, C.c_double, C.c_int, C.POINTER(Report)]),
        "hhgr_inject_fault": (C.c_int, [_vp, C.c_int]),
        "hhgr_recover_local": (C.c_int, [_vp, C.c_int, C.c_int, _dp]),
        "hhgr_recover_dn": (C.c_int, [_vp, _ip, C.c_int, C.c_int, C.c_int]),
        "hhgr_recover_dd": (C.c_int, [_vp, _ip, C.c_int, C.c_int, C.c_int]),
        "hhgr_adjoint_grad": (C.c_int, [_vp, _vp, C.c_double, C.c_int, _vp, _vp]),
        "hhgr_mass_apply": (C.c_int, [_vp, _vp, _vp]),
        "hhgr_batch_create": (C.c_int, [C.POINTER(_vp), C.c_int, _vp, C.POINTER(_vp)]),
        "hhgr_batch_run": (C.c_int, [_vp, C.c_double, C.c_int, C.POINTER(Report)]),
        "hhgr_batch_arm_dd": (C.c_int, [_vp, C.c_int, _ip, C.c_int, C.c_int, C.c_int]),
        "hhgr_batch_destroy": (None, [_vp]),
        "hhgr_set_graph": (C.c_int, [_vp, C.c_int]),
        "hhgr_tuning_info": (C.c_int, [_vp, C.c_int, _ip, _ip, _ip]),
        "hhgr_set_tuning": (C.c_int, [_vp, C.c_int, C.c_int, C.c_int, C.c_int]),
        "hhgr_autotune": (C.c_int, [_vp, C.c_char_p]),
        "hhgr_kernel_timing": (C.c_int, [_vp, C.c_int]),
        "hhgr_kernel_stats": (C.c_int, [_vp, C.POINTER(C.c_longlong), _dp, _dp]),
        "hhgr_debug_op": (C.c_int, [_vp, C.c_int, C.c_int, _vp, _vp, _vp]),
        "hhgr_solve_static": (C.c_int, [C.POINTER(Desc), _vp, C.c_int, C.c_double, C.c_int, _vp, C.POINTER(Report),
                                        _vp]),
        "hhgr_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


EXPORTED = ("hhgr_desc_default", "hhgr_workspace_bytes", "hhgr_create", "hhgr_destroy", "hhgr_sizes",
            "hhgr_set_rhs", "hhgr_set_coeff", "hhgr_set_geometry", "hhgr_set_solution", "hhgr_get_solution", "hhgr_vcycle",
            "hhgr_solve", "hhgr_inject_fault", "hhgr_recover_local", "hhgr_recover_dd", "hhgr_recover_dn", "hhgr_adjoint_grad",
            "hhgr_mass_apply", "hhgr_batch_create", "hhgr_batch_run", "hhgr_batch_destroy", "hhgr_batch_arm_dd", "hhgr_set_graph",
            "hhgr_tuning_info", "hhgr_set_tuning",
            "hhgr_autotune", "hhgr_kernel_timing", "hhgr_kernel_stats", "hhgr_debug_op", "hhgr_solve_static",
            "hhgr_mesh_workspace_bytes", "hhgr_create_mesh", "hhgr_set_fused_sweeps", "hhgr_mesh_boundary",
            "hhgr_mesh_set_coeff",
            "hhgr_last_error")


def _check(rc: int, allow=()):
    if rc != HHGR_OK and rc not in allow:
        msg = lib().hhgr_last_error()
        raise HHGRError(rc, msg.decode() if msg else "")
    return rc


def make_desc(n_sub=2, level=7, coarse_level=2, nu_pre=2, nu_post=1, omega=1.25, precision="fp64",
              variable_coeff=False, max_faults=8, general_geometry=False) -> Desc:
    d = Desc()
    lib().hhgr_desc_default(C.byref(d))
    d.n_sub, d.level, d.coarse_level = int(n_sub), int(level), int(coarse_level)
    d.nu_pre, d.nu_post, d.omega = int(nu_pre), int(nu_post), float(omega)
    d.precision = {"fp64": HHGR_FP64, "mixed": HHGR_MIXED}[precision]
    d.variable_coeff = int(bool(variable_coeff))
    d.max_faults = int(max_faults)
    d.general_geometry = int(bool(general_geometry))
    return d


def workspace_bytes(desc: Desc) -> int:
    n = C.c_size_t(0)
    _check(lib().hhgr_workspace_bytes(C.byref(desc), C.byref(n)))
    return int(n.value)


def _mesh_arrays(vertices, tets):
    xyz = np.ascontiguousarray(np.asarray(vertices, dtype=np.float64).reshape(-1, 3))
    tv = np.ascontiguousarray(np.asarray(tets, dtype=np.int32).reshape(-1, 4))
    return xyz, tv


def mesh_workspace_bytes(desc: Desc, vertices, tets) -> int:
    xyz, tv = _mesh_arrays(vertices, tets)
    n = C.c_size_t(0)
    _check(lib().hhgr_mesh_workspace_bytes(C.byref(desc), len(xyz), xyz.ctypes.data, len(tv), tv.ctypes.data,
                                           C.byref(n)))
    return int(n.value)


def _ptr(t: torch.Tensor) -> int:
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("expected a contiguous float64 device tensor")
    return t.data_ptr()


class Context:
    """One solver context; the workspace is a torch uint8 device tensor it keeps alive."""

    def __init__(self, device=None, stream=None, mesh=None, **desc_kw):
        """mesh = (vertices (nv, 3), tets (nt, 4)): an unstructured macro mesh
        (hhgr_create_mesh); otherwise the unit cube of make_desc(**desc_kw)."""
        self.desc = make_desc(**desc_kw)
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.mesh = mesh is not None
        if mesh is not None:
            xyz, tv = _mesh_arrays(*mesh)
            nbytes = mesh_workspace_bytes(self.desc, xyz, tv)
        else:
            nbytes = workspace_bytes(self.desc)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.stream = torch.cuda.current_stream(self.device) if stream is None else stream
        h = _vp()
        if mesh is not None:
            _check(lib().hhgr_create_mesh(C.byref(self.desc), len(xyz), xyz.ctypes.data, len(tv), tv.ctypes.data,
                                          self._ws_ptr, nbytes, self.stream.cuda_stream, C.byref(h)))
        else:
            _check(lib().hhgr_create(C.byref(self.desc), self._ws_ptr, nbytes, self.stream.cuda_stream, C.byref(h)))
        self._h = h
        nd, nt, ne = C.c_longlong(), C.c_int(), C.c_longlong()
        _check(lib().hhgr_sizes(self._h, C.byref(nd), C.byref(nt), C.byref(ne)))
        self.n_dofs, self.n_tets, self.n_elems = int(nd.value), int(nt.value), int(ne.value)
        self.N = self.desc.n_sub << self.desc.level
        self.n_boundary = 0
        if self.mesh:
            nb = C.c_longlong(0)
            _check(lib().hhgr_mesh_boundary(self._h, C.byref(nb), None))
            self.n_boundary = int(nb.value)
        self.workspace_nbytes = nbytes
        # incremented by every call that changes the solution, the operator
        # or the right-hand side (HHGSolve checks it before its backward)
        self.version = 0

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().hhgr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _vec(self):
        return torch.empty(self.n_dofs, dtype=torch.float64, device=self.device)

    def set_rhs(self, vec: torch.Tensor, kind: int = HHGR_RHS_LOAD):
        self.version += 1
        if kind == HHGR_RHS_DIRICHLET:
            want = self.n_boundary if self.mesh else (self.N + 1) ** 3
        else:
            want = self.n_dofs
        if vec.numel() != want:
            raise HHGRError(HHGR_EINVAL, f"right-hand side has {vec.numel()} entries, expected {want}")
        _check(lib().hhgr_set_rhs(self._h, _ptr(vec), int(kind)))
        self._keep_rhs = vec

    def set_coeff(self, k: torch.Tensor):
        self.version += 1
        _check(lib().hhgr_set_coeff(self._h, _ptr(k)))

    def set_geometry(self, vertices):
        """Macro vertex positions ((n+1)^3, 3), x fastest (host array)."""
        import numpy as np

        xyz = np.ascontiguousarray(vertices, dtype=np.float64).reshape(-1)
        if xyz.size != 3 * (self.desc.n_sub + 1) ** 3:
            raise HHGRError(HHGR_EINVAL, f"expected {(self.desc.n_sub + 1) ** 3} vertices, got {xyz.size / 3:g}")
        self.version += 1
        _check(lib().hhgr_set_geometry(self._h, xyz.ctypes.data_as(_dp)))

    def set_solution(self, u: torch.Tensor | None):
        """Initial guess from a device vector in vector order; None sets u = 0."""
        self.version += 1
        _check(lib().hhgr_set_solution(self._h, _ptr(u) if u is not None else None))
        self.stream.synchronize()

    def get_solution(self, out: torch.Tensor | None = None) -> torch.Tensor:
        out = self._vec() if out is None else out
        _check(lib().hhgr_get_solution(self._h, _ptr(out)))
        self.stream.synchronize()
        return out

    def vcycle(self, n: int = 1) -> float:
        self.version += 1
        rel = C.c_double(0.0)
        _check(lib().hhgr_vcycle(self._h, int(n), C.byref(rel)))
        return float(rel.value)

    def solve(self, rel_tol: float = 1e-8, max_cycles: int = 100, raise_on_noconv: bool = True):
        self.version += 1
        import numpy as np

        hist = (C.c_double * (max_cycles + 1))()
        rep = Report(0, 0.0, C.cast(hist, _dp), max_cycles + 1)
        rc = lib().hhgr_solve(self._h, float(rel_tol), int(max_cycles), C.byref(rep))
        _check(rc, allow=() if raise_on_noconv else (HHGR_ENOCONV,))
        return int(rep.cycles), float(rep.rel_res), np.array(hist[: rep.cycles + 1])

    def inject_fault(self, tet: int):
        self.version += 1
        _check(lib().hhgr_inject_fault(self._h, int(tet)))

    def recover_local(self, tet: int, n_cycles: int = 3) -> float:
        self.version += 1
        rel = C.c_double(0.0)
        _check(lib().hhgr_recover_local(self._h, int(tet), int(n_cycles), C.byref(rel)))
        return float(rel.value)

    def recover_dd(self, tets, n_intact: int, n_local: int):
        self.version += 1
        arr = (C.c_int * len(tets))(*[int(t) for t in tets])
        _check(lib().hhgr_recover_dd(self._h, arr, len(tets), int(n_intact), int(n_local)))

    def recover_dn(self, tets, n_intact: int, eta: int = 1):
        """Dirichlet-Neumann recovery (Alg. 2) of faulty tets: n_intact rounds of eta local
        cycles beside one intact Neumann cycle."""
        self.version += 1
        arr = (C.c_int * len(tets))(*[int(t) for t in tets])
        _check(lib().hhgr_recover_dn(self._h, arr, len(tets), int(n_intact), int(eta)))

    def adjoint_grad(self, g: torch.Tensor, rel_tol: float = 1e-13, max_cycles: int = 100, want_k: bool = True):
        dJdf = self._vec()
        # dJ/dk per element on the cube, per macro tetrahedron on a mesh
        nk = self.n_tets if self.mesh else self.n_elems
        dJdk = torch.empty(nk, dtype=torch.float64, device=self.device) if want_k else None
        _check(lib().hhgr_adjoint_grad(self._h, _ptr(g), float(rel_tol), int(max_cycles), _ptr(dJdf),
                                       _ptr(dJdk) if dJdk is not None else None))
        return dJdf, dJdk

    def mass_apply(self, x: torch.Tensor) -> torch.Tensor:
        y = self._vec()
        _check(lib().hhgr_mass_apply(self._h, _ptr(x), _ptr(y)))
        self.stream.synchronize()
        return y

    def set_graph(self, on: bool = True):
        _check(lib().hhgr_set_graph(self._h, int(bool(on))))

    def mesh_boundary(self) -> np.ndarray:
        """Positions (n, 3) of the finest level's boundary nodes of a mesh
        context, in the order HHGR_RHS_DIRICHLET takes the boundary values."""
        n = C.c_longlong(0)
        _check(lib().hhgr_mesh_boundary(self._h, C.byref(n), None))
        xyz = np.empty((int(n.value), 3))
        _check(lib().hhgr_mesh_boundary(self._h, C.byref(n), xyz.ctypes.data))
        return xyz

    def set_mesh_coeff(self, k_tet=None):
        """Coefficient k of eq. (2) constant on each macro tetrahedron of a
        mesh context (host values, one per tetrahedron; None: k = 1)."""
        self.version += 1
        if k_tet is None:
            _check(lib().hhgr_mesh_set_coeff(self._h, None))
            return
        import numpy as np

        if isinstance(k_tet, torch.Tensor):
            k_tet = k_tet.detach().cpu().numpy()
        k = np.ascontiguousarray(np.asarray(k_tet, dtype=np.float64).reshape(-1))
        if k.size != self.n_tets:
            raise ValueError("k_tet needs one value per tetrahedron")
        _check(lib().hhgr_mesh_set_coeff(self._h, k.ctypes.data))

    def set_fused_sweeps(self, level: int, on: bool = True):
        _check(lib().hhgr_set_fused_sweeps(self._h, int(level), int(bool(on))))

    def set_tuning(self, block_size: int = 256, xcd_order: int = 1, nodes_per_thread: int = 1, level: int = 0):
        """Fix the volume-kernel launch shape (level 0 = every level above the coarsest)."""
        _check(lib().hhgr_set_tuning(self._h, level, block_size, xcd_order, nodes_per_thread))

    def autotune(self, cache_path: str | None = None):
        _check(lib().hhgr_autotune(self._h, cache_path.encode() if cache_path else None))

    def tuning_info(self):
        """{level: (workgroup size, XCD-contiguous order, nodes per thread)} for every level above
        the coarsest."""
        out = {}
        for l in range(self.desc.coarse_level + 1, self.desc.level + 1):
            bs, xo, fu = C.c_int(), C.c_int(), C.c_int()
            _check(lib().hhgr_tuning_info(self._h, l, C.byref(bs), C.byref(xo), C.byref(fu)))
            out[l] = (int(bs.value), int(xo.value), int(fu.value))
        return out

    def kernel_timing(self, on: bool = True):
        _check(lib().hhgr_kernel_timing(self._h, int(bool(on))))

    def kernel_stats(self):
        n, ms, by = C.c_longlong(), C.c_double(), C.c_double()
        _check(lib().hhgr_kernel_stats(self._h, C.byref(n), C.byref(ms), C.byref(by)))
        return int(n.value), float(ms.value), float(by.value)


def debug_op(ctx: "Context", op: int, level: int, in0: torch.Tensor, in1: torch.Tensor | None = None):
    """One multigrid operator on one level (see hhgr_debug_op); returns the output vector."""
    n_out_level = level - 1 if op == 4 else level
    N = ctx.desc.n_sub << n_out_level
    # on a mesh context the level's vector fills the front of a finest-level
    # sized buffer (the caller knows the level's length)
    n = ctx.n_dofs if ctx.mesh else (N - 1) ** 3
    out = torch.zeros(n, dtype=torch.float64, device=ctx.device)
    _check(lib().hhgr_debug_op(ctx.handle, int(op), int(level), _ptr(in0), _ptr(in1) if in1 is not None else None,
                               _ptr(out)))
    return out


def solve_static(rhs: torch.Tensor, kind: int = HHGR_RHS_LOAD, rel_tol: float = 1e-8, max_cycles: int = 100,
                 out: torch.Tensor | None = None, stream=None, raise_on_noconv: bool = True, **desc_kw):
    """hhgr_solve_static: a whole solve in the library's static device scratch
    (no workspace).  Returns (u, cycles, rel_res, history)."""
    import numpy as np

    desc = make_desc(**desc_kw)
    N = desc.n_sub << desc.level
    u = torch.empty((N - 1) ** 3, dtype=torch.float64, device=rhs.device) if out is None else out
    stream = torch.cuda.current_stream(rhs.device) if stream is None else stream
    hist = (C.c_double * (max_cycles + 1))()
    rep = Report(0, 0.0, C.cast(hist, _dp), max_cycles + 1)
    rc = lib().hhgr_solve_static(C.byref(desc), _ptr(rhs), int(kind), float(rel_tol), int(max_cycles), _ptr(u),
                                 C.byref(rep), stream.cuda_stream)
    _check(rc, allow=() if raise_on_noconv else (HHGR_ENOCONV,))
    return u, int(rep.cycles), float(rep.rel_res), np.array(hist[: rep.cycles + 1])


class Batch:
    """Concurrent solves of independent contexts (graph branches)."""

    def __init__(self, contexts, stream=None):
        self.contexts = list(contexts)
        self.stream = torch.cuda.current_stream() if stream is None else stream
        arr = (_vp * len(self.contexts))(*[c.handle for c in self.contexts])
        h = _vp()
        _check(lib().hhgr_batch_create(arr, len(self.contexts), self.stream.cuda_stream, C.byref(h)))
        self._h = h

    def arm_dd(self, member: int, tets, n_intact: int, n_local: int):
        """Arm a Dirichlet-Dirichlet recovery of faulty tets of one member for the next run."""
        tets = [int(t) for t in tets]
        arr = (C.c_int * len(tets))(*tets)
        _check(lib().hhgr_batch_arm_dd(self._h, int(member), arr, len(tets), int(n_intact), int(n_local)))

    def run(self, rel_tol: float = 1e-8, max_cycles: int = 100, raise_on_noconv: bool = True):
        import numpy as np

        n = len(self.contexts)
        hists = [(C.c_double * (max_cycles + 1))() for _ in range(n)]
        reps = (Report * n)(*[Report(0, 0.0, C.cast(h, _dp), max_cycles + 1) for h in hists])
        rc = lib().hhgr_batch_run(self._h, float(rel_tol), int(max_cycles), reps)
        _check(rc, allow=() if raise_on_noconv else (HHGR_ENOCONV,))
        return [(int(r.cycles), float(r.rel_res), np.array(h[: r.cycles + 1])) for r, h in zip(reps, hists)]

    def close(self):
        if getattr(self, "_h", None):
            lib().hhgr_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HHGSolve(torch.autograd.Function):
    """u = A(k)^{-1} M f on a context created with variable_coeff=True (k per
    element), or on a mesh context (k per macro tetrahedron).

    forward(ctx_obj, f, k) -> u; backward returns dJ/df = M lambda and
    dJ/dk_T = -lambda^T A_T u with A lambda = dJ/du (adjoint multigrid solve).
    The adjoint reads the context's coefficient and solution, so forward saves
    u and k; if the context was used in between (another forward, a finite-
    difference probe), backward sets them back before the adjoint solve.
    """

    @staticmethod
    def forward(fctx, ctx_obj: Context, f: torch.Tensor, k: torch.Tensor, rel_tol: float = 1e-13,
                max_cycles: int = 100):
        if ctx_obj.mesh:
            ctx_obj.set_mesh_coeff(k)
        else:
            ctx_obj.set_coeff(k.contiguous())
        ctx_obj.set_rhs(f.contiguous(), HHGR_RHS_NODAL_F)
        ctx_obj.set_solution(None)
        ctx_obj.solve(rel_tol, max_cycles)
        u = ctx_obj.get_solution()
        fctx.ctx_obj = ctx_obj
        fctx.rel_tol, fctx.max_cycles = rel_tol, max_cycles
        fctx.version = ctx_obj.version
        fctx.save_for_backward(u, k)
        return u

    @staticmethod
    def backward(fctx, g: torch.Tensor):
        c = fctx.ctx_obj
        u, k = fctx.saved_tensors
        if c.version != fctx.version:
            if c.mesh:
                c.set_mesh_coeff(k)
            else:
                c.set_coeff(k.detach().contiguous())
            c.set_solution(u.detach().contiguous())
            fctx.version = c.version
        dJdf, dJdk = c.adjoint_grad(g.contiguous(), fctx.rel_tol, fctx.max_cycles, want_k=True)
        c.stream.synchronize()
        return None, dJdf, dJdk, None, None
