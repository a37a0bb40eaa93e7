"""ctypes binding of libd3m.so (names follow include/d3m.h)."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libd3m.so")

if not os.path.exists(library_path):
    raise ImportError(f"{library_path} is missing: build it with "
                      "`python -c 'import __graft_entry__ as g; g.build()'` (hipcc, gfx950)")

# The library and PyTorch exchange device pointers and streams, so the
# process must hold one HIP runtime.  PyTorch ships its own libamdhip64.so.7
# (same soname as the system one the library links): importing torch first
# loads PyTorch's, and the library's dependency then resolves to it.  Loading
# the library first would bind PyTorch to the other runtime instead.
try:
    import torch as _torch  # noqa: F401
except ImportError:  # host-only use without PyTorch
    _torch = None

_lib = C.CDLL(library_path)

FP64 = 0
FP32_IR = 1
KERNEL_IDS = {"update_gemm": 0, "panel": 1, "bunch_kaufman": 2, "assembly": 3, "solve": 4,
              "residual": 5}

_STATUS = {0: "D3M_OK", -1: "D3M_EINVAL", -2: "D3M_ESINGULAR", -3: "D3M_ENOMEM",
           -4: "D3M_EHIP", -5: "D3M_ESTATE", -6: "D3M_ENOCONV", -7: "D3M_ENODEV"}

EXPORT = {"edges": 1, "sub_edges": 2, "sub_ni": 3, "a_coo": 4, "lms": 5, "order": 6,
          "struct": 7, "kd": 8, "kfactor": 9, "lambda": 10}

# symbols declared in include/d3m.h
exported_symbols = ["d3m_default_options", "d3m_setup", "d3m_update_eps", "d3m_factor",
                    "d3m_solve", "d3m_adjoint", "d3m_rhs_planewave", "d3m_probe", "d3m_query",
                    "d3m_destroy", "d3m_last_error", "d3m_set_profile", "d3m_kernel_stats",
                    "d3m_debug_export", "d3m_setup_batch", "d3m_batch_layout", "d3m_rhs_planewave_batch",
                    "d3m_get_tuning", "d3m_set_tuning", "d3m_set_graphs", "d3m_debug_bk", "d3m_factor_growth",
                    "d3m_solve_noalloc", "d3m_rhs_dipole", "d3m_debug_check_schedule",
                    "d3m_debug_chain_wait_limit"]


class d3m_c128(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class d3m_mesh(C.Structure):
    _fields_ = [("n_vertices", C.c_int64), ("xyz", C.POINTER(C.c_double)),
                ("n_tets", C.c_int64), ("tets", C.POINTER(C.c_int64)),
                ("n_pec_faces", C.c_int64), ("pec_faces", C.POINTER(C.c_int64))]


def _mesh(xyz, tets, pec_faces, keep):
    """d3m_mesh over contiguous copies (kept alive in ``keep``)."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    tets = np.ascontiguousarray(tets, dtype=np.int64)
    pec = np.ascontiguousarray(np.zeros((0, 3)) if pec_faces is None else pec_faces, dtype=np.int64)
    if pec.ndim != 2 or pec.shape[1] != 3:
        raise ValueError("pec_faces must be [n][3] vertex ids")
    keep += [xyz, tets, pec]
    return d3m_mesh(xyz.shape[0], _ptr(xyz, C.c_double), tets.shape[0], _ptr(tets, C.c_int64),
                    pec.shape[0], _ptr(pec, C.c_int64) if pec.shape[0] else None)


class d3m_options(C.Structure):
    _fields_ = [("host_only", C.c_int32), ("quad_points", C.c_int32),
                ("ir_max_iter", C.c_int32), ("profile", C.c_int32), ("ir_tol", C.c_double),
                ("use_graph", C.c_int32), ("device", C.c_int32), ("pivot_scope", C.c_int32), ("s1_block", C.c_int32),
                ("pivot_fallback", C.c_int32), ("growth_limit_log10", C.c_int32), ("k_multifrontal", C.c_int32),
                ("s1_order", C.c_int32), ("reserved", C.c_int32 * 2)]


class d3m_info(C.Structure):
    _fields_ = [("n_edges", C.c_int64), ("n_tets", C.c_int64), ("n_subdomains", C.c_int32),
                ("n_blocks", C.c_int32), ("n_lm", C.c_int64), ("max_block", C.c_int32),
                ("n_levels", C.c_int32), ("factor_bytes", C.c_int64), ("device_bytes", C.c_int64),
                ("flops_domain", C.c_double), ("flops_block_ldlt", C.c_double),
                ("flops_update_gemm", C.c_double), ("solve_bytes", C.c_double),
                ("factored", C.c_int32), ("n_units", C.c_int32), ("n_unit_levels", C.c_int32),
                ("n_problems", C.c_int32), ("array_bytes", C.c_int64), ("mfma_flops_update", C.c_double),
                ("bytes_update_gemm", C.c_double), ("solve_vector_bytes", C.c_double),
                ("pivot_scope", C.c_int32), ("pivot_fallbacks", C.c_int32), ("k_multifrontal", C.c_int32),
                ("s1_order", C.c_int32), ("mf_pool_bytes", C.c_double), ("mf_update_bytes", C.c_double),
                ("mf_extend_add_bytes", C.c_double)]


class d3m_batch_item(C.Structure):
    _fields_ = [("mesh", d3m_mesh), ("part", C.POINTER(C.c_int32)), ("eps_r", C.POINTER(C.c_double))]


class d3m_tuning(C.Structure):
    _fields_ = [("s1_block", C.c_int32), ("solve_cols", C.c_int32), ("lookahead_tasks", C.c_int32),
                ("k_block", C.c_int32), ("side_early", C.c_int32), ("k_fuse", C.c_int32),
                ("panel_rows", C.c_int32), ("solve_seq", C.c_int32), ("solve_narrow", C.c_int32),
                ("k_overlap", C.c_int32), ("solve_chain", C.c_int32), ("reserved", C.c_int32 * 1)]


class d3m_bk_out(C.Structure):
    _fields_ = [("L", C.c_void_p), ("d", C.c_void_p), ("doff", C.c_void_p), ("dinv", C.c_void_p),
                ("dinvoff", C.c_void_p), ("kind", C.c_void_p), ("perm", C.c_void_p), ("tt", C.c_void_p),
                ("singular", C.c_void_p)]


class d3m_solve_info(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32), ("residual", C.c_double),
                ("copy_discrepancy", C.c_double)]


_h = C.c_void_p
_lib.d3m_default_options.argtypes = [C.POINTER(d3m_options)]
_lib.d3m_default_options.restype = None
_lib.d3m_setup.argtypes = [C.POINTER(d3m_mesh), C.POINTER(C.c_int32), C.POINTER(C.c_double),
                           C.c_double, d3m_c128, C.POINTER(d3m_options), C.POINTER(_h)]
_lib.d3m_setup_batch.argtypes = [C.POINTER(d3m_batch_item), C.c_int32, C.c_double, d3m_c128,
                                 C.POINTER(d3m_options), C.POINTER(_h)]
_lib.d3m_batch_layout.argtypes = [_h, C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
_lib.d3m_rhs_planewave_batch.argtypes = [_h, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int32,
                                         C.c_void_p]
_lib.d3m_set_graphs.argtypes = [_h, C.c_int]
_lib.d3m_get_tuning.argtypes = [_h, C.POINTER(d3m_tuning)]
_lib.d3m_set_tuning.argtypes = [_h, C.POINTER(d3m_tuning)]
_lib.d3m_update_eps.argtypes = [_h, C.POINTER(C.c_double)]
_lib.d3m_factor.argtypes = [_h, C.c_int, C.c_void_p]
_lib.d3m_solve.argtypes = [_h, C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(d3m_solve_info), C.c_void_p]
_lib.d3m_adjoint.argtypes = [_h, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]
_lib.d3m_rhs_planewave.argtypes = [_h, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int32, C.c_void_p]
_lib.d3m_probe.argtypes = [_h, C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
_lib.d3m_rhs_dipole.argtypes = [_h, C.POINTER(C.c_double), C.c_void_p, C.c_int32, C.c_void_p]
_lib.d3m_debug_check_schedule.argtypes = [_h, C.c_int32, C.c_char_p, C.c_int64]
_lib.d3m_debug_check_schedule.restype = C.c_int64
_lib.d3m_debug_chain_wait_limit.argtypes = [_h, C.c_double]
_lib.d3m_query.argtypes = [_h, C.POINTER(d3m_info)]
_lib.d3m_destroy.argtypes = [_h]
_lib.d3m_destroy.restype = None
_lib.d3m_last_error.restype = C.c_char_p
_lib.d3m_kernel_stats.argtypes = [_h, C.c_int, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                  C.POINTER(C.c_double)]
_lib.d3m_debug_export.argtypes = [_h, C.c_int, C.c_int64, C.c_void_p, C.c_int64]
_lib.d3m_debug_export.restype = C.c_int64
_lib.d3m_set_profile.argtypes = [_h, C.c_int]
_lib.d3m_debug_bk.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int, C.c_int, C.c_int, C.POINTER(d3m_bk_out)]
_lib.d3m_debug_bk.restype = C.c_int
_lib.d3m_factor_growth.argtypes = [_h, C.POINTER(C.c_double), C.POINTER(C.c_double)]
_lib.d3m_factor_growth.restype = C.c_int
_lib.d3m_solve_noalloc.argtypes = [_h, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]
_lib.d3m_solve_noalloc.restype = C.c_int
for _f in ("d3m_setup", "d3m_setup_batch", "d3m_batch_layout", "d3m_rhs_planewave_batch", "d3m_update_eps",
           "d3m_factor", "d3m_solve", "d3m_adjoint", "d3m_rhs_planewave", "d3m_rhs_dipole", "d3m_probe", "d3m_query",
           "d3m_set_profile", "d3m_kernel_stats", "d3m_get_tuning", "d3m_set_tuning", "d3m_set_graphs"):
    getattr(_lib, _f).restype = C.c_int


class D3MError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = _STATUS.get(code, str(code))


def _check(rc):
    if rc != 0:
        raise D3MError(rc, _lib.d3m_last_error().decode())
    return rc


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _stream_handle(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _options(*, host_only=False, profile=False, device=0, quad_points=12, ir_tol=1e-10, ir_max_iter=10,
             pivot_scope=0, s1_block=0, use_graph=False, pivot_fallback=True, growth_limit_log10=0,
             multifrontal=False, s1_order=0):
    opt = d3m_options()
    _lib.d3m_default_options(C.byref(opt))
    opt.host_only = int(host_only)
    # True: every kernel group; an int: that level (0 off, 1 update GEMMs, 2 all)
    opt.profile = 2 if profile is True else int(profile)
    opt.device = int(device)
    opt.quad_points = int(quad_points)
    opt.ir_tol = float(ir_tol)
    opt.ir_max_iter = int(ir_max_iter)
    opt.pivot_scope = int(pivot_scope)
    opt.s1_block = int(s1_block)
    opt.use_graph = int(use_graph)
    opt.pivot_fallback = int(bool(pivot_fallback))
    opt.growth_limit_log10 = int(growth_limit_log10)
    opt.k_multifrontal = int(bool(multifrontal))
    opt.s1_order = int(s1_order)
    return opt


def _check_like(t, ref, name):
    """t must be a contiguous tensor of ref's shape, dtype and device (the
    library writes or reads nrhs * n_edges * 16 bytes through its pointer)."""
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != ref.dtype or tuple(t.shape) != tuple(ref.shape) \
            or t.device != ref.device or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {ref.dtype} tensor of shape {tuple(ref.shape)} "
                         f"on {ref.device}")


def debug_bk(blocks, precision=FP64, variant=0, device=0):
    """Run the library's Bunch-Kaufman kernels on blocks [count, n, n]
    (complex symmetric; d3m_debug_bk).  Returns (status, outputs) where
    outputs holds L, d, doff, dinv, dinvoff, kind, perm, tt, singular as numpy
    arrays; status is 0 or the D3M_ESINGULAR code (other errors raise)."""
    a = np.ascontiguousarray(blocks, dtype=np.complex128)
    if a.ndim == 2:
        a = a[None]
    if a.ndim != 3 or a.shape[1] != a.shape[2]:
        raise ValueError("blocks must be [count, n, n]")
    count, n = a.shape[0], a.shape[1]
    res = {"L": np.zeros((count, n, n), np.complex128), "d": np.zeros((count, n), np.complex128),
           "doff": np.zeros((count, n), np.complex128), "dinv": np.zeros((count, n), np.complex128),
           "dinvoff": np.zeros((count, n), np.complex128), "kind": np.zeros((count, n), np.int32),
           "perm": np.zeros((count, n), np.int32), "tt": np.zeros((count, n, n), np.complex128),
           "singular": np.zeros(count, np.int32)}
    out = d3m_bk_out(*[C.c_void_p(res[k].ctypes.data) for k, _ in d3m_bk_out._fields_])
    if isinstance(precision, str):
        precision = {"fp64": FP64, "fp32_ir": FP32_IR}[precision]
    rc = _lib.d3m_debug_bk(C.c_void_p(a.ctypes.data), n, count, int(precision), int(variant), int(device),
                           C.byref(out))
    if rc not in (0, -2):
        _check(rc)
    return rc, res


class Solver:
    """One decomposed problem, or a batch of independent ones, on the GPU (a
    d3m_handle)."""

    def __init__(self, xyz, tets, part, eps_r, k, alpha, pec_faces=None, **kw):
        keep = []
        part = np.ascontiguousarray(part, dtype=np.int32)
        eps = np.ascontiguousarray(eps_r, dtype=np.float64)
        mesh = _mesh(xyz, tets, pec_faces, keep)
        opt = _options(**kw)
        a = complex(alpha)
        h = _h()
        _check(_lib.d3m_setup(C.byref(mesh), _ptr(part, C.c_int32), _ptr(eps, C.c_double),
                              float(k), d3m_c128(a.real, a.imag), C.byref(opt), C.byref(h)))
        self._adopt(h, k, opt)

    @classmethod
    def batch(cls, problems, k, alpha, **kw):
        """One handle over independent problems (d3m_setup_batch).  problems:
        sequence of objects with xyz, tets, part and eps_r (e.g. Problem)."""
        keep = []
        items = (d3m_batch_item * len(problems))()
        for i, p in enumerate(problems):
            part = np.ascontiguousarray(p.part, dtype=np.int32)
            eps = np.ascontiguousarray(p.eps_r, dtype=np.float64)
            keep += [part, eps]
            items[i].mesh = _mesh(p.xyz, p.tets, getattr(p, "pec_faces", None), keep)
            items[i].part = _ptr(part, C.c_int32)
            items[i].eps_r = _ptr(eps, C.c_double)
        opt = _options(**kw)
        a = complex(alpha)
        h = _h()
        _check(_lib.d3m_setup_batch(items, len(problems), float(k), d3m_c128(a.real, a.imag), C.byref(opt),
                                    C.byref(h)))
        obj = cls.__new__(cls)
        obj._adopt(h, k, opt)
        return obj

    def _adopt(self, h, k, opt):
        self._handle = h
        # bumped whenever the factors held by the handle may change (new
        # eps_r, a factorisation, a re-planned schedule): lets the autograd
        # backward tell whether the factors are still those of its forward
        self.generation = 0
        self.k = float(k)
        self.host_only = bool(opt.host_only)
        self.info = self.query()
        self.n_edges = self.info["n_edges"]
        self.n_tets = self.info["n_tets"]

    @classmethod
    def from_problem(cls, prob, **kw):
        return cls(prob.xyz, prob.tets, prob.part, prob.eps_r, prob.k, prob.alpha,
                   pec_faces=getattr(prob, "pec_faces", None), **kw)

    def close(self):
        if getattr(self, "_handle", None):
            _lib.d3m_destroy(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- steps -------------------------------------------------------------
    def update_eps(self, eps_r):
        eps = np.ascontiguousarray(eps_r, dtype=np.float64)
        if eps.shape != (self.n_tets,):
            raise ValueError(f"eps_r must be float64 [{self.n_tets}]")
        self.generation += 1
        _check(_lib.d3m_update_eps(self._handle, _ptr(eps, C.c_double)))

    def factor(self, precision=FP64, stream=None):
        if isinstance(precision, str):
            precision = {"fp64": FP64, "fp32_ir": FP32_IR}[precision]
        hs = C.c_void_p(0) if self.host_only else _stream_handle(stream)
        self.generation += 1
        _check(_lib.d3m_factor(self._handle, int(precision), hs))

    def solve(self, rhs, out=None, stream=None, with_info=False):
        """E = S^{-1} f for rhs [nrhs, n_edges] complex128 (torch tensor on the
        GPU or host, or a numpy array)."""
        import torch
        if isinstance(rhs, np.ndarray):
            rhs = torch.from_numpy(np.ascontiguousarray(rhs, dtype=np.complex128))
        rhs = rhs.contiguous()
        if rhs.dtype != torch.complex128 or rhs.dim() != 2 or rhs.shape[1] != self.n_edges:
            raise ValueError("rhs must be complex128 [nrhs, n_edges]")
        if out is None:
            out = torch.empty_like(rhs)
        else:
            _check_like(out, rhs, "out")
        info = d3m_solve_info()
        rc = _lib.d3m_solve(self._handle, C.c_void_p(rhs.data_ptr()), rhs.shape[0],
                            C.c_void_p(out.data_ptr()), C.byref(info) if with_info else None,
                            _stream_handle(stream) if rhs.is_cuda else C.c_void_p(0))
        _check(rc)
        if with_info:
            return out, {"iterations": info.iterations, "converged": bool(info.converged),
                         "residual": info.residual, "copy_discrepancy": info.copy_discrepancy}
        return out

    def solve_noalloc(self, rhs, out, stream=None):
        """d3m_solve_noalloc: FP64 solve into a caller tensor, with the
        library's fixed device scratch (rhs and out: contiguous complex128
        CUDA tensors [nrhs, n_edges]).  Enqueues kernels only; no wait."""
        import torch
        if not isinstance(rhs, torch.Tensor) or rhs.dtype != torch.complex128 or rhs.dim() != 2 \
                or rhs.shape[1] != self.n_edges or not rhs.is_cuda or not rhs.is_contiguous():
            raise ValueError("rhs must be a contiguous complex128 CUDA tensor [nrhs, n_edges]")
        _check_like(out, rhs, "out")
        _check(_lib.d3m_solve_noalloc(self._handle, C.c_void_p(rhs.data_ptr()), rhs.shape[0],
                                      C.c_void_p(out.data_ptr()), _stream_handle(stream)))
        return out

    def adjoint(self, grad_E, E, want_w=False, stream=None):
        import torch
        if not isinstance(grad_E, torch.Tensor) or grad_E.dtype != torch.complex128 or grad_E.dim() != 2 \
                or grad_E.shape[1] != self.n_edges:
            raise ValueError("grad_E must be a complex128 tensor [nrhs, n_edges]")
        grad_E = grad_E.contiguous()
        if not isinstance(E, torch.Tensor):
            raise ValueError("E must be a complex128 tensor [nrhs, n_edges]")
        E = E.contiguous()
        _check_like(E, grad_E, "E")
        dev = grad_E.device
        grad = torch.empty(self.n_tets, dtype=torch.float64, device=dev)
        w = torch.empty_like(grad_E) if want_w else None
        _check(_lib.d3m_adjoint(self._handle, C.c_void_p(grad_E.data_ptr()), C.c_void_p(E.data_ptr()),
                                grad_E.shape[0], C.c_void_p(grad.data_ptr()),
                                C.c_void_p(w.data_ptr()) if w is not None else None,
                                _stream_handle(stream) if grad_E.is_cuda else C.c_void_p(0)))
        return (grad, w) if want_w else grad

    def rhs_planewave(self, dirs, pols):
        d = np.ascontiguousarray(np.atleast_2d(dirs), dtype=np.float64)
        p = np.ascontiguousarray(np.atleast_2d(pols), dtype=np.float64)
        f = np.zeros((d.shape[0], self.n_edges), dtype=np.complex128)
        _check(_lib.d3m_rhs_planewave(self._handle, _ptr(d, C.c_double), _ptr(p, C.c_double), d.shape[0],
                                      C.c_void_p(f.ctypes.data)))
        return f

    def check_schedule(self, force_side=False, drop_waits=False):
        """Static race check of the factorisation schedule (no GPU): the
        number of unordered conflicting tile accesses and a description.
        drop_waits plants a missing-wait mistake into the modelled schedule."""
        buf = C.create_string_buffer(8192)
        n = _lib.d3m_debug_check_schedule(self._handle, int(bool(force_side)) | (2 if drop_waits else 0), buf,
                                          len(buf))
        if n < 0:
            _check(int(n))
        return int(n), buf.value.decode()

    def check_solve_chain(self, drop_wait=False):
        """Host simulation of the work-queue K solve sweeps (no GPU): the
        number of violations found and a description.  drop_wait plants a
        missing wait into every item."""
        buf = C.create_string_buffer(8192)
        n = _lib.d3m_debug_check_schedule(self._handle, 4 | (8 if drop_wait else 0), buf, len(buf))
        if n < 0:
            _check(int(n))
        return int(n), buf.value.decode()

    def set_chain_wait_limit(self, seconds):
        """Bound of one dependency wait of the work-queue K solve sweeps
        (seconds; 0 makes every unmet wait run out: failure-path tests)."""
        _check(_lib.d3m_debug_chain_wait_limit(self._handle, C.c_double(seconds)))

    def rhs_dipole(self, pos, moment):
        """Point-dipole loads (impressed currents), one per right-hand side:
        pos [nrhs][3], moment [nrhs][3] complex (current moment I l)."""
        r = np.ascontiguousarray(np.atleast_2d(pos), dtype=np.float64)
        m = np.ascontiguousarray(np.atleast_2d(moment), dtype=np.complex128)
        if r.shape != m.shape or r.shape[1] != 3:
            raise ValueError("pos and moment must both be [nrhs][3]")
        f = np.zeros((r.shape[0], self.n_edges), dtype=np.complex128)
        _check(_lib.d3m_rhs_dipole(self._handle, _ptr(r, C.c_double), C.c_void_p(m.ctypes.data), r.shape[0],
                                   C.c_void_p(f.ctypes.data)))
        return f

    def rhs_planewave_batch(self, dirs, pols):
        """dirs, pols [count][nrhs][3]: each problem of a batch with its own waves."""
        d = np.ascontiguousarray(dirs, dtype=np.float64)
        p = np.ascontiguousarray(pols, dtype=np.float64)
        if d.ndim != 3 or d.shape != p.shape or d.shape[0] != self.layout()[0]:
            raise ValueError("dirs and pols must be [count][nrhs][3]")
        f = np.zeros((d.shape[1], self.n_edges), dtype=np.complex128)
        _check(_lib.d3m_rhs_planewave_batch(self._handle, _ptr(d, C.c_double), _ptr(p, C.c_double), d.shape[1],
                                            C.c_void_p(f.ctypes.data)))
        return f

    def layout(self):
        """(count, edge_off[count + 1], tet_off[count + 1]) of a batch."""
        n = C.c_int32()
        _check(_lib.d3m_batch_layout(self._handle, C.byref(n), None, None))
        eo = np.zeros(n.value + 1, dtype=np.int64)
        to = np.zeros(n.value + 1, dtype=np.int64)
        _check(_lib.d3m_batch_layout(self._handle, None, _ptr(eo, C.c_int64), _ptr(to, C.c_int64)))
        return n.value, eo, to

    def probe(self, points):
        pts = np.ascontiguousarray(np.atleast_2d(points), dtype=np.float64)
        n = pts.shape[0]
        edges = np.zeros((n, 6), dtype=np.int64)
        coef = np.zeros((n, 6, 3), dtype=np.float64)
        _check(_lib.d3m_probe(self._handle, _ptr(pts, C.c_double), n, _ptr(edges, C.c_int64),
                              _ptr(coef, C.c_double)))
        return edges, coef

    def growth(self):
        """(max |L-hat| of step 1, max |L-hat| of -K) of the last factorisation
        (d3m_factor_growth)."""
        a = C.c_double()
        b = C.c_double()
        _check(_lib.d3m_factor_growth(self._handle, C.byref(a), C.byref(b)))
        return a.value, b.value

    def query(self):
        inf = d3m_info()
        _check(_lib.d3m_query(self._handle, C.byref(inf)))
        return {name: getattr(inf, name) for name, _ in d3m_info._fields_ if name not in ("reserved", "pad0")}

    def set_graphs(self, use_graph):
        """Replay captured HIP graphs (True) or launch eagerly (False) from now on."""
        _check(_lib.d3m_set_graphs(self._handle, int(bool(use_graph))))

    TUNING_KEYS = ("s1_block", "solve_cols", "lookahead_tasks", "k_block", "side_early", "k_fuse", "panel_rows",
                   "solve_seq", "solve_narrow", "k_overlap", "solve_chain")

    def tuning(self):
        t = d3m_tuning()
        _check(_lib.d3m_get_tuning(self._handle, C.byref(t)))
        return {k: getattr(t, k) for k in self.TUNING_KEYS}

    def set_tuning(self, **kw):
        """Change launch-shape choices (keys of TUNING_KEYS; 0 = default).  A
        new s1_block, k_block or k_fuse re-plans the factor schedule and
        drops the factors."""
        t = d3m_tuning()
        _check(_lib.d3m_get_tuning(self._handle, C.byref(t)))
        for k, v in kw.items():
            if k not in self.TUNING_KEYS:
                raise KeyError(k)
            setattr(t, k, int(v))
        self.generation += 1
        _check(_lib.d3m_set_tuning(self._handle, C.byref(t)))

    def set_profile(self, level):
        """Profiling level for later calls: 0 off, 1 update GEMMs only, 2 all."""
        _check(_lib.d3m_set_profile(self._handle, int(level)))

    def kernel_stats(self, kernel, reset=False):
        kid = KERNEL_IDS[kernel] if isinstance(kernel, str) else int(kernel)
        n = C.c_int64()
        ms = C.c_double()
        fl = C.c_double()
        _check(_lib.d3m_kernel_stats(self._handle, kid, int(reset), C.byref(n), C.byref(ms), C.byref(fl)))
        return {"launches": n.value, "total_ms": ms.value, "flops": fl.value}

    # ---- host products for parity tests ------------------------------------
    def export(self, what, index=0):
        sel = EXPORT[what]
        nbytes = _lib.d3m_debug_export(self._handle, sel, int(index), None, 0)
        if nbytes < 0:
            _check(int(nbytes))
        buf = np.zeros(int(nbytes), dtype=np.uint8)
        got = _lib.d3m_debug_export(self._handle, sel, int(index), C.c_void_p(buf.ctypes.data), int(nbytes))
        if got < 0:
            _check(int(got))
        if what in ("edges",):
            return buf.view(np.int64).reshape(-1, 2)
        if what in ("sub_edges", "sub_ni"):
            return buf.view(np.int64)
        if what == "a_coo":
            rec = buf.view(np.dtype([("row", "<i8"), ("col", "<i8"), ("re", "<f8"), ("im", "<f8")]))
            return rec["row"].copy(), rec["col"].copy(), rec["re"] + 1j * rec["im"]
        if what == "lms":
            return buf.view(np.int64).reshape(-1, 3)
        if what == "order":
            return buf.view(np.int32).copy()
        if what == "struct":
            a = buf.view(np.int32)
            l = self.info["n_blocks"]
            off = a[:l + 1]
            lst = a[l + 1:]
            return [list(lst[off[j]:off[j + 1]]) for j in range(l)]
        if what == "kd":
            v = buf.view(np.complex128)
            m = int(round(np.sqrt(v.size)))
            return v.reshape(m, m).copy()
        if what == "kfactor":
            n = self.info["n_lm"]
            nu = int(buf[:4].view(np.int32)[0])
            sizes = buf[4:4 + 4 * nu].view(np.int32).copy()
            o = 4 + 4 * nu
            perm = buf[o:o + 4 * n].view(np.int32).copy()
            rest = buf[o + 4 * n:].view(np.complex128)
            return sizes, perm, rest[:n].copy(), rest[n:2 * n].copy(), rest[2 * n:].reshape(n, n).copy()
        if what == "lambda":
            return buf.view(np.complex128).reshape(int(index), -1).copy()
        return buf
