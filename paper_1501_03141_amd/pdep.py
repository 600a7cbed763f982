"""ctypes binding of libpdep.so (include/pdep.h): argument marshalling only.

Every step of the chi0/PDEP path runs in the HIP library.  PyTorch is used only as
plumbing: its caching allocator backs the library's device memory, its current HIP
stream is the stream the library queues on, and torch tensors can be passed as
device-resident inputs and outputs.  Loading fails loudly if the library is missing;
there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import re
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpdep.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "pdep.h")

PDEP_OK = 0
PDEP_EINVAL = -1
PDEP_ENOMEM = -2
PDEP_ENOTCONV = -3
PDEP_EGAP = -4
PDEP_EDEVICE = -5
PDEP_EBUSY = -6
PDEP_ENOTFOUND = -7
PDEP_FP64 = 0
PDEP_MIXED_FP32 = 1
PDEP_MIXED_BF16X3 = 2
PDEP_DEVICE_PTRS = 1
PDEP_CG_GRAPHS = 2

_NAMES = {0: "PDEP_OK", -1: "PDEP_EINVAL", -2: "PDEP_ENOMEM", -3: "PDEP_ENOTCONV", -4: "PDEP_EGAP",
          -5: "PDEP_EDEVICE", -6: "PDEP_EBUSY", -7: "PDEP_ENOTFOUND"}


class PdepError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


class Cell(C.Structure):
    _fields_ = [("L", C.c_double * 3), ("n", C.c_int * 3), ("ecut", C.c_double)]


class Opts(C.Structure):
    _fields_ = [("n_v", C.c_int), ("precision", C.c_int), ("cg_tol", C.c_double), ("cg_maxit", C.c_int),
                ("inner_tol", C.c_double), ("refine_maxit", C.c_int), ("precond", C.c_int),
                ("gap_min", C.c_double), ("gs_tol", C.c_double), ("gs_maxit", C.c_int),
                ("hbm_budget", C.c_size_t), ("rhs_tile", C.c_int), ("stream", C.c_void_p),
                ("alloc", Allocator), ("flags", C.c_uint32)]


class Info(C.Structure):
    _fields_ = [("n_pw", C.c_int), ("n_v", C.c_int), ("n_grid", C.c_int), ("gap", C.c_double),
                ("volume", C.c_double), ("gs_iterations", C.c_int), ("gs_residual", C.c_double)]


class ApplyStats(C.Structure):
    _fields_ = [("n_rhs", C.c_int), ("cg_iter_max", C.c_int), ("cg_iter_total", C.c_longlong),
                ("op_applications", C.c_longlong), ("refine_steps", C.c_int), ("n_notconv", C.c_int),
                ("max_rel_residual", C.c_double), ("ms", C.c_double), ("fft_chunk", C.c_int),
                ("n_fp32_fallback_rows", C.c_int), ("graph_launches", C.c_longlong),
                ("graph_captures", C.c_longlong), ("graph_updates", C.c_longlong)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class EigOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxit", C.c_int), ("max_subspace", C.c_int), ("n_buffer", C.c_int),
                ("reducible", C.c_int), ("scr_tol", C.c_double), ("scr_maxit", C.c_int)]


class EigStats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("chi0_columns", C.c_int), ("max_residual", C.c_double),
                ("cg_iter_total", C.c_longlong), ("ms", C.c_double), ("n_notconv", C.c_int),
                ("scr_passes", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ChibarStats(C.Structure):
    _fields_ = [("passes", C.c_int), ("chi0_columns", C.c_longlong), ("n_notconv", C.c_int),
                ("max_rel_residual", C.c_double), ("cg_iter_total", C.c_longlong), ("cg_notconv", C.c_int),
                ("ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class QpOpts(C.Structure):
    _fields_ = [("n_lanczos", C.c_int), ("n_freq", C.c_int), ("omega0", C.c_double), ("eta", C.c_double),
                ("e_fermi", C.c_double), ("secant_tol", C.c_double), ("secant_maxit", C.c_int),
                ("dE", C.c_double)]


class QpResult(C.Structure):
    _fields_ = [("eps_ks", C.c_double), ("sigma_x", C.c_double), ("sigma_c_ks", C.c_double * 2),
                ("z", C.c_double), ("e_lin", C.c_double), ("e_qp", C.c_double), ("sigma_c_qp", C.c_double * 2),
                ("iterations", C.c_int), ("converged", C.c_int)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["sigma_c_ks"] = complex(self.sigma_c_ks[0], self.sigma_c_ks[1])
        d["sigma_c_qp"] = complex(self.sigma_c_qp[0], self.sigma_c_qp[1])
        return d


class QpStats(C.Structure):
    _fields_ = [("chains", C.c_int), ("max_length", C.c_int), ("h_applications", C.c_longlong),
                ("secant_iterations", C.c_int), ("residue_points", C.c_int), ("ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LanczosStats(C.Structure):
    _fields_ = [("chains", C.c_int), ("max_length", C.c_int), ("h_applications", C.c_longlong),
                ("ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerOpts(C.Structure):
    _fields_ = [("max_running", C.c_int), ("hbm_budget", C.c_size_t), ("queue_capacity", C.c_int),
                ("flags", C.c_uint32), ("fake_ms_per_gb", C.c_double)]


class Job(C.Structure):
    _fields_ = [("cell", Cell), ("vloc", C.c_void_p), ("opts", Opts), ("n_pdep", C.c_int),
                ("seed", C.c_uint64), ("eig", EigOpts)]


class JobResult(C.Structure):
    _fields_ = [("status", C.c_int), ("n_pdep", C.c_int), ("eig_iterations", C.c_int), ("gap", C.c_double),
                ("queue_ms", C.c_double), ("run_ms", C.c_double), ("latency_ms", C.c_double),
                ("hbm_estimate", C.c_size_t)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Chi0Result(C.Structure):
    _fields_ = [("status", C.c_int), ("n_pert", C.c_int), ("batch_requests", C.c_int), ("batch_pert", C.c_int),
                ("queue_ms", C.c_double), ("run_ms", C.c_double), ("latency_ms", C.c_double),
                ("stats", ApplyStats)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "stats"}
        d["stats"] = self.stats.as_dict()
        return d


class ServerStats(C.Structure):
    _fields_ = [("queued", C.c_int), ("running", C.c_int), ("done", C.c_int), ("failed", C.c_int),
                ("committed_bytes", C.c_size_t), ("peak_committed_bytes", C.c_size_t), ("peak_running", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


PDEP_SERVER_FAKE = 1
JOB_QUEUED, JOB_RUNNING, JOB_DONE, JOB_FAILED = 0, 1, 2, 3

_lib = None


def load(path: str = LIB_PATH):
    """Load libpdep.so and declare the signatures.  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built: run `python -c 'import __graft_entry__ as g; g.build()'`")
    # One HIP runtime per process: torch ships its own libamdhip64 / rocBLAS / rocSOLVER
    # with the same sonames as /opt/rocm.  Loading torch first makes the library bind to
    # those already-loaded copies instead of starting a second runtime next to torch's.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    P = C.c_void_p
    D = C.POINTER(C.c_double)
    lib.pdep_default_opts.argtypes = [C.POINTER(Opts)]
    lib.pdep_default_opts.restype = None
    lib.pdep_last_error.argtypes = []
    lib.pdep_last_error.restype = C.c_char_p
    lib.pdep_setup.argtypes = [C.POINTER(Cell), P, C.POINTER(Opts), P, P, C.POINTER(C.c_void_p)]
    lib.pdep_get_info.argtypes = [P, C.POINTER(Info)]
    lib.pdep_get_gvectors.argtypes = [P, C.POINTER(C.c_int), P]
    lib.pdep_get_orbitals.argtypes = [P, P, P]
    lib.chi0_apply.argtypes = [P, C.c_int, P, P, C.POINTER(ApplyStats)]
    lib.chi0_apply_raw.argtypes = [P, C.c_int, P, P, C.POINTER(ApplyStats)]
    lib.chi0_apply_noalloc.argtypes = [P, C.c_int, P, P, C.POINTER(ApplyStats)]
    lib.pdep_eigs.argtypes = [P, C.c_int, C.c_uint64, P, C.POINTER(EigOpts), D, P, C.POINTER(EigStats)]
    lib.chibar_apply.argtypes = [P, C.c_int, P, P, C.c_double, C.c_int, C.POINTER(ChibarStats)]
    lib.pdep_body_lanczos.argtypes = [P, C.c_int, P, C.c_int, C.c_int, D, D, C.POINTER(LanczosStats)]
    lib.pdep_head_wings.argtypes = [P, C.c_int, P, C.c_int, C.c_int, D, D, D, D, D, D, C.POINTER(LanczosStats)]
    lib.pdep_qp_energies.argtypes = [P, C.c_int, P, C.c_int, C.POINTER(C.c_int), D, C.POINTER(QpOpts),
                                     C.POINTER(QpResult), C.c_int, D, D, C.POINTER(QpStats)]
    lib.pdep_destroy.argtypes = [P]
    lib.pdep_profile_enable.argtypes = [C.c_int]
    lib.pdep_profile_enable.restype = C.c_int
    lib.pdep_profile_read.argtypes = [C.c_int, D, C.POINTER(C.c_longlong), D, D, C.c_int]
    lib.pdep_profile_read.restype = C.c_int
    lib.pdep_profile_kernel_name.argtypes = [C.c_int]
    lib.pdep_profile_kernel_name.restype = C.c_char_p
    lib.pdep_profile_set_classes.argtypes = [C.c_uint]
    lib.pdep_profile_set_classes.restype = C.c_int
    lib.pdep_server_create.argtypes = [C.POINTER(ServerOpts), C.POINTER(C.c_void_p)]
    lib.pdep_submit.argtypes = [P, C.POINTER(Job), C.POINTER(C.c_uint64)]
    lib.pdep_poll.argtypes = [P, C.c_uint64, C.POINTER(C.c_int), C.POINTER(JobResult), D, C.c_int]
    lib.pdep_server_wait.argtypes = [P, C.c_uint64, C.c_double, C.POINTER(C.c_int)]
    lib.pdep_server_stats_get.argtypes = [P, C.POINTER(ServerStats)]
    lib.pdep_server_destroy.argtypes = [P]
    lib.pdep_server_add_system.argtypes = [P, C.POINTER(Cell), C.c_void_p, C.POINTER(Opts), C.c_int,
                                           C.POINTER(C.c_uint64)]
    lib.pdep_server_remove_system.argtypes = [P, C.c_uint64]
    lib.pdep_server_system_info.argtypes = [P, C.c_uint64, C.POINTER(Info)]
    lib.pdep_submit_chi0.argtypes = [P, C.c_uint64, C.c_int, C.c_void_p, C.POINTER(C.c_uint64)]
    lib.pdep_poll_chi0.argtypes = [P, C.c_uint64, C.POINTER(C.c_int), C.POINTER(Chi0Result), C.c_void_p, C.c_int]
    lib.pdep_submit_eigs.argtypes = [P, C.c_uint64, C.c_int, C.c_uint64, C.POINTER(EigOpts), C.POINTER(C.c_uint64)]
    lib.pdep_poll_eigs.argtypes = [P, C.c_uint64, C.POINTER(C.c_int), C.POINTER(JobResult), D, C.c_int]
    for name in ("pdep_server_create", "pdep_submit", "pdep_poll", "pdep_server_wait", "pdep_server_stats_get",
                 "pdep_server_destroy", "pdep_server_add_system", "pdep_server_remove_system",
                 "pdep_server_system_info", "pdep_submit_chi0",
                 "pdep_poll_chi0", "pdep_submit_eigs", "pdep_poll_eigs"):
        getattr(lib, name).restype = C.c_int
    for name in ("pdep_setup", "pdep_get_info", "pdep_get_gvectors", "pdep_get_orbitals", "chi0_apply",
                 "chi0_apply_raw", "chi0_apply_noalloc", "chibar_apply", "pdep_body_lanczos", "pdep_head_wings",
                 "pdep_eigs", "pdep_destroy"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def header_functions(path: str = HEADER_PATH):
    """Names of the functions declared in include/pdep.h."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s+\**([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while", "return")))


def _check(code: int, allow=()):
    if code != PDEP_OK and code not in allow:
        msg = _lib.pdep_last_error().decode() if _lib is not None else ""
        raise PdepError(code, msg)
    return code


def profile_enable(on: bool = True):
    _check(load().pdep_profile_enable(1 if on else 0))


def profile_classes(names=None):
    """Time only the named kernel classes (None: all of them)."""
    lib = load()
    if names is None:
        mask = 0xFFFFFFFF
    else:
        idx = {lib.pdep_profile_kernel_name(k).decode(): k for k in range(32)}
        mask = 0
        for n in names:
            if n not in idx:
                raise ValueError(f"unknown kernel class {n!r}")
            mask |= 1 << idx[n]
    _check(lib.pdep_profile_set_classes(C.c_uint(mask)))


def profile_read(reset: bool = True):
    """{kernel class: dict(ms, launches, bytes, flops)} since the last reset."""
    lib = load()
    n = 64
    tot = (C.c_double * n)()
    cnt = (C.c_longlong * n)()
    byt = (C.c_double * n)()
    flo = (C.c_double * n)()
    _check(lib.pdep_profile_read(1 if reset else 0, tot, cnt, byt, flo, n))
    out = {}
    for k in range(n):
        name = lib.pdep_profile_kernel_name(k).decode()
        if not name:
            break
        out[name] = dict(ms=tot[k], launches=cnt[k], bytes=byt[k], flops=flo[k])
    return out


def _torch_allocator():
    import torch

    def alloc(nbytes, _ctx):
        dev = torch.cuda.current_device()
        return torch.cuda.caching_allocator_alloc(int(nbytes), dev, torch.cuda.current_stream(dev))

    def free(ptr, _ctx):
        # a context collected at interpreter shutdown may outlive torch's allocator; the
        # process is ending, so its memory goes with it
        cuda = getattr(torch, "cuda", None)
        if cuda is None or not hasattr(cuda, "caching_allocator_delete"):
            return
        try:
            cuda.caching_allocator_delete(ptr)
        except Exception:
            pass
    a = Allocator(ALLOC_FN(alloc), FREE_FN(free), None)
    return a


class Context:
    """One Kohn-Sham system resident on the GPU (pdep_setup ... pdep_destroy).

    Complex arrays are numpy complex128 (host mode) or torch complex128 CUDA tensors
    (device mode, ``device_ptrs=True``).  PDEP vectors live on S' (G = 0 removed), in
    the library's Miller order (see :meth:`miller`).
    """

    def __init__(self, L, n, ecut, vloc, n_v, precision=PDEP_FP64, cg_tol=1e-10, cg_maxit=2000,
                 inner_tol=1e-5, refine_maxit=8, precond=1, gap_min=1e-3, gs_tol=1e-10, gs_maxit=400,
                 hbm_budget=0, rhs_tile=0, psi=None, eps=None, device_ptrs=False, use_torch=True,
                 cg_graphs=False):
        self._lib = load()
        self._h = C.c_void_p()
        cell = Cell((C.c_double * 3)(*[float(x) for x in L]), (C.c_int * 3)(*[int(x) for x in n]), float(ecut))
        o = Opts()
        self._lib.pdep_default_opts(C.byref(o))
        o.n_v = int(n_v)
        o.precision = int(precision)
        o.cg_tol = float(cg_tol)
        o.cg_maxit = int(cg_maxit)
        o.inner_tol = float(inner_tol)
        o.refine_maxit = int(refine_maxit)
        o.precond = int(precond)
        o.gap_min = float(gap_min)
        o.gs_tol = float(gs_tol)
        o.gs_maxit = int(gs_maxit)
        o.hbm_budget = int(hbm_budget)
        o.rhs_tile = int(rhs_tile)
        o.flags = (PDEP_DEVICE_PTRS if device_ptrs else 0) | (PDEP_CG_GRAPHS if cg_graphs else 0)
        self.device_ptrs = bool(device_ptrs)
        self._alloc = None
        if use_torch:
            import torch
            if not torch.cuda.is_available():
                raise RuntimeError("no GPU visible to torch")
            self._alloc = _torch_allocator()
            o.alloc = self._alloc
            o.stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        v = np.ascontiguousarray(np.asarray(vloc, dtype=np.float64).ravel())
        psi_p = eps_p = None
        if psi is not None:
            psi_a = np.ascontiguousarray(np.asarray(psi, dtype=np.complex128))
            eps_a = np.ascontiguousarray(np.asarray(eps, dtype=np.float64))
            psi_p, eps_p = psi_a.ctypes.data, eps_a.ctypes.data
        self._opts = o
        _check(self._lib.pdep_setup(C.byref(cell), v.ctypes.data, C.byref(o), psi_p, eps_p, C.byref(self._h)))
        info = Info()
        _check(self._lib.pdep_get_info(self._h, C.byref(info)))
        self.n_pw = info.n_pw
        self.n_v = info.n_v
        self.n_grid = info.n_grid
        self.gap = info.gap
        self.volume = info.volume
        self.gs_iterations = info.gs_iterations
        self.gs_residual = info.gs_residual

    # --------------------------------------------------------------------------------
    def miller(self) -> np.ndarray:
        n = C.c_int()
        _check(self._lib.pdep_get_gvectors(self._h, C.byref(n), None))
        m = np.empty((n.value, 3), dtype=np.int32)
        _check(self._lib.pdep_get_gvectors(self._h, None, m.ctypes.data))
        return m

    def orbitals(self):
        eps = np.empty(self.n_v, dtype=np.float64)
        psi = np.empty((self.n_v, self.n_pw), dtype=np.complex128)
        _check(self._lib.pdep_get_orbitals(self._h, eps.ctypes.data, psi.ctypes.data))
        return eps, psi

    def _ptr(self, a, dtype, shape, out=False):
        if self.device_ptrs:
            import torch
            if not (isinstance(a, torch.Tensor) and a.is_cuda and a.is_contiguous()):
                raise TypeError("device mode expects a contiguous CUDA tensor")
            want = torch.complex128 if dtype == np.complex128 else torch.float64
            if a.dtype != want or tuple(a.shape) != tuple(shape):
                raise TypeError(f"expected {want} tensor of shape {shape}, got {a.dtype} {tuple(a.shape)}")
            return a.data_ptr(), a
        arr = np.ascontiguousarray(np.asarray(a, dtype=dtype))
        if arr.shape != tuple(shape):
            raise ValueError(f"expected shape {shape}, got {arr.shape}")
        return arr.ctypes.data, arr

    def _new(self, dtype, shape):
        if self.device_ptrs:
            import torch
            return torch.empty(shape, dtype=torch.complex128 if dtype == np.complex128 else torch.float64,
                               device="cuda")
        return np.empty(shape, dtype=dtype)

    def chi0_apply(self, phi, out=None, allow_notconv=False):
        """chi0bar applied to the rows of phi [n_pert, N_pw - 1]; returns (result, stats)."""
        n_pert = int(phi.shape[0])
        shape = (n_pert, self.n_pw - 1)
        p, keep = self._ptr(phi, np.complex128, shape)
        if out is None:
            out = self._new(np.complex128, shape)
        o, keep_o = self._ptr(out, np.complex128, shape, out=True)
        st = ApplyStats()
        _check(self._lib.chi0_apply(self._h, n_pert, p, o, C.byref(st)),
               allow=(PDEP_ENOTCONV,) if allow_notconv else ())
        return (keep_o if not self.device_ptrs else out), st.as_dict()

    def chi0_apply_noalloc(self, phi, out=None, allow_notconv=False):
        """chi0_apply through the entry point that allocates no device memory."""
        n_pert = int(phi.shape[0])
        shape = (n_pert, self.n_pw - 1)
        p, keep = self._ptr(phi, np.complex128, shape)
        if out is None:
            out = self._new(np.complex128, shape)
        o, keep_o = self._ptr(out, np.complex128, shape, out=True)
        st = ApplyStats()
        _check(self._lib.chi0_apply_noalloc(self._h, n_pert, p, o, C.byref(st)),
               allow=(PDEP_ENOTCONV,) if allow_notconv else ())
        return (keep_o if not self.device_ptrs else out), st.as_dict()

    def chi0_apply_raw(self, dv, allow_notconv=False):
        """Density response (real grids [n_pert, N_g]) to real grid potentials dv."""
        n_pert = int(dv.shape[0])
        shape = (n_pert, self.n_grid)
        p, keep = self._ptr(dv, np.float64, shape)
        out = self._new(np.float64, shape)
        o, keep_o = self._ptr(out, np.float64, shape, out=True)
        st = ApplyStats()
        _check(self._lib.chi0_apply_raw(self._h, n_pert, p, o, C.byref(st)),
               allow=(PDEP_ENOTCONV,) if allow_notconv else ())
        return (keep_o if not self.device_ptrs else out), st.as_dict()

    def chibar_apply(self, phi, tol=1e-9, maxit=200, out=None, allow_notconv=False):
        """The reducible chibar (Hartree-only self-consistent response) applied to the rows
        of phi [n_pert, N_pw - 1]; returns (result, stats)."""
        n_pert = int(phi.shape[0])
        shape = (n_pert, self.n_pw - 1)
        p, keep = self._ptr(phi, np.complex128, shape)
        if out is None:
            out = self._new(np.complex128, shape)
        o, keep_o = self._ptr(out, np.complex128, shape, out=True)
        st = ChibarStats()
        _check(self._lib.chibar_apply(self._h, n_pert, p, o, float(tol), int(maxit), C.byref(st)),
               allow=(PDEP_ENOTCONV,) if allow_notconv else ())
        return (keep_o if not self.device_ptrs else out), st.as_dict()

    def body_lanczos(self, phi, freq, n_lanczos=40):
        """The body of chi0bar at the imaginary frequencies freq in the basis phi
        [n_pert, N_pw - 1] by deflated Lanczos chains: (body [n_freq, n_pert, n_pert], stats)."""
        n_pert = int(phi.shape[0])
        p, keep = self._ptr(phi, np.complex128, (n_pert, self.n_pw - 1))
        f = np.ascontiguousarray(np.asarray(freq, dtype=np.float64).ravel())
        body = np.empty((f.size, n_pert, n_pert), dtype=np.float64)
        st = LanczosStats()
        _check(self._lib.pdep_body_lanczos(self._h, n_pert, p, int(n_lanczos), int(f.size),
                                           f.ctypes.data_as(C.POINTER(C.c_double)),
                                           body.ctypes.data_as(C.POINTER(C.c_double)), C.byref(st)))
        return body, st.as_dict()

    def head_wings(self, phi, freq, n_lanczos=40, allow_notconv=False):
        """Head F [nf, 3, 3], wings U [nf, 3, n], body B [nf, n, n], Lambda [nf, n, n]
        and Xi [nf] at the imaginary frequencies freq (q -> 0), and the stats."""
        n = int(phi.shape[0])
        p, keep = self._ptr(phi, np.complex128, (n, self.n_pw - 1))
        f = np.ascontiguousarray(np.asarray(freq, dtype=np.float64).ravel())
        nf = f.size
        out = dict(F=np.empty((nf, 3, 3)), U=np.empty((nf, 3, n)), B=np.empty((nf, n, n)),
                   Lambda=np.empty((nf, n, n)), Xi=np.empty(nf))
        dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))  # noqa: E731
        st = LanczosStats()
        _check(self._lib.pdep_head_wings(self._h, n, p, int(n_lanczos), nf, dp(f), dp(out["F"]), dp(out["U"]),
                                         dp(out["B"]), dp(out["Lambda"]), dp(out["Xi"]), C.byref(st)),
               allow=(PDEP_ENOTCONV,) if allow_notconv else ())
        return out, st.as_dict()

    def qp_energies(self, phi, states, vxc=None, energies=None, n_lanczos=40, n_freq=64, omega0=0.5,
                    eta=1e-3, e_fermi=0.0, secant_tol=1e-8, secant_maxit=40, dE=1e-3, allow_notconv=False):
        """G0W0 quasiparticle energies of the occupied `states` with W_p in the basis phi:
        ([dict per state], Sigma_C at `energies` [n_states, n_e] complex or None, stats)."""
        n = int(phi.shape[0])
        p, keep = self._ptr(phi, np.complex128, (n, self.n_pw - 1))
        st_idx = np.ascontiguousarray(np.asarray(states, dtype=np.int32).ravel())
        ns = st_idx.size
        dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))  # noqa: E731
        vx = None
        vx_arr = None
        if vxc is not None:
            vx_arr = np.ascontiguousarray(np.asarray(vxc, dtype=np.float64).ravel())
            assert vx_arr.size == ns
            vx = dp(vx_arr)
        ne = 0
        en = None
        sig = None
        if energies is not None:
            en = np.ascontiguousarray(np.asarray(energies, dtype=np.float64).reshape(ns, -1))
            ne = en.shape[1]
            sig = np.empty((ns, ne, 2))
        res = (QpResult * ns)()
        o = QpOpts(int(n_lanczos), int(n_freq), float(omega0), float(eta), float(e_fermi), float(secant_tol),
                   int(secant_maxit), float(dE))
        st = QpStats()
        _check(self._lib.pdep_qp_energies(self._h, n, p, ns, st_idx.ctypes.data_as(C.POINTER(C.c_int)), vx,
                                          C.byref(o), res, ne, dp(en) if en is not None else None,
                                          dp(sig) if sig is not None else None, C.byref(st)),
               allow=(PDEP_ENOTCONV,) if allow_notconv else ())
        out = [r.as_dict() for r in res]
        sc = sig[..., 0] + 1j * sig[..., 1] if sig is not None else None
        return out, sc, st.as_dict()

    def eigs(self, n_pdep, seed=0, phi0=None, tol=1e-9, maxit=60, max_subspace=0, n_buffer=0,
             want_basis=False, allow_notconv=False, reducible=False, scr_tol=0.0, scr_maxit=0):
        """PDEP: (eps descending [n_pdep], basis [n_pdep, N_pw-1] or None, stats).  With
        reducible=True the Davidson iteration runs on chibar; eps is the same quantity."""
        eps = np.empty(n_pdep, dtype=np.float64)
        p0 = None
        keep = None
        if phi0 is not None:
            p0, keep = self._ptr(phi0, np.complex128, (n_pdep, self.n_pw - 1))
        basis = self._new(np.complex128, (n_pdep, self.n_pw - 1)) if want_basis else None
        bptr = None
        keep_b = None
        if basis is not None:
            bptr, keep_b = self._ptr(basis, np.complex128, (n_pdep, self.n_pw - 1), out=True)
        eo = EigOpts(float(tol), int(maxit), int(max_subspace), int(n_buffer), 1 if reducible else 0,
                     float(scr_tol), int(scr_maxit))
        st = EigStats()
        _check(self._lib.pdep_eigs(self._h, int(n_pdep), C.c_uint64(int(seed)), p0, C.byref(eo),
                                   eps.ctypes.data_as(C.POINTER(C.c_double)), bptr, C.byref(st)),
               allow=(PDEP_ENOTCONV,) if allow_notconv else ())
        if basis is not None and not self.device_ptrs:
            basis = keep_b
        return eps, basis, st.as_dict()

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _check(self._lib.pdep_destroy(self._h))
            self._h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Serving loop (pdep_server_*): jobs of (cell, V_loc, N_v, N_pdep, seed, options)
    admitted under an HBM budget and run concurrently on their own streams; resident
    systems serving chi0 requests in batches (pdep_server_add_system, pdep_submit_chi0)."""

    def __init__(self, max_running=4, hbm_budget=0, queue_capacity=0, fake=False, fake_ms_per_gb=100.0):
        self._lib = load()
        o = ServerOpts(int(max_running), int(hbm_budget), int(queue_capacity),
                       PDEP_SERVER_FAKE if fake else 0, float(fake_ms_per_gb))
        self._h = C.c_void_p()
        _check(self._lib.pdep_server_create(C.byref(o), C.byref(self._h)))
        self._keep = {}

    def submit(self, L, n, ecut, vloc, n_v, n_pdep, seed=0, precision=PDEP_MIXED_FP32, cg_tol=1e-8,
               eig_tol=1e-7, eig_maxit=60, n_buffer=0, max_subspace=0, **opt):
        o = Opts()
        self._lib.pdep_default_opts(C.byref(o))
        o.n_v = int(n_v)
        o.precision = int(precision)
        o.cg_tol = float(cg_tol)
        for k, v in opt.items():
            setattr(o, k, v)
        v = np.ascontiguousarray(np.asarray(vloc, dtype=np.float64).ravel())
        if v.size != int(np.prod([int(x) for x in n])):
            raise ValueError(f"vloc has {v.size} values for a {tuple(n)} grid")
        job = Job(Cell((C.c_double * 3)(*[float(x) for x in L]), (C.c_int * 3)(*[int(x) for x in n]), float(ecut)),
                  v.ctypes.data, o, int(n_pdep), C.c_uint64(int(seed)),
                  EigOpts(float(eig_tol), int(eig_maxit), int(max_subspace), int(n_buffer), 0, 0.0, 0))
        t = C.c_uint64()
        _check(self._lib.pdep_submit(self._h, C.byref(job), C.byref(t)))
        self._keep[t.value] = int(n_pdep)
        return t.value

    def poll(self, ticket):
        """(state, result dict or None, eps or None); never blocks."""
        st = C.c_int()
        res = JobResult()
        n = self._keep.get(ticket, 0)
        eps = np.empty(max(n, 1), dtype=np.float64)
        _check(self._lib.pdep_poll(self._h, C.c_uint64(ticket), C.byref(st), C.byref(res),
                                   eps.ctypes.data_as(C.POINTER(C.c_double)), n))
        if st.value == JOB_DONE:
            return st.value, res.as_dict(), eps[:n].copy()
        if st.value == JOB_FAILED:
            d = res.as_dict()
            d["error"] = self._lib.pdep_last_error().decode()
            return st.value, d, None
        return st.value, None, None

    def wait(self, ticket, timeout_ms=-1.0):
        st = C.c_int()
        _check(self._lib.pdep_server_wait(self._h, C.c_uint64(ticket), float(timeout_ms), C.byref(st)))
        return st.value

    def add_system(self, L, n, ecut, vloc, n_v, max_batch_pert=0, precision=PDEP_MIXED_FP32, cg_tol=1e-8, **opt):
        """Set up a resident system (pdep_server_add_system); returns its id."""
        o = Opts()
        self._lib.pdep_default_opts(C.byref(o))
        o.n_v = int(n_v)
        o.precision = int(precision)
        o.cg_tol = float(cg_tol)
        for k, v in opt.items():
            setattr(o, k, v)
        v = np.ascontiguousarray(np.asarray(vloc, dtype=np.float64).ravel())
        if v.size != int(np.prod([int(x) for x in n])):
            raise ValueError(f"vloc has {v.size} values for a {tuple(n)} grid")
        cell = Cell((C.c_double * 3)(*[float(x) for x in L]), (C.c_int * 3)(*[int(x) for x in n]), float(ecut))
        sid = C.c_uint64()
        _check(self._lib.pdep_server_add_system(self._h, C.byref(cell), v.ctypes.data, C.byref(o),
                                                int(max_batch_pert), C.byref(sid)))
        return sid.value

    def remove_system(self, system_id):
        _check(self._lib.pdep_server_remove_system(self._h, C.c_uint64(system_id)))

    def system_info(self, system_id):
        """Sizes and ground-state figures of a resident system (pdep_server_system_info)."""
        i = Info()
        _check(self._lib.pdep_server_system_info(self._h, C.c_uint64(system_id), C.byref(i)))
        return {k: getattr(i, k) for k, _ in Info._fields_}

    def submit_chi0(self, system_id, phi):
        """Queue chi0bar applied to phi [n_pert, N_pw - 1] (complex) on a resident system."""
        a = np.ascontiguousarray(np.asarray(phi, dtype=np.complex128))
        npw = self.system_info(system_id)["n_pw"]
        if a.ndim != 2 or a.shape[1] != npw - 1:
            raise ValueError(f"phi must be [n_pert, {npw - 1}], got {a.shape}")
        t = C.c_uint64()
        _check(self._lib.pdep_submit_chi0(self._h, C.c_uint64(system_id), int(a.shape[0]), a.ctypes.data, C.byref(t)))
        self._keep[t.value] = (int(a.shape[0]), int(a.shape[1]))
        return t.value

    def submit_eigs(self, system_id, n_pdep, seed=0, eig_tol=1e-7, eig_maxit=60, n_buffer=0, max_subspace=0):
        """Queue a PDEP Davidson on a resident system (reuses its orbitals)."""
        eo = EigOpts(float(eig_tol), int(eig_maxit), int(max_subspace), int(n_buffer), 0, 0.0, 0)
        t = C.c_uint64()
        _check(self._lib.pdep_submit_eigs(self._h, C.c_uint64(system_id), int(n_pdep), C.c_uint64(int(seed)),
                                          C.byref(eo), C.byref(t)))
        self._keep[t.value] = int(n_pdep)
        return t.value

    def poll_eigs(self, ticket):
        """(state, result dict or None, eps or None) of a request of submit_eigs."""
        st = C.c_int()
        res = JobResult()
        n = self._keep.get(ticket, 0)
        eps = np.empty(max(n, 1), dtype=np.float64)
        _check(self._lib.pdep_poll_eigs(self._h, C.c_uint64(ticket), C.byref(st), C.byref(res),
                                        eps.ctypes.data_as(C.POINTER(C.c_double)), n))
        if st.value == JOB_DONE:
            return st.value, res.as_dict(), eps[:n].copy()
        if st.value == JOB_FAILED:
            d = res.as_dict()
            d["error"] = self._lib.pdep_last_error().decode()
            return st.value, d, None
        return st.value, None, None

    def poll_chi0(self, ticket):
        """(state, result dict or None, out [n_pert, N_pw - 1] or None); never blocks."""
        st = C.c_int()
        res = Chi0Result()
        kept = self._keep.get(ticket)
        n, w = kept if isinstance(kept, tuple) else (0, 1)   # not a chi0 request: the library says so
        out = np.empty((max(n, 1), w), dtype=np.complex128)
        _check(self._lib.pdep_poll_chi0(self._h, C.c_uint64(ticket), C.byref(st), C.byref(res),
                                        out.ctypes.data if n > 0 else None, n))
        if st.value == JOB_DONE:
            return st.value, res.as_dict(), out
        if st.value == JOB_FAILED:
            d = res.as_dict()
            d["error"] = self._lib.pdep_last_error().decode()
            return st.value, d, None
        return st.value, None, None

    def stats(self):
        s = ServerStats()
        _check(self._lib.pdep_server_stats_get(self._h, C.byref(s)))
        return s.as_dict()

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.pdep_server_destroy(self._h)
            self._h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
