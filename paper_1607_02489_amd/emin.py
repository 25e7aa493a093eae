"""ctypes binding of libemin.so (the HIP C ABI in include/emin.h).

Argument marshalling only: every step of the setup runs in the library's
kernels.  PyTorch provides device memory (tensors) and the stream.  There is
no CPU fallback: without the built library or a GPU, loading fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libemin.so")

EMIN_PREC_F64, EMIN_PREC_MIXED = 0, 1
(EMIN_FLAG_ENERGY, EMIN_FLAG_VALIDATE, EMIN_FLAG_AUTOTUNE, EMIN_FLAG_PATTERN_VALUES,
 EMIN_FLAG_ENERGY_ATA, EMIN_FLAG_STAGED_PRODUCT, EMIN_FLAG_GMRES,
 EMIN_FLAG_PETROV_GALERKIN) = 1, 2, 4, 8, 16, 32, 64, 128
MAX_ITERS = 32
(VIEW_PV, VIEW_PP, VIEW_AC, VIEW_BC, VIEW_MV, VIEW_MP, VIEW_S, VIEW_ORDER, VIEW_CP, VIEW_CBAR,
 VIEW_CV, VIEW_XVC, VIEW_P2VC, VIEW_KEEPV, VIEW_KEEPP, VIEW_DIR) = range(16)
STATUS = ["OK", "ERR_ARG", "ERR_SHAPE", "ERR_PATTERN", "ERR_VALUE", "ERR_INFEASIBLE",
          "ERR_BREAKDOWN", "ERR_BUDGET", "ERR_DEVICE", "ERR_OOM", "ERR_CAPACITY", "ERR_COLOCATE",
          "ERR_CANCELLED"]
SYMBOLS = ["emin_pattern", "emin_pattern_alloc", "emin_pattern_info", "emin_pattern_view", "emin_setup", "emin_rap",
           "emin_sync_report", "emin_memcpy_d2h", "emin_pattern_destroy", "emin_status_string",
           "emin_version", "emin_last_error", "emin_fp_probe", "emin_release_cached", "emin_profile_enable", "emin_profile_collect",
           "emin_hierarchy_build", "emin_hierarchy_resetup", "emin_hierarchy_info",
           "emin_hierarchy_level", "emin_hierarchy_device_bytes", "emin_hierarchy_destroy",
           "emin_hierarchy_build_batch", "emin_batch_create", "emin_batch_run",
           "emin_batch_destroy", "emin_server_create", "emin_server_submit", "emin_server_poll",
           "emin_server_wait", "emin_server_cancel", "emin_server_release", "emin_server_stats", "emin_server_destroy",
           "emin_pattern_with_cpoints", "emin_setup_with_pattern", "emin_profile_launches",
           "emin_setup_pg", "emin_rap_pg", "emin_galerkin", "emin_matrix_view",
           "emin_matrix_destroy", "emin_infsup", "emin_solver_create", "emin_solver_info",
           "emin_solver_bs_step", "emin_solver_vcycle", "emin_solver_gmres", "emin_solver_destroy"]
PROF_KINDS = ["spmm", "update", "spgemm", "alg3", "alg4", "vpattern", "r6", "r7"]
EMIN_PROF_ONLY = 1 << 30


class EminError(RuntimeError):
    def __init__(self, status, where=""):
        name = STATUS[status] if 0 <= status < len(STATUS) else str(status)
        detail = ""
        try:
            detail = lib().emin_last_error().decode(errors="replace")
        except Exception:
            pass
        super().__init__(f"{where}: {name}" + (f" ({detail})" if detail else ""))
        self.status = status


class c_csr(C.Structure):
    _fields_ = [("nrows", C.c_int64), ("ncols", C.c_int64), ("nnz", C.c_int64),
                ("rowptr", C.c_void_p), ("col", C.c_void_p), ("val", C.c_void_p)]


class c_system(C.Structure):
    _fields_ = [("dim", C.c_int32), ("Ahat", c_csr), ("Bdiv", c_csr), ("xv", C.c_void_p),
                ("p2v", C.c_void_p), ("Wv", C.c_void_p), ("Wp", C.c_void_p), ("Gt", C.c_void_p)]


class c_params(C.Structure):
    _fields_ = [("tau1_v", C.c_double), ("tau1_p", C.c_double), ("tau2_sq", C.c_double),
                ("iters", C.c_int32), ("precision", C.c_int32), ("flags", C.c_uint32)]


class c_sizes(C.Structure):
    _fields_ = [(k, C.c_int64) for k in
                ["n_v", "n_p", "n_vc", "n_pc", "n_cp_alg3", "n_cp_extra", "n_mid", "n_cv_extra",
                 "nnz_Pv", "nnz_Pp", "nnz_Mv", "nnz_Mp", "nnz_Ac", "nnz_Bc", "device_bytes",
                 "sched_v", "sched_p"]]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class c_report(C.Structure):
    _fields_ = [("status", C.c_int32), ("its_v", C.c_int32), ("its_p", C.c_int32),
                ("reserved", C.c_int32),
                ("energy_v", C.c_double * (MAX_ITERS + 1)), ("energy_p", C.c_double * (MAX_ITERS + 1)),
                ("rho_v", C.c_double * (MAX_ITERS + 1)), ("rho_p", C.c_double * (MAX_ITERS + 1)),
                ("gamma_v", C.c_double * MAX_ITERS), ("gamma_p", C.c_double * MAX_ITERS),
                ("its_r", C.c_int32), ("reserved2", C.c_int32),
                ("energy_r", C.c_double * (MAX_ITERS + 1)), ("rho_r", C.c_double * (MAX_ITERS + 1)),
                ("gamma_r", C.c_double * MAX_ITERS)]


class c_kstat(C.Structure):
    _fields_ = [("launches", C.c_int64), ("total_ms", C.c_double), ("bytes", C.c_double),
                ("flops", C.c_double)]


class c_klaunch(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("ms", C.c_double),
                ("bytes", C.c_double), ("flops", C.c_double)]


class c_view(C.Structure):
    _fields_ = [("n", C.c_int64), ("ncols", C.c_int64), ("nnz", C.c_int64),
                ("rowptr", C.c_void_p), ("col", C.c_void_p), ("val", C.c_void_p),
                ("data", C.c_void_p)]


_lib = None


def lib():
    """Load libemin.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError(f"{LIBPATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIBPATH)
        P = C.POINTER
        L.emin_pattern.argtypes = [P(c_system), P(c_params), C.c_void_p, P(C.c_void_p)]
        L.emin_pattern_with_cpoints.argtypes = [P(c_system), P(c_params), C.c_void_p, C.c_int64,
                                                C.c_void_p, P(C.c_void_p)]
        L.emin_pattern_alloc.argtypes = [P(c_system), P(c_params), P(c_allocator), C.c_void_p,
                                         P(C.c_void_p)]
        L.emin_setup_with_pattern.argtypes = [P(c_csr), C.c_void_p, C.c_void_p, C.c_int64,
                                              C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                              C.c_int32, C.c_int32, C.c_uint32, C.c_void_p,
                                              C.c_void_p, C.c_void_p]
        L.emin_setup_with_pattern_noalloc.argtypes = L.emin_setup_with_pattern.argtypes
        L.emin_pattern_info.argtypes = [C.c_void_p, P(c_sizes)]
        L.emin_pattern_view.argtypes = [C.c_void_p, C.c_int32, P(c_view)]
        L.emin_setup.argtypes = [C.c_void_p, P(c_system), P(c_params), C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_void_p]
        L.emin_rap.argtypes = [C.c_void_p, P(c_system), C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_int32, C.c_void_p]
        L.emin_setup_pg.argtypes = [C.c_void_p, P(c_system), P(c_params), C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_void_p]
        L.emin_rap_pg.argtypes = [C.c_void_p, P(c_system), C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.emin_sync_report.argtypes = [C.c_void_p, C.c_void_p, P(c_report)]
        L.emin_memcpy_d2h.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
        L.emin_pattern_destroy.argtypes = [C.c_void_p]
        L.emin_pattern_destroy.restype = None
        L.emin_status_string.argtypes = [C.c_int]
        L.emin_status_string.restype = C.c_char_p
        L.emin_version.restype = C.c_char_p
        L.emin_last_error.restype = C.c_char_p
        L.emin_release_cached.restype = C.c_int64
        L.emin_fp_probe.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
        L.emin_hierarchy_build.argtypes = [P(c_system), P(c_params), C.c_int32, C.c_int64,
                                           C.c_void_p, P(C.c_void_p)]
        L.emin_hierarchy_resetup.argtypes = [C.c_void_p, P(c_system), C.c_void_p]
        L.emin_hierarchy_info.argtypes = [C.c_void_p, P(C.c_int32), P(c_sizes), C.c_int32]
        L.emin_hierarchy_level.argtypes = [C.c_void_p, C.c_int32, P(C.c_void_p), P(C.c_void_p),
                                           P(C.c_void_p), P(C.c_void_p), P(C.c_void_p),
                                           P(C.c_void_p)]
        L.emin_hierarchy_device_bytes.argtypes = [C.c_void_p]
        L.emin_hierarchy_device_bytes.restype = C.c_int64
        L.emin_hierarchy_destroy.argtypes = [C.c_void_p]
        L.emin_hierarchy_destroy.restype = None
        L.emin_hierarchy_build_batch.argtypes = [P(P(c_system)), C.c_int32, P(c_params), C.c_int32,
                                                 C.c_int64, C.c_int32, P(C.c_void_p)]
        L.emin_batch_create.argtypes = [P(C.c_void_p), P(P(c_system)), C.c_int32, C.c_void_p,
                                        P(C.c_void_p)]
        L.emin_batch_run.argtypes = [C.c_void_p, C.c_void_p]
        L.emin_batch_destroy.argtypes = [C.c_void_p]
        L.emin_batch_destroy.restype = None
        L.emin_server_create.argtypes = [C.c_int64, C.c_int32, P(C.c_void_p)]
        L.emin_server_submit.argtypes = [C.c_void_p, P(c_system), P(c_params), C.c_int32,
                                         C.c_int64, P(C.c_int64)]
        L.emin_server_poll.argtypes = [C.c_void_p, C.c_int64, P(C.c_int32)]
        L.emin_server_wait.argtypes = [C.c_void_p, C.c_int64, P(C.c_void_p), P(C.c_double),
                                       P(C.c_double)]
        L.emin_server_release.argtypes = [C.c_void_p, C.c_int64]
        L.emin_server_cancel.argtypes = [C.c_void_p, C.c_int64, P(C.c_int32)]
        L.emin_server_stats.argtypes = [C.c_void_p, P(C.c_int64), P(C.c_int32), P(C.c_int32)]
        L.emin_server_destroy.argtypes = [C.c_void_p]
        L.emin_server_destroy.restype = None
        L.emin_galerkin.argtypes = [P(c_csr), P(c_csr), C.c_void_p, P(C.c_void_p)]
        L.emin_matrix_view.argtypes = [C.c_void_p, P(c_csr)]
        L.emin_matrix_destroy.argtypes = [C.c_void_p]
        L.emin_matrix_destroy.restype = None
        L.emin_infsup.argtypes = [P(c_csr), P(c_csr), P(c_csr), C.c_int32, C.c_int32, C.c_double,
                                  P(C.c_double), P(C.c_double), P(C.c_int32), P(C.c_int32),
                                  C.c_void_p]
        L.emin_solver_create.argtypes = [P(c_system), C.c_void_p, C.c_int32, C.c_double,
                                         C.c_int32, C.c_int32, C.c_void_p, P(C.c_void_p)]
        L.emin_solver_info.argtypes = [C.c_void_p, C.c_int32, P(C.c_int64), P(C.c_int32)]
        L.emin_solver_bs_step.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                          C.c_void_p]
        L.emin_solver_vcycle.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.emin_solver_gmres.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                        C.c_int32, P(C.c_int32), P(C.c_double), C.c_void_p]
        L.emin_solver_destroy.argtypes = [C.c_void_p]
        L.emin_solver_destroy.restype = None
        L.emin_profile_enable.argtypes = [C.c_int]
        L.emin_autotune_stats.argtypes = [P(C.c_int64)]
        L.emin_profile_collect.argtypes = [P(c_kstat), C.c_int32]
        L.emin_profile_launches.argtypes = [P(c_klaunch), C.c_int32, P(C.c_int32)]
        _lib = L
    return _lib


def _check(st, where):
    if st != 0:
        raise EminError(st, where)


def params(tau1_v=0.06, tau1_p=0.06, tau2_sq=1.5e-3, iters=5, mixed=False, energy=False,
           validate=False, autotune=False, energy_ata=False, staged=False,
           gmres=False, pg=False) -> c_params:
    """energy_ata: the velocity block's EMIN energy is the A^T A-norm of the
    filtered operator (sec. 4.3, eq. (min_problem), non-symmetric operators).
    staged: the masked product runs on coordinate tiles whose Z rows are
    staged in LDS (instead of gathering them row by row from device memory)."""
    flags = ((EMIN_FLAG_ENERGY if energy else 0) | (EMIN_FLAG_VALIDATE if validate else 0) |
             (EMIN_FLAG_AUTOTUNE if autotune else 0) | (EMIN_FLAG_ENERGY_ATA if energy_ata else 0) |
             (EMIN_FLAG_STAGED_PRODUCT if staged else 0) | (EMIN_FLAG_GMRES if gmres else 0) |
             (EMIN_FLAG_PETROV_GALERKIN if pg else 0))
    return c_params(tau1_v, tau1_p, tau2_sq, iters, EMIN_PREC_MIXED if mixed else EMIN_PREC_F64,
                    flags)


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _sync():
    """Waits for all queued device work (before a handle's memory is reused)."""
    import torch
    if torch.cuda.is_available():
        torch.cuda.synchronize()


def d2h(ptr, n, dtype, stream=None) -> np.ndarray:
    out = np.empty(int(n), dtype=dtype)
    if n:
        _check(lib().emin_memcpy_d2h(out.ctypes.data, C.c_void_p(ptr), out.nbytes,
                                     _stream(stream)), "memcpy")
    return out


# ----------------------------------------------------------------------------
@dataclass
class DeviceSystem:
    """A level's system in device memory (torch tensors or handle-owned views)."""
    dim: int
    n_v: int
    n_p: int
    A: tuple            # (nnz, rowptr_ptr, col_ptr, val_ptr)
    B: tuple
    xv: int
    p2v: int
    keep: list = field(default_factory=list)   # keeps tensors / handles alive
    Gt: int = 0         # gradient block's transpose on B's pattern (0: B itself)

    @staticmethod
    def upload(sys, device="cuda") -> "DeviceSystem":
        import torch
        t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dt)
        Ar, Ac, Av = (t(sys.Ahat.rowptr, torch.int64), t(sys.Ahat.col, torch.int32),
                      t(sys.Ahat.val, torch.float64))
        Br, Bc, Bv = (t(sys.Bdiv.rowptr, torch.int64), t(sys.Bdiv.col, torch.int32),
                      t(sys.Bdiv.val, torch.float64))
        xv = t(sys.xv.reshape(-1), torch.float64)
        p2v = t(sys.p2v, torch.int32)
        gt = (sys.meta or {}).get("Gt") if hasattr(sys, "meta") else None
        Gt = t(gt, torch.float64) if gt is not None else None
        return DeviceSystem(sys.dim, sys.n_v, sys.n_p,
                            (sys.Ahat.nnz, Ar.data_ptr(), Ac.data_ptr(), Av.data_ptr()),
                            (sys.Bdiv.nnz, Br.data_ptr(), Bc.data_ptr(), Bv.data_ptr()),
                            xv.data_ptr(), p2v.data_ptr(), [Ar, Ac, Av, Br, Bc, Bv, xv, p2v, Gt],
                            Gt.data_ptr() if Gt is not None else 0)

    def c(self) -> c_system:
        A = c_csr(self.n_v, self.n_v, self.A[0], self.A[1], self.A[2], self.A[3])
        B = c_csr(self.n_p, self.dim * self.n_v, self.B[0], self.B[1], self.B[2], self.B[3])
        return c_system(self.dim, A, B, self.xv, self.p2v, None, None, self.Gt or None)


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class c_allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


class Allocator:
    """An emin_allocator_t over Python callables alloc(nbytes) -> int device
    pointer (0 on failure) and free(ptr).  Keep it alive while any handle
    built with it exists."""

    def __init__(self, alloc, free):
        def _a(n, _ctx):
            try:
                return int(alloc(int(n))) or None
            except Exception:
                return None

        def _f(p, _ctx):
            free(int(p))
        self._a, self._f = ALLOC_FN(_a), FREE_FN(_f)
        self.c = c_allocator(self._a, self._f, None)


def torch_allocator(stream=None) -> Allocator:
    """Device memory from torch's caching allocator (on the current device and
    the given stream, default the current one)."""
    import torch
    dev = torch.cuda.current_device()
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    return Allocator(lambda n: torch.cuda.caching_allocator_alloc(n, dev, st),
                     torch.cuda.caching_allocator_delete)


class Pattern:
    """emin_pattern handle of one level (emin_pattern_with_cpoints when
    cpoints, a device int32 tensor of ascending coarse pressures, is given;
    emin_pattern_alloc when allocator, an Allocator, is given)."""

    def __init__(self, dsys: DeviceSystem, prm: c_params, stream=None, cpoints=None,
                 allocator=None):
        self.dsys = dsys
        self._c = dsys.c()
        self.allocator = allocator
        h = C.c_void_p()
        if allocator is not None:
            _check(lib().emin_pattern_alloc(C.byref(self._c), C.byref(prm),
                                            C.byref(allocator.c), _stream(stream), C.byref(h)),
                   "emin_pattern_alloc")
        elif cpoints is None:
            _check(lib().emin_pattern(C.byref(self._c), C.byref(prm), _stream(stream),
                                      C.byref(h)), "emin_pattern")
        else:
            _check(lib().emin_pattern_with_cpoints(C.byref(self._c), C.byref(prm),
                                                   C.c_void_p(cpoints.data_ptr()),
                                                   int(cpoints.numel()), _stream(stream),
                                                   C.byref(h)), "emin_pattern_with_cpoints")
        self.h = h
        s = c_sizes()
        _check(lib().emin_pattern_info(h, C.byref(s)), "emin_pattern_info")
        self.sizes = s.as_dict()

    def view(self, what) -> c_view:
        v = c_view()
        _check(lib().emin_pattern_view(self.h, what, C.byref(v)), "emin_pattern_view")
        return v

    def csr_host(self, what, vals=None):
        """(rowptr, col, val) host copies of a CSR view; vals = device ptr."""
        v = self.view(what)
        rp = d2h(v.rowptr, v.n + 1, np.int64)
        col = d2h(v.col, v.nnz, np.int32)
        vp = vals if vals is not None else v.val
        val = d2h(vp, v.nnz, np.float64) if vp else None
        return v.n, v.ncols, rp, col, val

    def array_host(self, what, dtype):
        v = self.view(what)
        return d2h(v.data, v.n, dtype)

    def setup(self, prm: c_params, Pv, Pp, report=None, stream=None):
        _check(lib().emin_setup(self.h, C.byref(self._c), C.byref(prm), C.c_void_p(Pv),
                                C.c_void_p(Pp), _stream(stream),
                                C.c_void_p(report) if report else None), "emin_setup")

    def rap(self, Pv, Pp, Ac, Bc, stream=None, mixed=False):
        _check(lib().emin_rap(self.h, C.byref(self._c), C.c_void_p(Pv), C.c_void_p(Pp),
                              C.c_void_p(Ac), C.c_void_p(Bc),
                              EMIN_PREC_MIXED if mixed else EMIN_PREC_F64, _stream(stream)),
               "emin_rap")

    def setup_pg(self, prm: c_params, Pv, Pp, Rvt, report=None, stream=None):
        """emin_setup_pg: P and the Petrov-Galerkin restriction's R_v^T."""
        _check(lib().emin_setup_pg(self.h, C.byref(self._c), C.byref(prm), C.c_void_p(Pv),
                                   C.c_void_p(Pp), C.c_void_p(Rvt), _stream(stream),
                                   C.c_void_p(report) if report else None), "emin_setup_pg")

    def rap_pg(self, Pv, Pp, Rvt, Ac, Bc, Gct, stream=None):
        _check(lib().emin_rap_pg(self.h, C.byref(self._c), C.c_void_p(Pv), C.c_void_p(Pp),
                                 C.c_void_p(Rvt), C.c_void_p(Ac), C.c_void_p(Bc), C.c_void_p(Gct),
                                 _stream(stream)), "emin_rap_pg")

    def coarse_system(self, Ac, Bc, Gct=None) -> DeviceSystem:
        a, b = self.view(VIEW_AC), self.view(VIEW_BC)
        x, p = self.view(VIEW_XVC), self.view(VIEW_P2VC)
        s = self.sizes
        return DeviceSystem(self.dsys.dim, s["n_vc"], s["n_pc"],
                            (a.nnz, a.rowptr, a.col, Ac.data_ptr()),
                            (b.nnz, b.rowptr, b.col, Bc.data_ptr()),
                            x.data, p.data, [self, Ac, Bc, Gct],
                            Gct.data_ptr() if Gct is not None else 0)

    def close(self):
        if self.h:
            _sync()
            lib().emin_pattern_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def setup_with_pattern(M_dev, N_dev, ncoarse, cid, W, Wc, iters, P, mixed=False, energy=False,
                       validate=False, report=None, stream=None, noalloc=False):
    """emin_setup_with_pattern (emin_setup_with_pattern_noalloc with
    noalloc).  M_dev = (n, nnz, rowptr, col, val) and N_dev = (nnz, rowptr,
    col) device tensors; cid, W, Wc, P device tensors."""
    n, mnnz, mrp, mcol, mval = M_dev
    nnnz, nrp, ncol = N_dev
    Mc = c_csr(n, n, mnnz, mrp.data_ptr(), mcol.data_ptr(), mval.data_ptr())
    flags = (EMIN_FLAG_ENERGY if energy else 0) | (EMIN_FLAG_VALIDATE if validate else 0)
    fn = lib().emin_setup_with_pattern_noalloc if noalloc else lib().emin_setup_with_pattern
    _check(fn(C.byref(Mc), C.c_void_p(nrp.data_ptr()),
                                         C.c_void_p(ncol.data_ptr()), int(ncoarse), int(nnnz),
                                         C.c_void_p(cid.data_ptr()), C.c_void_p(W.data_ptr()),
                                         C.c_void_p(Wc.data_ptr()), iters,
                                         EMIN_PREC_MIXED if mixed else EMIN_PREC_F64, flags,
                                         C.c_void_p(P.data_ptr()), _stream(stream),
                                         C.c_void_p(report.data_ptr()) if report is not None
                                         else None),
           "emin_setup_with_pattern_noalloc" if noalloc else "emin_setup_with_pattern")


def release_cached() -> int:
    """emin_release_cached: frees the library's cached device chunks (bytes)."""
    return int(lib().emin_release_cached())


def autotune_stats() -> dict:
    """Process-wide autotuner counters of the masked-product schedule."""
    out = (C.c_int64 * 4)()
    _check(lib().emin_autotune_stats(out), "emin_autotune_stats")
    return dict(tuned=int(out[0]), reused=int(out[1]), candidates_timed=int(out[2]),
                table=int(out[3]))


def autotune_reset():
    _check(lib().emin_autotune_reset(), "emin_autotune_reset")


def sched_name(code: int) -> str:
    """Readable form of a schedule code from the level sizes."""
    parts = (["staged"] if code & 64 else []) + (["batch16"] if code & 128 else []) + [
        "maps" if code & 1 else "search-only", "2x-lanes" if code & 2 else "tight-lanes",
        "xcd-by-class" if code & 4 else ("xcd-merged" if code & 8 else "xcd-contiguous")]
    return "+".join(parts) + ["", " (tuned)", " (reused)", ""][(code >> 4) & 3]


def profile_enable(on=True, kinds=None):
    """Time kernel classes with HIP events: all of them, or only `kinds`
    (names of profile_collect's keys)."""
    if not on:
        v = 0
    elif kinds is None:
        v = 1
    else:
        v = EMIN_PROF_ONLY
        for k in kinds:
            v |= 1 << PROF_KINDS.index(k)
    _check(lib().emin_profile_enable(v), "emin_profile_enable")


def profile_collect() -> dict:
    arr = (c_kstat * len(PROF_KINDS))()
    _check(lib().emin_profile_collect(arr, len(PROF_KINDS)), "emin_profile_collect")
    return {k: dict(launches=int(a.launches), ms=float(a.total_ms), bytes=float(a.bytes),
                    flops=float(a.flops)) for k, a in zip(PROF_KINDS, arr) if a.launches}


def profile_launches(cap=1 << 16) -> list:
    """Per-launch records (kind name, ms, algorithmic bytes), in launch order;
    clears the records as profile_collect does."""
    arr = (c_klaunch * cap)()
    n = C.c_int32()
    _check(lib().emin_profile_launches(arr, cap, C.byref(n)), "emin_profile_launches")
    return [dict(kind=PROF_KINDS[arr[i].kind] if 0 <= arr[i].kind < len(PROF_KINDS) else
                 str(arr[i].kind), ms=float(arr[i].ms), bytes=float(arr[i].bytes),
                 flops=float(arr[i].flops)) for i in range(min(n.value, cap))]


def sync_report(rep_tensor, stream=None, raise_on_error=True) -> c_report:
    r = c_report()
    st = lib().emin_sync_report(C.c_void_p(rep_tensor.data_ptr()), _stream(stream), C.byref(r))
    if st != 0 and raise_on_error:
        raise EminError(st, "emin_sync_report")
    return r


def new_report(device="cuda"):
    import torch
    return torch.zeros(C.sizeof(c_report), dtype=torch.uint8, device=device)


@dataclass
class Level:
    pattern: Pattern
    Pv: object          # torch float64 tensors
    Pp: object
    Ac: object
    Bc: object
    report: object


class Hierarchy:
    """Alg. 1 without relaxation: nlevels levels (nlevels-1 transfers).

    build() runs emin_pattern + emin_setup + emin_rap level by level;
    resetup() reruns only the numeric phases (emin_setup + emin_rap) on the
    stored patterns, as for a new Picard linearisation with the same structure.
    """

    def __init__(self, sys, nlevels, prm: c_params, min_dofs=0, device="cuda"):
        self.fine = DeviceSystem.upload(sys, device)
        self.nlevels = nlevels
        self.prm = c_params.from_buffer_copy(prm)
        self.prm.flags &= ~EMIN_FLAG_PATTERN_VALUES   # re-setups take new values
        self.min_dofs = min_dofs
        self.device = device
        self.levels: list[Level] = []

    def build(self, stream=None):
        import torch
        self.levels = []
        # each level's setup follows its pattern on the same values
        first = c_params.from_buffer_copy(self.prm)
        first.flags |= EMIN_FLAG_PATTERN_VALUES
        cur = self.fine
        for _ in range(self.nlevels - 1):
            if cur.dim * cur.n_v + cur.n_p <= self.min_dofs:
                break
            pat = Pattern(cur, self.prm, stream)
            s = pat.sizes
            f64 = dict(dtype=torch.float64, device=self.device)
            L = Level(pat, torch.empty(max(s["nnz_Pv"], 1), **f64),
                      torch.empty(max(s["nnz_Pp"], 1), **f64),
                      torch.empty(max(s["nnz_Ac"], 1), **f64),
                      torch.empty(max(s["nnz_Bc"], 1), **f64), new_report(self.device))
            pat.setup(first, L.Pv.data_ptr(), L.Pp.data_ptr(), L.report.data_ptr(), stream)
            pat.rap(L.Pv.data_ptr(), L.Pp.data_ptr(), L.Ac.data_ptr(), L.Bc.data_ptr(), stream,
                    mixed=self.prm.precision == EMIN_PREC_MIXED)
            self.levels.append(L)
            cur = pat.coarse_system(L.Ac, L.Bc)
        self.coarsest = cur
        return self

    def resetup(self, stream=None, prm: c_params = None):
        """Numeric phases of every level on the stored patterns and drop masks.
        prm (default: the hierarchy's) may change the precision: a hierarchy
        built in FP64 and re-set up in mixed precision runs the FP32 products
        on the patterns of the FP64 pass."""
        p = self.prm if prm is None else c_params.from_buffer_copy(prm)
        p.flags &= ~EMIN_FLAG_PATTERN_VALUES
        for L in self.levels:
            L.pattern.setup(p, L.Pv.data_ptr(), L.Pp.data_ptr(), L.report.data_ptr(), stream)
            L.pattern.rap(L.Pv.data_ptr(), L.Pp.data_ptr(), L.Ac.data_ptr(), L.Bc.data_ptr(),
                          stream, mixed=p.precision == EMIN_PREC_MIXED)

    def p_nnz(self):
        return sum(L.pattern.sizes["nnz_Pv"] + L.pattern.sizes["nnz_Pp"] for L in self.levels)

    def close(self):
        for L in reversed(self.levels):
            L.pattern.close()
        self.levels = []


# ----------------------------------------------------------------------------
# native hierarchies, batches and the serving loop
# ----------------------------------------------------------------------------
class HierarchyView:
    """Read access to a native hierarchy's levels (borrowed device pointers)."""

    def __init__(self, h):
        self.h = h

    def ntransfers(self) -> int:
        n = C.c_int32()
        _check(lib().emin_hierarchy_info(self.h, C.byref(n), None, 0), "emin_hierarchy_info")
        return n.value

    def sizes(self):
        n = self.ntransfers()
        arr = (c_sizes * max(n, 1))()
        k = C.c_int32()
        _check(lib().emin_hierarchy_info(self.h, C.byref(k), arr, n), "emin_hierarchy_info")
        return [arr[i].as_dict() for i in range(n)]

    def level_host(self, level):
        """Host copies (Pv, Pp, Ac, Bc values) of one transfer level."""
        p, pv, pp, ac, bc, rep = (C.c_void_p() for _ in range(6))
        _check(lib().emin_hierarchy_level(self.h, level, C.byref(p), C.byref(pv), C.byref(pp),
                                          C.byref(ac), C.byref(bc), C.byref(rep)),
               "emin_hierarchy_level")
        z = self.sizes()[level]
        return dict(Pv=d2h(pv.value, z["nnz_Pv"], np.float64),
                    Pp=d2h(pp.value, z["nnz_Pp"], np.float64),
                    Ac=d2h(ac.value, z["nnz_Ac"], np.float64),
                    Bc=d2h(bc.value, z["nnz_Bc"], np.float64), pattern=p.value,
                    report=rep.value)

    def level_csr(self, level):
        """Host CSR tuples (nrows, ncols, rowptr, col, val) of one transfer
        level's Pv, Pp (transfers) and Ac, Bc (the next level's operators)."""
        d = self.level_host(level)
        p = C.c_void_p(d["pattern"])
        out = {}
        for key, what in (("Pv", VIEW_PV), ("Pp", VIEW_PP), ("Ac", VIEW_AC), ("Bc", VIEW_BC)):
            v = c_view()
            _check(lib().emin_pattern_view(p, what, C.byref(v)), "emin_pattern_view")
            out[key] = (int(v.n), int(v.ncols), d2h(v.rowptr, v.n + 1, np.int64),
                        d2h(v.col, v.nnz, np.int32), d[key])
        return out

    def device_bytes(self) -> int:
        return int(lib().emin_hierarchy_device_bytes(self.h))


class NativeHierarchy(HierarchyView):
    """emin_hierarchy_build: every level built by the library's C++ driver."""

    def __init__(self, dsys: DeviceSystem, prm: c_params, nlevels: int, min_dofs: int = 0,
                 stream=None, handle=None):
        self.dsys = dsys
        self._c = dsys.c()
        if handle is None:
            h = C.c_void_p()
            _check(lib().emin_hierarchy_build(C.byref(self._c), C.byref(prm), nlevels, min_dofs,
                                              _stream(stream), C.byref(h)),
                   "emin_hierarchy_build")
            handle = h
        super().__init__(handle)

    def resetup(self, stream=None, dsys: DeviceSystem = None):
        if dsys is not None:
            self.dsys, self._c = dsys, dsys.c()
        _check(lib().emin_hierarchy_resetup(self.h, C.byref(self._c), _stream(stream)),
               "emin_hierarchy_resetup")

    def close(self):
        if self.h:
            _sync()
            lib().emin_hierarchy_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_batch(dsystems, prm: c_params, nlevels: int, min_dofs: int = 0, max_parallel: int = 16):
    n = len(dsystems)
    cs = [d.c() for d in dsystems]
    ptrs = (C.POINTER(c_system) * n)(*[C.pointer(c) for c in cs])
    out = (C.c_void_p * n)()
    _check(lib().emin_hierarchy_build_batch(ptrs, n, C.byref(prm), nlevels, min_dofs,
                                            max_parallel, out), "emin_hierarchy_build_batch")
    return [NativeHierarchy(d, prm, nlevels, min_dofs, handle=C.c_void_p(out[i]))
            for i, d in enumerate(dsystems)]


class Batch:
    """All numeric phases of several hierarchies captured as one hipGraph."""

    def __init__(self, hierarchies, stream=None):
        self.hs = hierarchies
        n = len(hierarchies)
        self._cs = [h._c for h in hierarchies]
        hp = (C.c_void_p * n)(*[h.h for h in hierarchies])
        sp = (C.POINTER(c_system) * n)(*[C.pointer(c) for c in self._cs])
        b = C.c_void_p()
        _check(lib().emin_batch_create(hp, sp, n, _stream(stream), C.byref(b)), "emin_batch_create")
        self.b = b

    def run(self, stream=None):
        _check(lib().emin_batch_run(self.b, _stream(stream)), "emin_batch_run")

    def close(self):
        if self.b:
            lib().emin_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """The serving loop: admission by device-memory budget, worker streams."""

    def __init__(self, budget_bytes: int, slots: int):
        s = C.c_void_p()
        _check(lib().emin_server_create(int(budget_bytes), slots, C.byref(s)), "emin_server_create")
        self.s = s
        self._borrowed = {}

    def submit(self, dsys: DeviceSystem, prm: c_params, nlevels: int, min_dofs: int = 0) -> int:
        c = dsys.c()
        t = C.c_int64()
        _check(lib().emin_server_submit(self.s, C.byref(c), C.byref(prm), nlevels, min_dofs,
                                        C.byref(t)), "emin_server_submit")
        self._borrowed[t.value] = (dsys, c)
        return t.value

    def done(self, ticket) -> bool:
        d = C.c_int32()
        _check(lib().emin_server_poll(self.s, ticket, C.byref(d)), "emin_server_poll")
        return bool(d.value)

    def wait(self, ticket):
        h = C.c_void_p()
        q, r = C.c_double(), C.c_double()
        _check(lib().emin_server_wait(self.s, ticket, C.byref(h), C.byref(q), C.byref(r)),
               "emin_server_wait")
        return HierarchyView(h), q.value, r.value

    def cancel(self, ticket) -> bool:
        """emin_server_cancel: True when the request left the queue unstarted."""
        c = C.c_int32()
        _check(lib().emin_server_cancel(self.s, ticket, C.byref(c)), "emin_server_cancel")
        return bool(c.value)

    def release(self, ticket):
        _check(lib().emin_server_release(self.s, ticket), "emin_server_release")
        self._borrowed.pop(ticket, None)

    def stats(self):
        m, q, r = C.c_int64(), C.c_int32(), C.c_int32()
        _check(lib().emin_server_stats(self.s, C.byref(m), C.byref(q), C.byref(r)),
               "emin_server_stats")
        return dict(in_use=m.value, queued=q.value, running=r.value)

    def close(self):
        if self.s:
            lib().emin_server_destroy(self.s)
            self.s = None
            self._borrowed.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------
# inf-sup diagnostic (sec. 6.1)
# ----------------------------------------------------------------------------
class DeviceMatrix:
    """A square or rectangular CSR in device memory: torch tensors
    (rowptr int64, col int32, val float64) or a library-owned matrix."""

    def __init__(self, nrows, ncols, nnz, rowptr, col, val, keep=None, handle=None):
        self.nrows, self.ncols, self.nnz = int(nrows), int(ncols), int(nnz)
        self.rowptr, self.col, self.val = rowptr, col, val
        self.keep = keep
        self.handle = handle

    @staticmethod
    def upload(m, device="cuda") -> "DeviceMatrix":
        import torch
        t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dt)
        r, c, v = t(m.rowptr, torch.int64), t(m.col, torch.int32), t(m.val, torch.float64)
        return DeviceMatrix(m.nrows, m.ncols, len(m.col), r.data_ptr(), c.data_ptr(),
                            v.data_ptr(), keep=(r, c, v))

    def c(self) -> c_csr:
        return c_csr(self.nrows, self.ncols, self.nnz, self.rowptr, self.col, self.val)

    def host(self):
        rp = d2h(self.rowptr, self.nrows + 1, np.int64)
        return rp, d2h(self.col, self.nnz, np.int32), d2h(self.val, self.nnz, np.float64)

    def close(self):
        if self.handle:
            _sync()
            lib().emin_matrix_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def galerkin(M: DeviceMatrix, P: DeviceMatrix, stream=None) -> DeviceMatrix:
    """emin_galerkin: P^T M P on the device."""
    h = C.c_void_p()
    mc, pc = M.c(), P.c()
    _check(lib().emin_galerkin(C.byref(mc), C.byref(pc), _stream(stream), C.byref(h)),
           "emin_galerkin")
    v = c_csr()
    _check(lib().emin_matrix_view(h, C.byref(v)), "emin_matrix_view")
    return DeviceMatrix(v.nrows, v.ncols, v.nnz, v.rowptr, v.col, v.val, keep=(M, P), handle=h)


def infsup(B: DeviceMatrix, Mv: DeviceMatrix, Mp: DeviceMatrix, dim: int, steps: int,
           rel: float = 1e-8, stream=None, resid: bool = False):
    """emin_infsup: (sigma_min, zero singular values, Lanczos steps taken),
    and the Ritz residual of sigma_min^2 last when resid is set."""
    sig, res, nz, st = C.c_double(), C.c_double(), C.c_int32(), C.c_int32()
    bc, vc, pc = B.c(), Mv.c(), Mp.c()
    _check(lib().emin_infsup(C.byref(bc), C.byref(vc), C.byref(pc), dim, steps, rel,
                             C.byref(sig), C.byref(res), C.byref(nz), C.byref(st),
                             _stream(stream)),
           "emin_infsup")
    if resid:
        return sig.value, nz.value, st.value, res.value
    return sig.value, nz.value, st.value


class Solver:
    """emin_solver_*: Braess-Sarazin V-cycle and V-cycle-preconditioned GMRES
    on a NativeHierarchy built from dsys (both must outlive the solver)."""

    def __init__(self, dsys: DeviceSystem, hier, nu=2, omega=0.666, gs_sweeps=5,
                 coarse_steps=10, stream=None):
        self.dsys, self.hier = dsys, hier
        self._c = dsys.c()
        h = C.c_void_p()
        _check(lib().emin_solver_create(C.byref(self._c), hier.h, nu, omega, gs_sweeps,
                                        coarse_steps, _stream(stream), C.byref(h)),
               "emin_solver_create")
        self.h = h

    def info(self, level=0):
        n, g = C.c_int64(), C.c_int32()
        _check(lib().emin_solver_info(self.h, level, C.byref(n), C.byref(g)), "emin_solver_info")
        return n.value, g.value

    def bs_step(self, level, x, f, stream=None):
        _check(lib().emin_solver_bs_step(self.h, level, C.c_void_p(x.data_ptr()),
                                         C.c_void_p(f.data_ptr()), _stream(stream)),
               "emin_solver_bs_step")

    def vcycle(self, f, x, stream=None):
        _check(lib().emin_solver_vcycle(self.h, C.c_void_p(f.data_ptr()),
                                        C.c_void_p(x.data_ptr()), _stream(stream)),
               "emin_solver_vcycle")

    def gmres(self, f, x, rtol=1e-6, maxit=200, stream=None):
        its, rel = C.c_int32(), C.c_double()
        _check(lib().emin_solver_gmres(self.h, C.c_void_p(f.data_ptr()), C.c_void_p(x.data_ptr()),
                                       rtol, maxit, C.byref(its), C.byref(rel), _stream(stream)),
               "emin_solver_gmres")
        return its.value, rel.value

    def close(self):
        if self.h:
            _sync()
            lib().emin_solver_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
