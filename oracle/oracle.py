"""ctypes wrapper of the plain C oracle (oracle/liboracle.so).

TEST INFRASTRUCTURE ONLY: the parity reference for the HIP library.  Only
the tests, the benchmark's CPU-baseline leg and the smoke check use it.
Array layouts follow the generator's (``paper_1607_02489_amd.synth``).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from paper_1607_02489_amd.synth import CSR, System

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "liboracle.so")

STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_SHAPE", 3: "ERR_PATTERN", 4: "ERR_VALUE",
          5: "ERR_INFEASIBLE", 6: "ERR_BREAKDOWN"}

# paper sec. 6: tau1 = 0.06, tau2 = sqrt(1.5e-3)
TAU1 = 0.06
TAU2_SQ = 1.5e-3


class c_csr(C.Structure):
    _fields_ = [("nrows", C.c_int64), ("ncols", C.c_int64),
                ("rowptr", C.POINTER(C.c_int64)), ("col", C.POINTER(C.c_int32)),
                ("val", C.POINTER(C.c_double))]


class c_level(C.Structure):
    _fields_ = [("status", C.c_int), ("dim", C.c_int),
                ("Mv", c_csr), ("Mp", c_csr),
                ("keep_v", C.POINTER(C.c_uint8)), ("keep_p", C.POINTER(C.c_uint8)),
                ("nnz_z", C.c_int64),
                ("dir", C.POINTER(C.c_uint8)),
                ("is_cp", C.POINTER(C.c_uint8)), ("S", c_csr),
                ("sdist", C.POINTER(C.c_int32)), ("order", C.POINTER(C.c_int32)),
                ("n_cp", C.c_int64), ("n_alg3", C.c_int64),
                ("cbar", C.POINTER(C.c_uint8)), ("n_mid", C.c_int64),
                ("is_cv", C.POINTER(C.c_uint8)), ("n_cv", C.c_int64), ("n_extra_v", C.c_int64),
                ("Pv", c_csr), ("Pp", c_csr),
                ("energy_v", C.POINTER(C.c_double)), ("energy_p", C.POINTER(C.c_double)),
                ("rho_v", C.POINTER(C.c_double)), ("rho_p", C.POINTER(C.c_double)),
                ("its_v", C.c_int), ("its_p", C.c_int),
                ("Ac", c_csr), ("Bc", c_csr),
                ("xv_c", C.POINTER(C.c_double)), ("p2v_c", C.POINTER(C.c_int32)),
                ("Rvt", c_csr), ("Gct", c_csr),
                ("energy_r", C.POINTER(C.c_double)), ("rho_r", C.POINTER(C.c_double)),
                ("its_r", C.c_int)]


class c_opts(C.Structure):
    _fields_ = [("tau1_v", C.c_double), ("tau1_p", C.c_double), ("tau2_sq", C.c_double),
                ("iters", C.c_int), ("energy_ata", C.c_int), ("gmres", C.c_int), ("pg", C.c_int),
                ("cp_in", C.POINTER(C.c_uint8))]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            from oracle.build import build
            build()
        L = C.CDLL(LIBPATH)
        P = C.POINTER
        L.orc_free.argtypes = [C.c_void_p]
        L.orc_csr_free.argtypes = [P(c_csr)]
        L.orc_spgemm.argtypes = [P(c_csr), P(c_csr), P(c_csr)]
        L.orc_transpose.argtypes = [P(c_csr), P(c_csr)]
        L.orc_filter.argtypes = [P(c_csr), C.c_double, P(c_csr), P(C.c_uint8)]
        L.orc_symmetrize.argtypes = [P(c_csr), P(c_csr)]
        L.orc_dirichlet.argtypes = [P(c_csr), P(C.c_uint8)]
        L.orc_coarsen_pressure.argtypes = [P(c_csr), P(C.c_double), C.c_int, P(C.c_uint8),
                                           P(c_csr), P(P(C.c_int32)), P(P(C.c_int32)),
                                           P(C.c_int64), P(C.c_int64)]
        L.orc_midpoints.argtypes = [P(c_csr), P(C.c_uint8), P(C.c_double), C.c_int, C.c_double,
                                    P(C.c_uint8), P(C.c_int64)]
        L.orc_velocity_pattern.argtypes = [P(c_csr), P(C.c_uint8), P(C.c_uint8), P(c_csr),
                                           P(C.c_int64)]
        L.orc_pressure_pattern.argtypes = [P(c_csr), P(C.c_uint8), P(c_csr)]
        L.orc_emin.argtypes = [P(c_csr), P(c_csr), P(C.c_int32), P(C.c_double), P(C.c_double),
                               C.c_int, P(C.c_double), P(C.c_double), P(C.c_double), P(C.c_int)]
        L.orc_rap.argtypes = [P(c_csr), P(c_csr), C.c_int, P(c_csr), P(c_csr), P(c_csr),
                              P(c_csr)]
        L.orc_emin_gmres.argtypes = [P(c_csr), P(c_csr), P(C.c_int32), P(C.c_double),
                                     P(C.c_double), C.c_int, P(C.c_double), P(C.c_int)]
        L.orc_level.argtypes = [C.c_int, P(c_csr), P(c_csr), P(C.c_double), P(C.c_int32),
                                C.c_double, C.c_double, C.c_double, C.c_int, C.c_int,
                                P(c_level)]
        L.orc_level_cp.argtypes = [C.c_int, P(c_csr), P(c_csr), P(C.c_double), P(C.c_int32),
                                   C.c_double, C.c_double, C.c_double, C.c_int, C.c_int,
                                   P(C.c_uint8), P(c_level)]
        L.orc_level_ex.argtypes = [C.c_int, P(c_csr), P(c_csr), P(C.c_double), P(C.c_double),
                                   P(C.c_int32), P(c_opts), P(c_level)]
        L.orc_level_free.argtypes = [P(c_level)]
        _lib = L
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


class _In:
    """Keeps numpy arrays alive while a c_csr views them."""

    def __init__(self, m: CSR, with_val=True):
        self.rowptr = np.ascontiguousarray(m.rowptr, dtype=np.int64)
        self.col = np.ascontiguousarray(m.col, dtype=np.int32)
        self.val = (np.ascontiguousarray(m.val, dtype=np.float64)
                    if (with_val and m.val is not None) else None)
        self.c = c_csr(m.nrows, m.ncols, _ptr(self.rowptr, C.c_int64), _ptr(self.col, C.c_int32),
                       _ptr(self.val, C.c_double) if self.val is not None else
                       C.POINTER(C.c_double)())


def _out(c: c_csr, free=True) -> CSR:
    n = c.nrows
    rp = np.ctypeslib.as_array(c.rowptr, shape=(n + 1,)).copy() if n >= 0 else None
    nnz = int(rp[-1])
    col = np.ctypeslib.as_array(c.col, shape=(max(nnz, 1),))[:nnz].copy()
    val = (np.ctypeslib.as_array(c.val, shape=(max(nnz, 1),))[:nnz].copy()
           if bool(c.val) else None)
    if free:
        lib().orc_csr_free(C.byref(c))
    return CSR(int(n), int(c.ncols), rp, col, val)


def _arr(p, n, dt):
    if n <= 0:
        return np.zeros(0, dtype=dt)
    return np.ctypeslib.as_array(p, shape=(n,)).astype(dt, copy=True)


def _check(st):
    if st != 0:
        raise OracleError(st)


class OracleError(RuntimeError):
    def __init__(self, status):
        super().__init__(f"oracle status {STATUS.get(status, status)}")
        self.status = status


# ----------------------------------------------------------------------------
def spgemm(A: CSR, B: CSR) -> CSR:
    a, b, c = _In(A), _In(B), c_csr()
    _check(lib().orc_spgemm(C.byref(a.c), C.byref(b.c), C.byref(c)))
    return _out(c)


def transpose(A: CSR) -> CSR:
    a, c = _In(A), c_csr()
    _check(lib().orc_transpose(C.byref(a.c), C.byref(c)))
    return _out(c)


def filter_lump(A: CSR, tau1: float):
    a, c = _In(A), c_csr()
    keep = np.zeros(max(A.nnz, 1), dtype=np.uint8)
    _check(lib().orc_filter(C.byref(a.c), tau1, C.byref(c), _ptr(keep, C.c_uint8)))
    return _out(c), keep[:A.nnz].astype(bool)


def symmetrize(A: CSR) -> CSR:
    a, c = _In(A), c_csr()
    _check(lib().orc_symmetrize(C.byref(a.c), C.byref(c)))
    return _out(c)


def dirichlet(A: CSR) -> np.ndarray:
    a = _In(A)
    d = np.zeros(max(A.nrows, 1), dtype=np.uint8)
    _check(lib().orc_dirichlet(C.byref(a.c), _ptr(d, C.c_uint8)))
    return d[:A.nrows].astype(bool)


@dataclass
class Coarsening:
    is_c: np.ndarray        # bool[n]
    S: CSR                  # fine C indices within distance 3 (sorted)
    sdist: np.ndarray       # distances of the S entries
    order: np.ndarray       # C points in selection order
    n_alg3: int


def coarsen_pressure(G: CSR, x: np.ndarray, dim: int) -> Coarsening:
    g = _In(G, with_val=False)
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = G.nrows
    is_c = np.zeros(max(n, 1), dtype=np.uint8)
    S = c_csr()
    sd = C.POINTER(C.c_int32)()
    order = C.POINTER(C.c_int32)()
    nc, na = C.c_int64(), C.c_int64()
    _check(lib().orc_coarsen_pressure(C.byref(g.c), _ptr(x, C.c_double), dim, _ptr(is_c, C.c_uint8),
                                      C.byref(S), C.byref(sd), C.byref(order),
                                      C.byref(nc), C.byref(na)))
    Sm = _out(S)
    sdist = _arr(sd, Sm.nnz, np.int32)
    lib().orc_free(sd)
    o = _arr(order, nc.value, np.int32)
    lib().orc_free(order)
    return Coarsening(is_c[:n].astype(bool), Sm, sdist, o, int(na.value))


def pressure_pattern(S: CSR, is_c: np.ndarray) -> CSR:
    s = _In(S, with_val=False)
    f = np.ascontiguousarray(is_c, dtype=np.uint8)
    c = c_csr()
    _check(lib().orc_pressure_pattern(C.byref(s.c), _ptr(f, C.c_uint8), C.byref(c)))
    return _out(c)


def midpoints(S: CSR, is_c: np.ndarray, x: np.ndarray, dim: int, tau2_sq: float = TAU2_SQ):
    s = _In(S, with_val=False)
    f = np.ascontiguousarray(is_c, dtype=np.uint8)
    cbar = f.copy()
    x = np.ascontiguousarray(x, dtype=np.float64)
    na = C.c_int64()
    _check(lib().orc_midpoints(C.byref(s.c), _ptr(f, C.c_uint8), _ptr(x, C.c_double), dim,
                               tau2_sq, _ptr(cbar, C.c_uint8), C.byref(na)))
    return cbar.astype(bool), int(na.value)


def velocity_pattern(G: CSR, dirf: np.ndarray, cv0: np.ndarray):
    g = _In(G, with_val=False)
    d = np.ascontiguousarray(dirf, dtype=np.uint8)
    cv = np.ascontiguousarray(cv0, dtype=np.uint8).copy()
    c = c_csr()
    ne = C.c_int64()
    _check(lib().orc_velocity_pattern(C.byref(g.c), _ptr(d, C.c_uint8), _ptr(cv, C.c_uint8),
                                      C.byref(c), C.byref(ne)))
    return cv.astype(bool), _out(c), int(ne.value)


@dataclass
class EminResult:
    P: CSR
    energy: np.ndarray
    rho: np.ndarray
    gamma: np.ndarray
    its: int
    status: int


def emin(M: CSR, N: CSR, cidx: np.ndarray, W: np.ndarray, Wc: np.ndarray, iters: int,
         raise_on_error: bool = True) -> EminResult:
    m = _In(M)
    p = _In(CSR(N.nrows, N.ncols, N.rowptr, N.col, np.zeros(N.nnz)))
    ci = np.ascontiguousarray(cidx, dtype=np.int32)
    W = np.ascontiguousarray(W, dtype=np.float64)
    Wc = np.ascontiguousarray(Wc, dtype=np.float64)
    e = np.zeros(iters + 1); r = np.zeros(iters + 1); g = np.zeros(max(iters, 1))
    its = C.c_int()
    st = lib().orc_emin(C.byref(m.c), C.byref(p.c), _ptr(ci, C.c_int32), _ptr(W, C.c_double),
                        _ptr(Wc, C.c_double), iters, _ptr(e, C.c_double), _ptr(r, C.c_double),
                        _ptr(g, C.c_double), C.byref(its))
    if st != 0 and raise_on_error:
        raise OracleError(st)
    P = CSR(N.nrows, N.ncols, N.rowptr.copy(), N.col.copy(), p.val.copy())
    return EminResult(P, e, r, g[:iters], its.value, st)


def emin_gmres(K: CSR, N: CSR, cidx: np.ndarray, W: np.ndarray, Wc: np.ndarray, iters: int,
               raise_on_error: bool = True) -> EminResult:
    """GMRES form of the constrained minimisation on a non-symmetric operator K
    (orc_emin_gmres); rho holds the squared residual norms."""
    m = _In(K)
    p = _In(CSR(N.nrows, N.ncols, N.rowptr, N.col, np.zeros(N.nnz)))
    ci = np.ascontiguousarray(cidx, dtype=np.int32)
    W = np.ascontiguousarray(W, dtype=np.float64)
    Wc = np.ascontiguousarray(Wc, dtype=np.float64)
    r = np.zeros(iters + 1)
    its = C.c_int()
    st = lib().orc_emin_gmres(C.byref(m.c), C.byref(p.c), _ptr(ci, C.c_int32), _ptr(W, C.c_double),
                              _ptr(Wc, C.c_double), iters, _ptr(r, C.c_double), C.byref(its))
    if st != 0 and raise_on_error:
        raise OracleError(st)
    P = CSR(N.nrows, N.ncols, N.rowptr.copy(), N.col.copy(), p.val.copy())
    return EminResult(P, np.zeros(iters + 1), r, np.zeros(max(iters, 0)), its.value, st)


def rap(Ahat: CSR, Bdiv: CSR, dim: int, Pv: CSR, Pp: CSR):
    a, b, pv, pp = _In(Ahat), _In(Bdiv), _In(Pv), _In(Pp)
    ac, bc = c_csr(), c_csr()
    _check(lib().orc_rap(C.byref(a.c), C.byref(b.c), dim, C.byref(pv.c), C.byref(pp.c),
                         C.byref(ac), C.byref(bc)))
    return _out(ac), _out(bc)


# ----------------------------------------------------------------------------
@dataclass
class Level:
    """Everything one level of the oracle produces (numpy copies)."""
    dim: int
    Mv: CSR
    Mp: CSR
    keep_v: np.ndarray
    keep_p: np.ndarray
    dir: np.ndarray
    is_cp: np.ndarray
    S: CSR
    sdist: np.ndarray
    order: np.ndarray
    n_alg3: int
    cbar: np.ndarray
    n_mid: int
    is_cv: np.ndarray
    n_extra_v: int
    Pv: CSR
    Pp: CSR
    energy_v: np.ndarray
    energy_p: np.ndarray
    rho_v: np.ndarray
    rho_p: np.ndarray
    its_v: int
    its_p: int
    Ac: CSR
    Bc: CSR
    xv_c: np.ndarray
    p2v_c: np.ndarray
    Rvt: CSR = None          # Petrov-Galerkin: R_v^T on Pv's pattern
    Gct: CSR = None          # coarse gradient block's transpose on Bc's pattern
    rho_r: np.ndarray = None
    its_r: int = 0

    def coarse_system(self, meta=None) -> System:
        m = dict(meta or {})
        if self.Gct is not None:
            m["Gt"] = self.Gct.val
        return System(self.dim, self.Ac, self.Bc, self.xv_c, self.p2v_c, meta=m)


def level(sys: System, tau1_v: float = TAU1, tau1_p: float = TAU1, tau2_sq: float = TAU2_SQ,
          iters: int = 5, energy_ata: bool = False, cpoints=None, gmres: bool = False,
          pg: bool = False) -> Level:
    """One level of Alg. 1 (orc_level).  energy_ata: the velocity block's EMIN
    energy is the A^T A-norm of the filtered operator (sec. 4.3, eq.
    (min_problem), for non-symmetric operators) instead of the norm of its
    symmetric part; the velocity graph is the same either way.  cpoints: the
    coarse pressures (bool[n_p]) given instead of chosen by Alg. 3
    (orc_level_cp)."""
    a, b = _In(sys.Ahat), _In(sys.Bdiv)
    xv = np.ascontiguousarray(sys.xv, dtype=np.float64)
    p2v = np.ascontiguousarray(sys.p2v, dtype=np.int32)
    L = c_level()
    cp = (None if cpoints is None else
          np.ascontiguousarray(np.asarray(cpoints, dtype=bool).astype(np.uint8)))
    o = c_opts(tau1_v, tau1_p, tau2_sq, iters, 1 if energy_ata else 0, 1 if gmres else 0,
               1 if pg else 0, _ptr(cp, C.c_uint8) if cp is not None else C.POINTER(C.c_uint8)())
    gt = sys.meta.get("Gt") if getattr(sys, "meta", None) else None
    gt = None if gt is None else np.ascontiguousarray(gt, dtype=np.float64)
    st = lib().orc_level_ex(sys.dim, C.byref(a.c), C.byref(b.c),
                            _ptr(gt, C.c_double) if gt is not None else C.POINTER(C.c_double)(),
                            _ptr(xv, C.c_double), _ptr(p2v, C.c_int32), C.byref(o), C.byref(L))
    try:
        _check(st)
        nv, np_, d = sys.n_v, sys.n_p, sys.dim
        out = Level(
            dim=d,
            Mv=_out(L.Mv, free=False), Mp=_out(L.Mp, free=False),
            keep_v=_arr(L.keep_v, sys.Ahat.nnz, np.uint8).astype(bool),
            keep_p=_arr(L.keep_p, L.nnz_z, np.uint8).astype(bool),
            dir=_arr(L.dir, nv, np.uint8).astype(bool),
            is_cp=_arr(L.is_cp, np_, np.uint8).astype(bool),
            S=_out(L.S, free=False), sdist=None,
            order=_arr(L.order, L.n_cp, np.int32), n_alg3=int(L.n_alg3),
            cbar=_arr(L.cbar, np_, np.uint8).astype(bool), n_mid=int(L.n_mid),
            is_cv=_arr(L.is_cv, nv, np.uint8).astype(bool), n_extra_v=int(L.n_extra_v),
            Pv=_out(L.Pv, free=False), Pp=_out(L.Pp, free=False),
            energy_v=_arr(L.energy_v, iters + 1, np.float64),
            energy_p=_arr(L.energy_p, iters + 1, np.float64),
            rho_v=_arr(L.rho_v, iters + 1, np.float64),
            rho_p=_arr(L.rho_p, iters + 1, np.float64),
            its_v=int(L.its_v), its_p=int(L.its_p),
            Ac=_out(L.Ac, free=False), Bc=_out(L.Bc, free=False),
            xv_c=_arr(L.xv_c, int(L.n_cv) * d, np.float64).reshape(-1, d),
            p2v_c=_arr(L.p2v_c, int(L.n_cp), np.int32))
        out.sdist = _arr(L.sdist, out.S.nnz, np.int32)
        if pg:
            out.Rvt = _out(L.Rvt, free=False)
            out.Gct = _out(L.Gct, free=False)
            out.rho_r = _arr(L.rho_r, iters + 1, np.float64)
            out.its_r = int(L.its_r)
        return out
    finally:
        lib().orc_level_free(C.byref(L))


def hierarchy(sys: System, nlevels: int, tau1_v: float = TAU1, tau1_p: float = TAU1,
              tau2_sq: float = TAU2_SQ, iters: int = 5, min_dofs: int = 0,
              energy_ata: bool = False, gmres: bool = False, pg: bool = False):
    """Alg. 1 without relaxation: levels 0..nlevels-1 (nlevels-1 transfers),
    stopping early when a level has at most min_dofs dofs."""
    out = []
    cur = sys
    for _ in range(nlevels - 1):
        if cur.dofs <= min_dofs:
            break
        L = level(cur, tau1_v, tau1_p, tau2_sq, iters, energy_ata=energy_ata, gmres=gmres, pg=pg)
        out.append(L)
        cur = L.coarse_system()
    return out, cur


# ----------------------------------------------------------------------------
# inf-sup diagnostic (sec. 6.1, Table 3)
# ----------------------------------------------------------------------------
def galerkin(M: CSR, P: CSR) -> CSR:
    """P^T M P with the oracle's sparse product and transpose (the projection
    of a mass matrix to the next level, sec. 6.1)."""
    return spgemm(transpose(P), spgemm(M, P))


def lumped_abs(M: CSR) -> np.ndarray:
    """lump(|M|): the diagonal of row sums of |m_ij|, as a vector."""
    rows = np.repeat(np.arange(M.nrows), np.diff(M.rowptr))
    out = np.zeros(M.nrows)
    np.add.at(out, rows, np.abs(M.val))
    return out


def infsup_singular_values(B: CSR, Mv: CSR, Mp: CSR, dim: int):
    """sec. 6.1: every singular value of the mass-scaled divergence
    B~ = lump(|M_p|)^(-1/2) B lump(|M_v|)^(-1/2), M_v acting on each velocity
    component (I_d (x) M_v), by dense SVD (small problems), descending."""
    dp = lumped_abs(Mp)
    dv = np.tile(lumped_abs(Mv), dim)
    Bd = np.zeros((B.nrows, B.ncols))
    rows = np.repeat(np.arange(B.nrows), np.diff(B.rowptr))
    Bd[rows, B.col] = B.val
    Bt = Bd / np.sqrt(dp)[:, None] / np.sqrt(dv)[None, :]
    return np.linalg.svd(Bt, compute_uv=False)


def infsup_sigma_min(B: CSR, Mv: CSR, Mp: CSR, dim: int, rel: float = 1e-8):
    """sec. 6.1: the smallest non-zero singular value of B~ (as in
    infsup_singular_values); singular values below rel * sigma_max count as
    zero.  Returns (sigma_min, number of zero singular values, sigma_max)."""
    sv = infsup_singular_values(B, Mv, Mp, dim)
    smax = float(sv.max()) if sv.size else 0.0
    nz = sv[sv > rel * smax]
    return (float(nz.min()) if nz.size else 0.0), int(sv.size - nz.size), smax
