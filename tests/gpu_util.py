"""Helpers of the GPU parity tests: run one level through the C ABI and fetch
every stage to host memory, and compare it with the oracle's level."""
from __future__ import annotations

import sys

import numpy as np

from paper_1607_02489_amd.synth import CSR, System
from tests.helpers import relfro


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_level(sys_: System, tau1_v=0.06, tau1_p=0.06, tau2_sq=1.5e-3, iters=5, mixed=False,
              energy=True, dsys=None, energy_ata=False, cpoints=None, staged=False,
              gmres=False, pg=False):
    import torch
    from paper_1607_02489_amd import emin as E
    d = dsys if dsys is not None else E.DeviceSystem.upload(sys_)
    prm = E.params(tau1_v, tau1_p, tau2_sq, iters, mixed=mixed, energy=energy,
                   energy_ata=energy_ata, staged=staged, gmres=gmres, pg=pg)
    pat = E.Pattern(d, prm, cpoints=cpoints)
    s = pat.sizes
    f64 = dict(dtype=torch.float64, device="cuda")
    Pv = torch.empty(max(s["nnz_Pv"], 1), **f64)
    Pp = torch.empty(max(s["nnz_Pp"], 1), **f64)
    Ac = torch.empty(max(s["nnz_Ac"], 1), **f64)
    Bc = torch.empty(max(s["nnz_Bc"], 1), **f64)
    rep = E.new_report()
    Rvt = Gct = None
    if pg:
        Rvt = torch.empty(max(s["nnz_Pv"], 1), **f64)
        Gct = torch.empty(max(s["nnz_Bc"], 1), **f64)
        pat.setup_pg(prm, Pv.data_ptr(), Pp.data_ptr(), Rvt.data_ptr(), rep.data_ptr())
        pat.rap_pg(Pv.data_ptr(), Pp.data_ptr(), Rvt.data_ptr(), Ac.data_ptr(), Bc.data_ptr(),
                   Gct.data_ptr())
    else:
        pat.setup(prm, Pv.data_ptr(), Pp.data_ptr(), rep.data_ptr())
        pat.rap(Pv.data_ptr(), Pp.data_ptr(), Ac.data_ptr(), Bc.data_ptr(), mixed=mixed)
    torch.cuda.synchronize()
    r = E.sync_report(rep, raise_on_error=False)
    out = dict(sizes=s, status=r.status, its_v=r.its_v, its_p=r.its_p)
    if pg:
        out["its_r"] = r.its_r
        out["rho_r"] = np.array(r.rho_r[:iters + 1])
    out["energy_v"] = np.array(r.energy_v[:iters + 1])
    out["energy_p"] = np.array(r.energy_p[:iters + 1])
    out["rho_v"] = np.array(r.rho_v[:iters + 1])
    out["rho_p"] = np.array(r.rho_p[:iters + 1])

    def csr(what, vals=None):
        n, nc, rp, col, val = pat.csr_host(what, vals)
        return CSR(int(n), int(nc), rp, col, val)

    out["Mv"] = csr(E.VIEW_MV)
    out["Mp"] = csr(E.VIEW_MP)
    out["S"] = csr(E.VIEW_S)
    out["Pv"] = csr(E.VIEW_PV, Pv.data_ptr())
    out["Pp"] = csr(E.VIEW_PP, Pp.data_ptr())
    out["Ac"] = csr(E.VIEW_AC, Ac.data_ptr())
    out["Bc"] = csr(E.VIEW_BC, Bc.data_ptr())
    out["order"] = pat.array_host(E.VIEW_ORDER, np.int32)
    out["Cp"] = pat.array_host(E.VIEW_CP, np.int32)
    out["cbar"] = pat.array_host(E.VIEW_CBAR, np.uint8).astype(bool)
    out["Cv"] = pat.array_host(E.VIEW_CV, np.int32)
    out["xv_c"] = pat.array_host(E.VIEW_XVC, np.float64).reshape(-1, sys_.dim if sys_ else d.dim)
    out["p2v_c"] = pat.array_host(E.VIEW_P2VC, np.int32)
    out["keep_v"] = pat.array_host(E.VIEW_KEEPV, np.uint8).astype(bool)
    out["keep_p"] = pat.array_host(E.VIEW_KEEPP, np.uint8).astype(bool)
    out["dir"] = pat.array_host(E.VIEW_DIR, np.uint8).astype(bool)
    if pg:
        out["Rvt"] = csr(E.VIEW_PV, Rvt.data_ptr())
        out["Gct"] = csr(E.VIEW_BC, Gct.data_ptr())
    out["_keep"] = (pat, Pv, Pp, Ac, Bc, d, Rvt, Gct)
    return out


def same_pattern(a: CSR, b: CSR) -> bool:
    return (a.nrows == b.nrows and a.ncols == b.ncols and np.array_equal(a.rowptr, b.rowptr)
            and np.array_equal(a.col, b.col))


def rowmax_err(got: CSR, want: CSR, floor=1e-6) -> float:
    """Largest per-row error: max over rows of max|got - want| in the row
    divided by the row's largest |want| (floored at floor times the whole
    matrix's largest |want|, so rows that cancel to nothing compare at that
    scale).  Catches an error confined to a few entries that a Frobenius norm
    over the whole matrix would average away."""
    a = np.asarray(got.val, dtype=np.float64)
    b = np.asarray(want.val, dtype=np.float64)
    if b.size == 0:
        return 0.0
    rows = np.repeat(np.arange(want.nrows), np.diff(want.rowptr))
    err = np.zeros(want.nrows)
    scale = np.zeros(want.nrows)
    np.maximum.at(err, rows, np.abs(a - b))
    np.maximum.at(scale, rows, np.abs(b))
    scale = np.maximum(scale, floor * np.abs(b).max())
    scale[scale == 0.0] = 1.0
    return float((err / scale).max())


def compare_level(g, L, iters=5, tol=1e-10, values_exact=True):
    """Asserts parity of a GPU level `g` against the oracle level `L`."""
    assert g["status"] == 0, g["status"]
    # a1/a2: drop masks bit-exact; energy operators identical (same op order)
    assert np.array_equal(g["keep_v"], L.keep_v)
    assert np.array_equal(g["keep_p"], L.keep_p)
    assert np.array_equal(g["dir"], L.dir)
    for k in ("Mv", "Mp"):
        assert same_pattern(g[k], getattr(L, k)), k
        if values_exact:
            assert np.array_equal(g[k].val, getattr(L, k).val), k
    # a4-a8: coarsening and patterns bit-exact
    assert np.array_equal(g["order"], L.order)
    assert np.array_equal(g["Cp"], np.nonzero(L.is_cp)[0])
    assert same_pattern(g["S"], L.S)
    assert np.array_equal(g["cbar"], L.cbar)
    assert np.array_equal(g["Cv"], np.nonzero(L.is_cv)[0])
    assert same_pattern(g["Pv"], L.Pv)
    assert same_pattern(g["Pp"], L.Pp)
    assert g["sizes"]["n_cp_alg3"] == L.n_alg3
    assert g["sizes"]["n_cv_extra"] == L.n_extra_v
    # a9-a12: P to the FP64 tolerance; CG scalars too
    assert relfro(g["Pv"].val, L.Pv.val) <= tol
    assert relfro(g["Pp"].val, L.Pp.val) <= tol
    assert rowmax_err(g["Pv"], L.Pv) <= tol
    assert rowmax_err(g["Pp"], L.Pp) <= tol
    assert g["its_v"] == L.its_v and g["its_p"] == L.its_p
    assert relfro(g["energy_v"], L.energy_v) <= tol
    assert relfro(g["energy_p"], L.energy_p) <= tol
    # a13/a14: RAP patterns exact, values to tolerance; coarse descriptors exact
    assert same_pattern(g["Ac"], L.Ac)
    assert same_pattern(g["Bc"], L.Bc)
    assert relfro(g["Ac"].val, L.Ac.val) <= tol
    assert relfro(g["Bc"].val, L.Bc.val) <= tol
    assert rowmax_err(g["Ac"], L.Ac) <= tol
    assert rowmax_err(g["Bc"], L.Bc) <= tol
    assert np.array_equal(g["xv_c"], L.xv_c)
    assert np.array_equal(g["p2v_c"], L.p2v_c)


def host_coarse(g, dim) -> System:
    """The GPU's coarse system as host arrays (input of the next level)."""
    meta = {"Gt": g["Gct"].val} if "Gct" in g else {}
    return System(dim, g["Ac"], g["Bc"], g["xv_c"], g["p2v_c"], meta=meta)
