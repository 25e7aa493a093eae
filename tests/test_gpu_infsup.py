"""GPU tests of the inf-sup diagnostic of sec. 6.1 (Table 3): the coarse mass
matrices P^T M P and sigma_min of the mass-scaled divergence, through the C
ABI, against the oracle (dense products, dense SVD)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1607_02489_amd import synth
from paper_1607_02489_amd.synth import CSR
from tests.gpu_util import gpu_level, say
from tests.helpers import relfro

pytestmark = pytest.mark.gpu


def _dm(m):
    from paper_1607_02489_amd import emin as E
    return E.DeviceMatrix.upload(m)


@pytest.mark.parametrize("dim,n", [(2, 8), (2, 16), (3, 4)])
def test_infsup_full_lanczos_equals_dense_svd(dim, n):
    """With as many Lanczos steps as pressures the Ritz values are the
    eigenvalues of B~ B~^T: sigma_min and the number of zero singular values
    (one, the hydrostatic pressure) equal the dense SVD's."""
    from paper_1607_02489_amd import emin as E
    s = synth.make_system(dim, n, jitter=0.05, seed=1, mass=True)
    say(f"[gpu] inf-sup, full Lanczos, dim={dim} n={n}: n_p={s.n_p}")
    want, z, _ = O.infsup_sigma_min(s.Bdiv, s.meta["Mv"], s.meta["Mp"], dim)
    got, gz, steps = E.infsup(_dm(s.Bdiv), _dm(s.meta["Mv"]), _dm(s.meta["Mp"]), dim, s.n_p)
    assert gz == z == 1
    assert abs(got - want) <= 1e-8 * want, (got, want)


def test_galerkin_mass_and_level_chain():
    """Three levels of a 2-D Stokes cavity hierarchy: each level's mass
    matrices projected by the GPU's P (emin_galerkin) equal the oracle's
    P^T M P on the same inputs (pattern exact, values to 1e-13), and each
    level's sigma_min equals the dense SVD of that level's scaled divergence."""
    import torch
    from paper_1607_02489_amd import emin as E
    s = synth.make_system(2, 32, mass=True)
    cur, Mv, Mp = s, s.meta["Mv"], s.meta["Mp"]
    for lev in range(3):
        got, gz, _ = E.infsup(_dm(cur.Bdiv), _dm(Mv), _dm(Mp), 2, cur.n_p)
        want, z, _ = O.infsup_sigma_min(cur.Bdiv, Mv, Mp, 2)
        say(f"[gpu] level {lev}: n_p={cur.n_p} sigma_min gpu {got:.6f} oracle {want:.6f}")
        assert gz == z and abs(got - want) <= 1e-8 * want
        if cur.dofs < 300:
            break
        g = gpu_level(cur, iters=5)
        Pv, Pp = g["Pv"], g["Pp"]
        Mv1 = E.galerkin(_dm(Mv), _dm(Pv))
        Mp1 = E.galerkin(_dm(Mp), _dm(Pp))
        rp, col, val = Mv1.host()
        ref = O.galerkin(Mv, Pv)
        assert np.array_equal(rp, ref.rowptr) and np.array_equal(col, ref.col)
        assert relfro(val, ref.val) <= 1e-13
        rp2, col2, val2 = Mp1.host()
        ref2 = O.galerkin(Mp, Pp)
        assert np.array_equal(col2, ref2.col) and relfro(val2, ref2.val) <= 1e-13
        Mv, Mp = CSR(ref.nrows, ref.ncols, rp, col, val), CSR(ref2.nrows, ref2.ncols, rp2, col2, val2)
        cur = synth.System(2, g["Ac"], g["Bc"], g["xv_c"], g["p2v_c"])
        Mv1.close()
        Mp1.close()


def test_infsup_ritz_residual_brackets_an_eigenvalue():
    """Few Lanczos steps (2-D cavity 16x16, 289 pressures, 12 and 40 steps):
    the reported sigma_min^2 lies within the reported Ritz residual of an
    eigenvalue of B~ B~^T (dense SVD), and is not below the smallest non-zero
    one (Ritz values of the complement approach it from above)."""
    from paper_1607_02489_amd import emin as E
    s = synth.make_system(2, 16, jitter=0.05, seed=3, mass=True)
    sv = O.infsup_singular_values(s.Bdiv, s.meta["Mv"], s.meta["Mp"], 2)
    ev = np.sort(sv ** 2)
    lam_min = ev[ev > 1e-16 * ev[-1]].min()
    a = _dm(s.Bdiv), _dm(s.meta["Mv"]), _dm(s.meta["Mp"])
    prev = None
    for steps in (12, 40):
        sig, z, st, res = E.infsup(*a, 2, steps, resid=True)
        th = sig * sig
        say(f"[gpu] 16^2, {steps} steps: sigma {sig:.8f} resid {res:.3e}, "
            f"nearest eigenvalue gap {np.abs(ev - th).min():.3e}")
        assert z == 1 and st == steps
        assert np.abs(ev - th).min() <= res * (1 + 1e-8) + 1e-12 * ev[-1]
        assert th >= lam_min * (1 - 1e-12)
        if prev is not None:
            assert sig <= prev * (1 + 1e-12)
        prev = sig


def test_infsup_sizes_beyond_dense():
    """2-D Stokes cavity 128x128 (16,641 pressures): one zero singular value;
    the smallest Ritz value falls as steps grow (150, 400, 600) and has
    converged by 400 (residual below 1e-6 sigma^2 at 600, 400 and 600 equal to
    1e-8); sigma_min lies between the 64x64 value (250 steps, also converged)
    and pi: it rises towards pi under refinement."""
    from paper_1607_02489_amd import emin as E
    s = synth.make_system(2, 128, mass=True)
    a = _dm(s.Bdiv), _dm(s.meta["Mv"]), _dm(s.meta["Mp"])
    r = {k: E.infsup(*a, 2, k, resid=True) for k in (150, 400, 600)}
    c = synth.make_system(2, 64, mass=True)
    s64, _, _, r64 = E.infsup(_dm(c.Bdiv), _dm(c.meta["Mv"]), _dm(c.meta["Mp"]), 2, 250,
                              resid=True)
    for k, (sg, z, st, res) in r.items():
        say(f"[gpu] inf-sup 128^2, {k} steps: sigma {sg:.10f} resid {res:.3e} (zero: {z})")
    say(f"[gpu] inf-sup 64^2, 250 steps: sigma {s64:.10f} resid {r64:.3e}")
    s150, s400, s600 = r[150][0], r[400][0], r[600][0]
    assert all(v[1] == 1 for v in r.values())
    assert s150 >= s400 * (1 - 1e-12) and s400 >= s600 * (1 - 1e-12)
    assert r[600][3] <= 1e-6 * s600 ** 2 and r64 <= 1e-6 * s64 ** 2
    assert abs(s400 - s600) <= 1e-8 * s600
    assert s64 < s600 < np.pi
