"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Coarsening, mid-points, patterns and drop masks must match bit for bit; P,
RAP and the CG energies to 1e-10 relative Frobenius in FP64.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1607_02489_amd import synth
from tests.gpu_util import compare_level, gpu_level, host_coarse, say
from tests.helpers import relfro

pytestmark = pytest.mark.gpu

CASES = {
    "cfg1_stokes2d_8": lambda: (synth.stokes2d_small(), {}),
    "stokes2d_13_jitter": lambda: (synth.make_system(2, 13, jitter=0.1, seed=4), {}),
    "oseen2d_16_uniform": lambda: (synth.make_system(2, 16, nu=0.01, wind="stream", seed=2), {}),
    "oseen2d_40_jitter": lambda: (synth.make_system(2, 40, jitter=0.1, nu=0.002, wind="stream",
                                                    seed=9), {}),
    "stokes3d_5": lambda: (synth.make_system(3, 5, jitter=0.05, seed=3),
                           dict(tau1_v=0.038, tau1_p=0.04)),
    "oseen3d_6": lambda: (synth.make_system(3, 6, jitter=0.05, nu=0.02, wind="stream", seed=6),
                          dict(tau1_v=0.038, tau1_p=0.04)),
}


@pytest.mark.parametrize("case", list(CASES))
def test_level_parity(case):
    s, kw = CASES[case]()
    say(f"[gpu] level parity {case}: dofs={s.dofs}")
    L = O.level(s, iters=5, **kw)
    g = gpu_level(s, iters=5, **kw)
    compare_level(g, L)


def test_fp_div_sqrt_bitwise():
    """The integer decisions rely on IEEE-correct division and square root on
    the GPU (they are compared bitwise with the CPU's)."""
    import ctypes as C
    import torch
    from paper_1607_02489_amd import emin as E
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.uniform(1e-6, 10.0, 500000), np.exp(rng.uniform(-600, 600, 500000))])
    xt = torch.from_numpy(x).cuda()
    s = torch.empty_like(xt)
    r = torch.empty_like(xt)
    st = E.lib().emin_fp_probe(C.c_void_p(xt.data_ptr()), C.c_void_p(s.data_ptr()),
                               C.c_void_p(r.data_ptr()), C.c_int64(x.size), None)
    assert st == 0
    torch.cuda.synchronize()
    assert np.array_equal(s.cpu().numpy(), np.sqrt(x))
    assert np.array_equal(r.cpu().numpy(), 1.0 / x)


def test_deterministic_and_resetup():
    """Two setups on one pattern are bitwise equal (fixed reduction trees)."""
    import torch
    from paper_1607_02489_amd import emin as E
    s = synth.make_system(2, 24, jitter=0.1, seed=8)
    d = E.DeviceSystem.upload(s)
    prm = E.params(iters=5)
    pat = E.Pattern(d, prm)
    z = pat.sizes
    P1 = [torch.empty(max(z[k], 1), dtype=torch.float64, device="cuda") for k in ("nnz_Pv", "nnz_Pp")]
    P2 = [torch.empty_like(t) for t in P1]
    pat.setup(prm, P1[0].data_ptr(), P1[1].data_ptr())
    pat.setup(prm, P2[0].data_ptr(), P2[1].data_ptr())
    torch.cuda.synchronize()
    assert torch.equal(P1[0], P2[0]) and torch.equal(P1[1], P2[1])


def test_picard_resetup_matches_fresh_oracle():
    """emin_setup with new values on the stored structure (a new Picard
    linearisation) equals the oracle on those values when the drop masks
    agree."""
    import torch
    from paper_1607_02489_amd import emin as E
    a = synth.make_system(2, 16, nu=0.01, wind="stream", seed=2)
    b = synth.make_system(2, 16, nu=0.01, wind="stream", seed=2)
    b.Ahat.val = a.Ahat.val * 1.0 + 1e-9 * np.sign(a.Ahat.val)  # same structure, new values
    da, db = E.DeviceSystem.upload(a), E.DeviceSystem.upload(b)
    prm = E.params(iters=5)
    pat = E.Pattern(da, prm)
    z = pat.sizes
    Pv = torch.empty(z["nnz_Pv"], dtype=torch.float64, device="cuda")
    Pp = torch.empty(z["nnz_Pp"], dtype=torch.float64, device="cuda")
    pat._c = db.c()
    pat.setup(prm, Pv.data_ptr(), Pp.data_ptr())
    torch.cuda.synchronize()
    Lb = O.level(b, iters=5)
    La = O.level(a, iters=5)
    if np.array_equal(La.keep_v, Lb.keep_v) and np.array_equal(La.keep_p, Lb.keep_p):
        assert relfro(Pv.cpu().numpy(), Lb.Pv.val) <= 1e-10


def test_hierarchy_cfg2_small_per_level():
    """A 4-level Oseen hierarchy: every level's coarsening is bit-exact against
    the oracle run on the GPU's own input for that level."""
    s = synth.oseen2d(64)
    cur = s
    keep = []
    for lev in range(3):
        say(f"[gpu] hierarchy level {lev}: dofs={cur.dofs}")
        L = O.level(cur, iters=5)
        g = gpu_level(cur, iters=5)
        keep.append(g)
        compare_level(g, L)
        cur = host_coarse(g, s.dim)
