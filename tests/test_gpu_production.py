"""GPU tests of the production forms: the native hierarchy driver, batched
builds with a graph-captured numeric phase, and the serving loop.  Every
result must equal the same request built alone (the kernels are
deterministic, so bit for bit)."""
import numpy as np
import pytest

from paper_1607_02489_amd import synth
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _levels(view):
    return [view.level_host(l) for l in range(view.ntransfers())]


def _same(la, lb):
    assert len(la) == len(lb)
    for a, b in zip(la, lb):
        for k in ("Pv", "Pp", "Ac", "Bc"):
            assert np.array_equal(a[k], b[k]), k


def _systems():
    out = []
    for i, (n, re_) in enumerate([(12, 10.0), (16, 100.0), (20, 1.0), (9, 300.0), (24, 50.0),
                                  (14, 500.0)]):
        out.append(synth.make_system(2, n, nu=1.0 / re_, wind="stream", seed=1000 + i))
    return out


def test_native_hierarchy_matches_level_calls():
    import torch
    from paper_1607_02489_amd import emin as E
    s = synth.oseen2d(32)
    prm = E.params(iters=5)
    H = E.Hierarchy(s, 4, prm).build()
    torch.cuda.synchronize()
    N = E.NativeHierarchy(H.fine, prm, 4)
    torch.cuda.synchronize()
    assert N.ntransfers() == len(H.levels)
    for l, L in enumerate(H.levels):
        got = N.level_host(l)
        assert np.array_equal(got["Pv"], L.Pv.cpu().numpy()[:L.pattern.sizes["nnz_Pv"]])
        assert np.array_equal(got["Ac"], L.Ac.cpu().numpy()[:L.pattern.sizes["nnz_Ac"]])
    N.close()
    H.close()


def test_batch_build_equals_alone():
    import torch
    from paper_1607_02489_amd import emin as E
    systems = _systems()
    prm = E.params(iters=5, mixed=True)
    ds = [E.DeviceSystem.upload(s) for s in systems]
    say(f"[gpu] batch build of {len(ds)} systems")
    hs = E.build_batch(ds, prm, 4, min_dofs=200, max_parallel=len(ds))
    torch.cuda.synchronize()
    for d, h in zip(ds, hs):
        alone = E.NativeHierarchy(d, prm, 4, min_dofs=200)
        torch.cuda.synchronize()
        _same(_levels(h), _levels(alone))
        alone.close()
    for h in hs:
        h.close()


def test_batch_graph_replays_match_eager():
    """The captured numeric phase of several hierarchies, replayed after the
    level-0 values change (new Picard linearisations), equals an eager
    re-setup of twin hierarchies; replays alternate with other eager work."""
    import torch
    from paper_1607_02489_amd import emin as E
    systems = _systems()[:4]
    prm = E.params(iters=5)
    ds = [E.DeviceSystem.upload(s) for s in systems]
    hs = E.build_batch(ds, prm, 3, max_parallel=4)
    twins = [E.NativeHierarchy(d, prm, 3) for d in ds]
    torch.cuda.synchronize()
    B = E.Batch(hs)
    for rep in range(3):
        for d in ds:
            d.keep[2].mul_(1.0 + 0.01 * (rep + 1))       # Ahat values, in place
        torch.cuda.synchronize()
        B.run()
        for t in twins:
            t.resetup()
        torch.cuda.synchronize()
        for h, t in zip(hs, twins):
            _same(_levels(h), _levels(t))
    B.close()
    for h in hs + twins:
        h.close()


def test_batch_graph_replay_ata():
    """The captured numeric phase with the A^T A-norm energy: the replay also
    re-forms A~^T A~ from the new values before the masked products, and
    equals an eager re-setup of twin hierarchies."""
    import torch
    from paper_1607_02489_amd import emin as E
    systems = _systems()[:2]
    prm = E.params(iters=5, energy_ata=True)
    ds = [E.DeviceSystem.upload(s) for s in systems]
    hs = E.build_batch(ds, prm, 3, max_parallel=2)
    twins = [E.NativeHierarchy(d, prm, 3) for d in ds]
    torch.cuda.synchronize()
    B = E.Batch(hs)
    for rep in range(2):
        for d in ds:
            d.keep[2].mul_(1.0 + 0.02 * (rep + 1))       # Ahat values, in place
        torch.cuda.synchronize()
        B.run()
        for t in twins:
            t.resetup()
        torch.cuda.synchronize()
        for h, t in zip(hs, twins):
            _same(_levels(h), _levels(t))
    B.close()
    for h in hs + twins:
        h.close()


def test_server_mix_equals_alone_and_fifo_admission():
    import time
    import torch
    from paper_1607_02489_amd import emin as E
    systems = _systems()
    prm = E.params(iters=5, mixed=True)
    ds = [E.DeviceSystem.upload(s) for s in systems]
    alone = []
    for d in ds:
        h = E.NativeHierarchy(d, prm, 4, min_dofs=200)
        torch.cuda.synchronize()
        alone.append(_levels(h))
        h.close()
    # a budget that fits about two requests at a time forces queueing
    srv = E.Server(budget_bytes=3 * (64 << 20) * 5, slots=3)
    t0 = time.perf_counter()
    tickets, submitted = [], []
    for d in ds + ds:
        tickets.append(srv.submit(d, prm, 4, min_dofs=200))
        submitted.append(time.perf_counter() - t0)
    starts = []
    for i, t in enumerate(tickets):
        view, q_ms, r_ms = srv.wait(t)
        starts.append(submitted[i] + q_ms * 1e-3)
        _same(_levels(view), alone[i % len(ds)])
        srv.release(t)
    # admission in arrival order (start times follow ticket order up to clock noise)
    assert all(b >= a - 5e-3 for a, b in zip(starts, starts[1:]))
    assert srv.stats()["in_use"] == 0
    srv.close()


def test_server_rejects_over_budget():
    from paper_1607_02489_amd import emin as E
    srv = E.Server(budget_bytes=1 << 20, slots=1)
    d = E.DeviceSystem.upload(synth.make_system(2, 8))
    with pytest.raises(E.EminError) as ei:
        srv.submit(d, E.params(), 2)
    assert ei.value.status == 7                      # ERR_BUDGET
    srv.close()


def test_server_cancel_queued_request():
    """emin_server_cancel: with a budget that admits one request at a time, a
    request queued behind an unreleased one is cancelled (wait reports
    EMIN_ERR_CANCELLED), a finished one is not, and the queue moves on."""
    import torch
    from paper_1607_02489_amd import emin as E
    d = E.DeviceSystem.upload(synth.make_system(2, 16))
    prm = E.params(iters=5)
    srv = E.Server(budget_bytes=300 << 20, slots=2)
    a = srv.submit(d, prm, 2)
    srv.wait(a)
    b = srv.submit(d, prm, 2)          # cannot fit while a holds its memory
    assert srv.stats()["queued"] == 1
    assert srv.cancel(b) and not srv.cancel(a)
    with pytest.raises(E.EminError) as ei:
        srv.wait(b)
    assert ei.value.status == 12                     # ERR_CANCELLED
    srv.release(b)
    srv.release(a)
    c = srv.submit(d, prm, 2)
    view, _, _ = srv.wait(c)
    torch.cuda.synchronize()
    srv.release(c)
    assert srv.stats() == dict(in_use=0, queued=0, running=0)
    srv.close()


def test_device_bytes_cover_a_mixed_hierarchy():
    """The device bytes a hierarchy reports (what the server admits against)
    cover the device memory its mixed-precision build took, FP32 RAP copies
    included."""
    import torch
    from paper_1607_02489_amd import emin as E
    d = E.DeviceSystem.upload(synth.oseen2d(64))
    torch.cuda.synchronize()
    E.release_cached()
    free0 = torch.cuda.mem_get_info()[0]
    h = E.NativeHierarchy(d, E.params(iters=5, mixed=True), 4, min_dofs=200)
    torch.cuda.synchronize()
    # (the builds' temporaries went back to the process-wide chunk cache,
    # which no handle owns)
    E.release_cached()
    used = free0 - torch.cuda.mem_get_info()[0]
    rep = h.device_bytes()
    say(f"[gpu] mixed hierarchy: reported {rep / 2**20:.1f} MiB, device delta {used / 2**20:.1f} MiB")
    assert rep >= used - (8 << 20)      # (allocation granularity)
    h.close()


def test_autotuned_schedule_same_results_and_reuse():
    """Every candidate schedule of the masked product sums the same products
    in the same order, so the autotuned level equals the default one bitwise;
    a second pattern of the same shape reuses the tuned choice."""
    import torch
    from paper_1607_02489_amd import emin as E
    s = synth.oseen2d(48)
    E.autotune_reset()
    base = E.NativeHierarchy(E.DeviceSystem.upload(s), E.params(iters=5), 3)
    torch.cuda.synchronize()
    tuned = E.NativeHierarchy(E.DeviceSystem.upload(s), E.params(iters=5, autotune=True), 3)
    torch.cuda.synchronize()
    st = E.autotune_stats()
    say(f"[gpu] autotune stats {st}")
    assert st["tuned"] >= 1 and st["candidates_timed"] >= 8 * st["tuned"]
    _same(_levels(tuned), _levels(base))
    for z in tuned.sizes():
        assert (z["sched_v"] >> 4) & 3 in (1, 2) and (z["sched_p"] >> 4) & 3 in (1, 2)
    again = E.NativeHierarchy(E.DeviceSystem.upload(s), E.params(iters=5, autotune=True), 3)
    torch.cuda.synchronize()
    assert E.autotune_stats()["reused"] > st["reused"]
    assert all((z["sched_v"] >> 4) & 3 == 2 for z in again.sizes())
    _same(_levels(again), _levels(base))
    for h in (base, tuned, again):
        h.close()
    E.autotune_reset()


def test_pattern_values_flag_equals_full_setup():
    """emin_setup with EMIN_FLAG_PATTERN_VALUES right after emin_pattern reuses
    the pattern's filtered operators: P must equal a setup that forms them
    again, bit for bit; a hierarchy re-setup on the same values too."""
    import torch
    from paper_1607_02489_amd import emin as E
    s = synth.oseen2d(24)
    prm = E.params(iters=5)
    H = E.Hierarchy(s, 3, prm).build()     # first setups use the flag
    torch.cuda.synchronize()
    first = [(L.Pv.cpu().numpy().copy(), L.Pp.cpu().numpy().copy(), L.Ac.cpu().numpy().copy())
             for L in H.levels]
    assert H.prm.flags & E.EMIN_FLAG_PATTERN_VALUES == 0
    H.resetup()                            # forms the operators again
    torch.cuda.synchronize()
    for (pv, pp, ac), L in zip(first, H.levels):
        assert np.array_equal(pv, L.Pv.cpu().numpy())
        assert np.array_equal(pp, L.Pp.cpu().numpy())
        assert np.array_equal(ac, L.Ac.cpu().numpy())
    H.close()

