"""The caller's allocator (emin_pattern_alloc): a pattern handle whose device
memory comes from torch's caching allocator gives the same level as one on
the library's own memory, holds that memory while it lives and gives every
block back when destroyed; an allocator that fails part-way makes the call
fail with EMIN_ERR_OOM after every block it did hand out has come back."""
import numpy as np
import pytest

from paper_1607_02489_amd import synth
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _level(E, d, prm, allocator=None):
    import torch
    pat = E.Pattern(d, prm, allocator=allocator)
    s = pat.sizes
    f64 = dict(dtype=torch.float64, device="cuda")
    Pv = torch.empty(max(s["nnz_Pv"], 1), **f64)
    Pp = torch.empty(max(s["nnz_Pp"], 1), **f64)
    Ac = torch.empty(max(s["nnz_Ac"], 1), **f64)
    Bc = torch.empty(max(s["nnz_Bc"], 1), **f64)
    pat.setup(prm, Pv.data_ptr(), Pp.data_ptr())
    pat.rap(Pv.data_ptr(), Pp.data_ptr(), Ac.data_ptr(), Bc.data_ptr())
    torch.cuda.synchronize()
    return pat, [t.cpu().numpy() for t in (Pv, Pp, Ac, Bc)]


def test_torch_allocator_same_level_and_memory_returned():
    import torch
    from paper_1607_02489_amd import emin as E
    s = synth.make_system(2, 40, jitter=0.1, nu=0.02, wind="stream", seed=7)
    say(f"[gpu] caller allocator, 2-D Oseen 40x40: dofs={s.dofs}")
    d = E.DeviceSystem.upload(s)
    prm = E.params(iters=5)
    ref, want = _level(E, d, prm)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    alloc = E.torch_allocator()
    pat, got = _level(E, d, prm, allocator=alloc)
    held = torch.cuda.memory_allocated() - before
    for a, b in zip(got, want):
        assert np.array_equal(a, b)
    assert held >= 64 << 20            # at least one of the handle's chunks
    pat.close()
    torch.cuda.synchronize()
    after = torch.cuda.memory_allocated()
    say(f"[gpu] torch memory held by the handle: {held / 2**20:.1f} MiB, after close "
        f"{(after - before) / 2**20:.1f} MiB")
    assert after - before < (1 << 20)   # every block given back
    ref.close()


def test_failing_allocator_reports_oom_and_gives_back():
    """A counting allocator first learns how many blocks a build of a 2-D
    Oseen 128x128 level requests (N; the build's temporaries go back when it
    returns, the rest when the handle is destroyed); a second build whose
    N-th request fails reports EMIN_ERR_OOM, and the N - 1 blocks it did get
    are all back."""
    import torch
    from paper_1607_02489_amd import emin as E
    d = E.DeviceSystem.upload(synth.oseen2d(128))
    prm = E.params(iters=5)

    def counting(fail_at):
        out, calls = {}, [0]

        def alloc(n):
            calls[0] += 1
            if calls[0] == fail_at:
                return 0
            p = torch.cuda.caching_allocator_alloc(n)
            out[p] = n
            return p

        def free(p):
            out.pop(p)
            torch.cuda.caching_allocator_delete(p)
        return E.Allocator(alloc, free), out, calls

    a, out, calls = counting(0)
    pat = E.Pattern(d, prm, allocator=a)
    nblocks = calls[0]
    assert 1 <= len(out) <= nblocks
    pat.close()
    assert not out
    b, out2, calls2 = counting(nblocks)
    with pytest.raises(E.EminError) as ei:
        E.Pattern(d, prm, allocator=b)
    say(f"[gpu] failing allocator: {nblocks} blocks per build; failure at the last: status "
        f"{ei.value.status}, outstanding {len(out2)}")
    assert ei.value.status == 9         # EMIN_ERR_OOM
    assert calls2[0] == nblocks and not out2


def test_destroy_with_queued_work_keeps_chunks_from_reuse():
    """A handle destroyed while its set-up is still queued on one stream: its
    chunks go back to the cache with that work's completion point, so a level
    built at once on a second stream takes other memory until the work has
    run.  Both results equal the level built alone."""
    import torch
    from paper_1607_02489_amd import emin as E
    s = synth.stokes3d(16)
    say(f"[gpu] destroy with queued work, 3-D Stokes 16^3: dofs={s.dofs}")
    d = E.DeviceSystem.upload(s)
    prm = E.params(iters=5)
    ref, want = _level(E, d, prm)
    ref.close()
    torch.cuda.synchronize()
    E.release_cached()
    f64 = dict(dtype=torch.float64, device="cuda")
    pat = E.Pattern(d, prm)
    z = pat.sizes
    bufs = [torch.empty(max(z[k], 1), **f64) for k in ("nnz_Pv", "nnz_Pp", "nnz_Ac", "nnz_Bc")]
    Pv, Pp, Ac, Bc = (t.data_ptr() for t in bufs)
    for _ in range(4):            # enough queued work to outlast the next build's allocations
        pat.setup(prm, Pv, Pp)
        pat.rap(Pv, Pp, Ac, Bc)
    pat.close()                   # its set-ups may still be running
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        other, got = _level(E, d, prm)
    torch.cuda.synchronize()
    first = [t.cpu().numpy() for t in bufs]
    for a, b, c in zip(first, got, want):
        assert np.array_equal(a[:len(c)], c)
        assert np.array_equal(b, c)
    other.close()
