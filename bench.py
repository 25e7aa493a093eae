#!/usr/bin/env python3
"""EMIN-AMG setup benchmark on one MI355X.

A step is one pass of the whole hot path over one synthetic Q2-Q1 system:
for every level of the hierarchy, emin_pattern (aux operators, Alg. 3,
Alg. 4, patterns, symbolic RAP), emin_setup (constrained CG) and emin_rap.
The inputs are resident in device memory before the timed region.

Metric: P-nnz * iterations per second, counting the computed entries
sum over levels of (nnz(Pv) + nnz(Pp)) times the CG iterations.
The JSON line also carries the live roofline of the masked product (HIP
events around its launches, algorithmic bytes per launch), the incremental
(numeric-only) setup rate, p50/p99 step latency, and the CPU oracle's rate on
the same workload as a reported baseline.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # 2-D Oseen (Picard), 256x256 Q2-Q1, Re=100, 4-level FP64 hierarchy, 5 steps/level
    "oseen2d_256": dict(make=lambda s: s.oseen2d(256), nlevels=4, iters=5, tau1_v=0.06,
                        tau1_p=0.06, mixed=False, min_dofs=0,
                        desc="2-D Oseen Q2-Q1 256x256, Re=100, 4-level FP64 hierarchy, 5 EMIN CG steps per level"),
    # 3-D Stokes 48^3 Q2-Q1, jitter 0.05h; drop tolerances for the 27-point 3-D
    # stencils (tau1_v = 0.038 sits in the gap of the velocity entry ratios)
    "stokes3d_48": dict(make=lambda s: s.stokes3d(48), nlevels=4, iters=5, tau1_v=0.038,
                        tau1_p=0.04, mixed=False, min_dofs=1000,
                        desc="3-D Stokes Q2-Q1 48^3, jitter 0.05h, hierarchy to <=1000 dofs, 5 EMIN CG steps per level"),
    # 2-D Stokes 8x8 (smallest; parity case)
    "stokes2d_8": dict(make=lambda s: s.stokes2d_small(), nlevels=2, iters=5, tau1_v=0.06,
                       tau1_p=0.06, mixed=False, min_dofs=0,
                       desc="2-D Stokes Q2-Q1 8x8, jitter 0.1h, one transfer, 5 EMIN CG steps"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[k]


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def oracle_child(args):
    """The CPU-baseline leg, run in a child process beside the GPU work: the
    oracle (single-threaded C, FP64) builds the whole hierarchy of the same
    workload, repeated while less than `cpu_seconds` of CPU work have been
    spent (at least once).  Writes its timing and the last hierarchy's values
    (the accuracy reference) to args.out (an .npz of plain arrays)."""
    import numpy as np
    from oracle import oracle as O
    from paper_1607_02489_amd import synth
    wl = WORKLOADS[args.workload]
    system = wl["make"](synth)
    times = []
    levels = None
    t_end = time.perf_counter() + args.cpu_seconds
    while True:
        t0 = time.perf_counter()
        levels, _ = O.hierarchy(system, wl["nlevels"], tau1_v=wl["tau1_v"], tau1_p=wl["tau1_p"],
                                iters=wl["iters"], min_dofs=wl["min_dofs"],
                                energy_ata=bool(args.energy_ata))
        times.append(time.perf_counter() - t0)
        if time.perf_counter() >= t_end:
            break
    out = {"times": np.array(times), "nlevels": np.array([len(levels)])}
    for i, L in enumerate(levels):
        Wv = (~L.dir).astype(np.float64)
        for name in ("Pv", "Pp", "Ac", "Bc"):
            m = getattr(L, name)
            out[f"L{i}_{name}_rowptr"] = m.rowptr
            out[f"L{i}_{name}_col"] = m.col
            out[f"L{i}_{name}_val"] = m.val
            out[f"L{i}_{name}_shape"] = np.array([m.nrows, m.ncols])
        out[f"L{i}_Wv"] = Wv
        out[f"L{i}_Wcv"] = Wv[np.nonzero(L.is_cv)[0]]
    np.savez(args.out, **out)


def start_oracle_child(args):
    import subprocess
    import tempfile
    fd, path = tempfile.mkstemp(suffix=".npz", prefix="emin_oracle_")
    os.close(fd)
    cmd = [sys.executable, os.path.abspath(__file__), "--oracle-child", "--workload",
           args.workload, "--out", path, "--cpu-seconds", str(args.cpu_seconds)]
    if args.energy_ata:
        cmd.append("--energy-ata")
    env = dict(os.environ, OMP_NUM_THREADS="1")
    return subprocess.Popen(cmd, env=env), path


def finish_oracle_child(proc, path, p_nnz_iters):
    """Waits for the CPU-baseline child; returns (cpu_baseline, reference levels)."""
    import numpy as np
    from paper_1607_02489_amd.synth import CSR
    rc = proc.wait()
    if rc != 0:
        log(f"[bench] CPU oracle child failed with status {rc}")
        return None, None
    z = np.load(path, allow_pickle=False)
    os.remove(path)
    times = [float(t) for t in z["times"]]
    mean = sum(times) / len(times)
    refs = []
    for i in range(int(z["nlevels"][0])):
        r = {}
        for name in ("Pv", "Pp", "Ac", "Bc"):
            nr, nc = (int(v) for v in z[f"L{i}_{name}_shape"])
            r[name] = CSR(nr, nc, z[f"L{i}_{name}_rowptr"], z[f"L{i}_{name}_col"],
                          z[f"L{i}_{name}_val"])
        r["Wv"], r["Wcv"] = z[f"L{i}_Wv"], z[f"L{i}_Wcv"]
        r["Wp"], r["Wcp"] = np.ones(r["Pp"].nrows), np.ones(r["Pp"].ncols)
        refs.append(r)
    cpu = dict(value=p_nnz_iters / mean, unit="P-nnz*iters/s", cores=1, kind="oracle",
               sample=f"{len(times)} whole hierarchy setup(s) of the same workload by the "
                      f"single-threaded C oracle, in a child process beside the GPU run "
                      f"({sum(times):.1f} s of CPU work, mean {mean * 1e3:.0f} ms)",
               ms_per_setup=mean * 1e3, host_cpus=os.cpu_count(), cpu_model=_cpu_model())
    return cpu, refs


def _rowmax(a, ref):
    """Largest per-row max |a - ref| over the row's largest |ref| (floored at
    1e-6 of the matrix's largest |ref|)."""
    import numpy as np
    b = np.asarray(ref.val, np.float64)
    rows = np.repeat(np.arange(ref.nrows), np.diff(ref.rowptr))
    err = np.zeros(ref.nrows)
    sc = np.zeros(ref.nrows)
    np.maximum.at(err, rows, np.abs(np.asarray(a, np.float64) - b))
    np.maximum.at(sc, rows, np.abs(b))
    sc = np.maximum(sc, 1e-6 * np.abs(b).max())
    sc[sc == 0] = 1.0
    return float((err / sc).max())


def _relfro(a, b):
    import numpy as np
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(np.asarray(a, np.float64) - np.asarray(b, np.float64)) /
                 (nb if nb > 0 else 1.0))


def accuracy(H, ref_levels, label):
    """Relative Frobenius errors of P and of the Galerkin blocks, level by level,
    against a reference hierarchy with the same patterns, and the constraint
    residual ||P W_c - W|| / ||W|| of every computed P (default modes)."""
    import numpy as np
    import scipy.sparse as sp
    out = []
    for L, R in zip(H.levels, ref_levels):
        s = L.pattern.sizes
        d = {}
        for name, nnz in (("Pv", "nnz_Pv"), ("Pp", "nnz_Pp"), ("Ac", "nnz_Ac"), ("Bc", "nnz_Bc")):
            g = getattr(L, name)[:s[nnz]].double().cpu().numpy()
            r = R[name]
            d[name] = _relfro(g, r.val) if len(r.val) == len(g) else float("nan")
            if len(r.val) == len(g) and len(g):
                d[name + "_rowmax"] = _rowmax(g, r)
        for blk, Pr in (("v", R["Pv"]), ("p", R["Pp"])):
            g = getattr(L, "P" + blk)[:Pr.nnz].double().cpu().numpy()
            P = sp.csr_matrix((g, Pr.col, Pr.rowptr), shape=(Pr.nrows, Pr.ncols))
            W = R["W" + blk]
            Wc = R["Wc" + blk]
            nw = float(np.linalg.norm(W))
            d["constraint_" + blk] = float(np.linalg.norm(P @ Wc - W) / (nw if nw > 0 else 1.0))
        out.append({k: (float("%.3g" % v) if v == v else None) for k, v in d.items()})
    worst = lambda keys: max((lv[k] for lv in out for k in keys if lv.get(k) is not None),
                             default=None)
    return dict(reference=label, levels=out, max_P=worst(("Pv", "Pp")),
                max_RAP=worst(("Ac", "Bc")),
                max_rowmax=worst(("Pv_rowmax", "Pp_rowmax", "Ac_rowmax", "Bc_rowmax")),
                max_constraint=worst(("constraint_v", "constraint_p")),
                levels_compared=len(out))


def oracle_reference(levels):
    """Reference values and default modes from oracle levels."""
    import numpy as np
    out = []
    for L in levels:
        Wv = (~L.dir).astype(np.float64)
        out.append(dict(Pv=L.Pv, Pp=L.Pp, Ac=L.Ac, Bc=L.Bc, Wv=Wv, Wcv=Wv[np.nonzero(L.is_cv)[0]],
                        Wp=np.ones(L.Pp.nrows), Wcp=np.ones(L.Pp.ncols)))
    return out


def gpu_reference(H, E):
    """Reference values from a GPU hierarchy (patterns and modes from its views)."""
    import numpy as np
    from paper_1607_02489_amd.synth import CSR
    out = []
    for L in H.levels:
        pat = L.pattern
        Wv = (~pat.array_host(E.VIEW_DIR, np.uint8).astype(bool)).astype(np.float64)
        cv = pat.array_host(E.VIEW_CV, np.int32)
        ref = dict(Wv=Wv, Wcv=Wv[cv])
        for name, what in (("Pv", E.VIEW_PV), ("Pp", E.VIEW_PP), ("Ac", E.VIEW_AC),
                           ("Bc", E.VIEW_BC)):
            n, nc, rp, col, val = pat.csr_host(what, getattr(L, name).data_ptr())
            ref[name] = CSR(int(n), int(nc), rp, col, val)
        ref["Wp"] = np.ones(ref["Pp"].nrows)
        ref["Wcp"] = np.ones(ref["Pp"].ncols)
        out.append(ref)
    return out


def copy_bandwidth(torch, nbytes=1 << 30, reps=5):
    """Achievable HBM rate of a streaming device copy (torch's copy kernel):
    bytes read plus bytes written per copy, median of `reps`."""
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    ts = []
    for _ in range(reps + 1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ts = sorted(ts[1:])
    ms = ts[len(ts) // 2]
    del a, b
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def load_traffic(kernel, workload, precision):
    """HBM bytes per launch measured by rocprofv3 counters (FETCH_SIZE and
    WRITE_SIZE, scaled by the same counters on a copy kernel of known size),
    as recorded in profiles/; None when the record is missing or was taken on
    another version of the kernel source."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{precision}_traffic.json")
    src = os.path.join(ROOT, "paper_1607_02489_amd", "csrc", "emin_cg.hip")
    try:
        rec = json.load(open(path))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != sha:
        return None
    return rec.get("bytes_per_launch")


def batch_systems(synth, count=64, seed=1):
    """64 2-D Oseen systems: n ~ U{16..128}, Re log-uniform in [1, 500], wind
    seeds 1000+i (the stream-function recipe of the 2-D Oseen workload)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    ns = rng.integers(16, 129, size=count)
    res = np.exp(rng.uniform(np.log(1.0), np.log(500.0), size=count))
    return [synth.make_system(2, int(n), nu=1.0 / float(re), wind="stream", seed=1000 + i)
            for i, (n, re) in enumerate(zip(ns, res))], ns, res


def run_batch(args, E, synth, torch):
    """Config 4: 64 uneven hierarchies built concurrently (one stream per
    build), then every numeric re-setup replayed as one hipGraph launch;
    compared with plain FP64 built one after another."""
    t0 = time.perf_counter()
    systems, ns, res = batch_systems(synth)
    log(f"[bench] generated 64 systems ({sum(s.dofs for s in systems)} dofs) in "
        f"{time.perf_counter() - t0:.1f}s")
    ds = [E.DeviceSystem.upload(s) for s in systems]
    iters, nlev, mind = 5, 4, 200
    # masked-product schedules autotuned per problem shape (the first build of
    # a shape times the candidates, later ones reuse the choice)
    E.autotune_reset()
    mixed = E.params(iters=iters, mixed=True, autotune=True)
    mixed_default = E.params(iters=iters, mixed=True)
    fp64 = E.params(iters=iters)
    torch.cuda.synchronize()

    def pnnz(hs):
        return sum(z["nnz_Pv"] + z["nnz_Pp"] for h in hs for z in h.sizes())

    for _ in range(args.warmup):
        for h in E.build_batch(ds, mixed, nlev, mind, max_parallel=16):
            h.close()
    build_ms, seq_ms = [], []
    for k in range(args.steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        hs = E.build_batch(ds, mixed, nlev, mind, max_parallel=16)
        torch.cuda.synchronize()
        build_ms.append((time.perf_counter() - t) * 1e3)
        if k < args.steps - 1:
            for h in hs:
                h.close()
        log(f"[bench] batch build {k + 1}/{args.steps}: {build_ms[-1]:.1f} ms")
    p_nnz_iters = pnnz(hs) * iters
    tune = E.autotune_stats()
    codes = {}
    for h in hs:
        for z in h.sizes():
            for k in ("sched_v", "sched_p"):
                name = E.sched_name(z[k] & 0x4F)
                codes[name] = codes.get(name, 0) + 1
    stream = torch.cuda.current_stream()

    def replay_ms(batch):
        ts = []
        for _ in range(max(5, args.steps)):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            batch.run()
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return sorted(ts)[len(ts) // 2]

    B = E.Batch(hs)
    rm = replay_ms(B)
    # the same batch with the default schedules, for comparison
    hd = E.build_batch(ds, mixed_default, nlev, mind, max_parallel=16)
    torch.cuda.synchronize()
    Bd = E.Batch(hd)
    rmd = replay_ms(Bd)
    Bd.close()
    for h in hd:
        h.close()
    # plain FP64, one system after another (same GPU)
    for k in range(max(1, args.steps // 2)):
        torch.cuda.synchronize()
        t = time.perf_counter()
        seq = [E.NativeHierarchy(d, fp64, nlev, mind) for d in ds]
        torch.cuda.synchronize()
        seq_ms.append((time.perf_counter() - t) * 1e3)
        seq_pnnz = pnnz(seq) * iters
        seq_inc = []
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for h in seq:
                h.resetup()
            e1.record(stream)
            torch.cuda.synchronize()
            seq_inc.append(e0.elapsed_time(e1))
        for h in seq:
            h.close()
    B.close()
    for h in hs:
        h.close()
    bm = sorted(build_ms)[len(build_ms) // 2]
    sm = sorted(seq_ms)[len(seq_ms) // 2]
    si = sorted(seq_inc)[len(seq_inc) // 2]
    return {
        "metric": "EMIN setup P-nnz*iters/s",
        "value": p_nnz_iters / (bm * 1e-3),
        "unit": "P-nnz*iters/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": bm, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "batch64_oseen2d", "systems": 64,
                   "n_range": [int(ns.min()), int(ns.max())],
                   "re_range": [float(res.min()), float(res.max())],
                   "dofs_total": int(sum(s.dofs for s in systems)), "iters": iters,
                   "max_levels": nlev, "precision": "mixed"},
        "roofline": None, "cpu_baseline": None,
        "p_nnz_iters": p_nnz_iters,
        "graph_replay": {"ms": rm, "value": p_nnz_iters / (rm * 1e-3),
                         "what": "numeric phases of all 64 hierarchies as one hipGraph launch",
                         "default_schedule_ms": rmd},
        "autotune": {"stats": tune, "schedules": codes},
        "fp64_sequential": {"build_ms": sm, "value": seq_pnnz / (sm * 1e-3),
                            "incremental_ms": si, "incremental_value": seq_pnnz / (si * 1e-3)},
    }


def serve_pool(synth, sizes, seed=0):
    """Pool of 3-D Oseen channel systems, one per mesh size m: the Laplacian
    and convection parts on one structure, so a request with its own
    Reynolds number forms nu*A_S + K on the device."""
    return {m: synth.make_split_system(3, m, seed=seed, wind="channel", domain="channel")
            for m in sizes}


def run_serve(args, E, synth, torch):
    """Config 5: Poisson arrivals of 3-D Oseen channel setup requests admitted
    by a device-memory budget; latency from arrival to a finished hierarchy."""
    import threading
    import numpy as np
    rng = np.random.default_rng(5)
    sizes = list(range(16, 41, 4))
    t0 = time.perf_counter()
    pool = serve_pool(synth, sizes)
    log(f"[bench] serve pool of {len(pool)} channel systems in {time.perf_counter() - t0:.1f}s")
    # device copies of structure + the two value arrays per pool entry
    dev = {}
    for m, sysm in pool.items():
        d = E.DeviceSystem.upload(sysm)
        dev[m] = (d, torch.from_numpy(sysm.meta["S_val"]).cuda(),
                  torch.from_numpy(sysm.meta["K_val"]).cuda())
    lam, dur = 20.0, args.serve_seconds
    arrivals = np.cumsum(rng.exponential(1.0 / lam, size=int(lam * dur * 2)))
    arrivals = arrivals[arrivals < dur]
    ms = rng.integers(16, 41, size=arrivals.size)
    res = np.exp(rng.uniform(np.log(10.0), np.log(500.0), size=arrivals.size))
    prm = E.params(0.038, 0.04, 1.5e-3, 5, mixed=True)
    srv = E.Server(budget_bytes=200 << 30, slots=args.serve_slots)
    lat, qms, done_at, tickets = [], [], [], []
    pnnz_total = [0]
    lock = threading.Lock()

    def waiter(ticket, t_arr, req_tensors):
        view, q, r = srv.wait(ticket)
        t_done = time.perf_counter() - t_start
        pn = sum(z["nnz_Pv"] + z["nnz_Pp"] for z in view.sizes()) * 5
        srv.release(ticket)
        with lock:
            lat.append((t_done - t_arr) * 1e3)
            qms.append(q)
            done_at.append(t_done)
            pnnz_total[0] += pn

    threads = []
    sub = torch.cuda.Stream()     # forms each request's values; never a device-wide sync
    t_start = time.perf_counter()
    for a, m, re in zip(arrivals, ms, res):
        now = time.perf_counter() - t_start
        if a > now:
            time.sleep(a - now)
        key = sizes[int(np.argmin([abs(m - z) for z in sizes]))]
        d, sv, kv = dev[key]
        with torch.cuda.stream(sub):
            vals = (sv * (1.0 / re) + kv).contiguous()
        sub.synchronize()
        req = E.DeviceSystem(3, d.n_v, d.n_p, (d.A[0], d.A[1], d.A[2], vals.data_ptr()), d.B,
                             d.xv, d.p2v, [d, vals])
        t = srv.submit(req, prm, 4, 1000)
        th = threading.Thread(target=waiter, args=(t, a, req))
        th.start()
        threads.append(th)
    for th in threads:
        th.join()
    wall = max(done_at) if done_at else 0.0
    srv.close()
    return {
        "metric": "EMIN setup P-nnz*iters/s", "value": pnnz_total[0] / wall if wall else 0.0,
        "unit": "P-nnz*iters/s", "n_gpus": 1, "steps": len(lat), "warmup": 0,
        "ms_per_step": float(np.mean(lat)) if lat else None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "serve_oseen3d_channel", "arrival_rate_per_s": lam,
                   "duration_s": dur, "requests": int(arrivals.size),
                   "m_range": [16, 40], "pool_sizes": sizes, "re_range": [10, 500],
                   "budget_gb": 200, "slots": args.serve_slots, "precision": "mixed"},
        "roofline": None, "cpu_baseline": None,
        "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
        "queue_p50_ms": pct(qms, 50), "queue_p99_ms": pct(qms, 99),
        "requests_per_s": len(lat) / wall if wall else 0.0,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="stokes3d_48",
                    choices=sorted(WORKLOADS) + ["batch64_oseen2d", "serve_oseen3d_channel",
                                                 "copy_probe"])
    ap.add_argument("--energy-ata", action="store_true",
                    help="velocity EMIN energy in the A^T A-norm of the filtered operator")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="CPU oracle: repeat whole hierarchies while less than this much CPU "
                         "time has been spent (at least one)")
    ap.add_argument("--oracle-child", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--out", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tiled", action="store_true",
                    help="masked product on coordinate tiles with Z rows staged in LDS")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--serve-slots", type=int, default=8)
    args = ap.parse_args()
    if args.oracle_child:
        oracle_child(args)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the setup has no multi-GPU path (its numeric "
              "phase would shard by row slabs with halo exchanges; the greedy coarsening does "
              "not shard without changing the result).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1607_02489_amd import emin as E
    from paper_1607_02489_amd import synth

    if args.workload == "copy_probe":
        # streaming copy of a 1 GiB buffer: the achievable rate, and the known
        # byte counts that scale the HBM counters
        torch.cuda.init()
        gbs = copy_bandwidth(torch)
        print(json.dumps({"workload": "copy_probe", "bytes_read_per_copy": 1 << 30,
                          "bytes_written_per_copy": 1 << 30, "copies": 6, "copy_gbs": gbs}),
              flush=True)
        return
    if args.workload == "batch64_oseen2d":
        torch.cuda.init()
        print(json.dumps(run_batch(args, E, synth, torch)), flush=True)
        return
    if args.workload == "serve_oseen3d_channel":
        torch.cuda.init()
        print(json.dumps(run_serve(args, E, synth, torch)), flush=True)
        return
    print(json.dumps(run_standard(args, E, synth, torch)), flush=True)


def timed_builds(H, steps, warmup, torch, label, profile=False):
    """warmup untimed builds, then `steps` timed whole-hierarchy builds; with
    profile, the masked product's launches are timed (HIP events recorded by
    each launch) inside the timed region and returned one by one."""
    from paper_1607_02489_amd import emin as E
    for w in range(warmup):
        H.build()
        torch.cuda.synchronize()
        H.close()
        log(f"[bench] {label} warmup {w + 1}/{warmup} done")
    if profile:
        E.profile_enable(True, kinds=["spmm"])
        E.profile_launches()
    lat = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(steps):
        ts = time.perf_counter()
        H.build()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
        if k < steps - 1:
            H.close()
        log(f"[bench] {label} step {k + 1}/{steps}: {lat[-1] * 1e3:.1f} ms")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    launches = E.profile_launches() if profile else []
    E.profile_enable(False)
    return elapsed, lat, launches


def spmm_roofline(launches, elapsed_ms):
    """Roofline of the masked product from per-launch records: the launches
    with the largest algorithmic byte count are the level-0 velocity block's
    (its energy operator and pattern are the largest of the hierarchy); their
    average duration gives the achieved rate.  All launches are summarised
    beside it."""
    sp = [r for r in launches if r["kind"] == "spmm"]
    if not sp:
        return None
    top = max(r["bytes"] for r in sp)
    big = [r for r in sp if r["bytes"] == top]
    avg_ms = sum(r["ms"] for r in big) / len(big)
    achieved = top / (avg_ms * 1e-3) / 1e9
    all_ms = sum(r["ms"] for r in sp)
    all_bytes = sum(r["bytes"] for r in sp)
    return dict(kernel="k_spmm (masked product M*Z on the pattern of P), level-0 velocity block",
                bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=None, launches=len(big),
                avg_us=round(avg_ms * 1e3, 2), algorithmic_bytes_per_launch=round(top),
                all_levels={"launches": len(sp), "avg_us": round(all_ms / len(sp) * 1e3, 2),
                            "achieved": round(all_bytes / (all_ms * 1e-3) / 1e9, 1),
                            "share_of_step": round(all_ms / elapsed_ms, 4)})


def same_input_mixed(H, prm_mixed, torch):
    """Each level of the FP64 hierarchy set up again in mixed precision on
    its own (FP64) input: relative Frobenius errors of P and RAP per level."""
    out = []
    f64 = dict(dtype=torch.float64, device="cuda")
    for L in H.levels:
        z = L.pattern.sizes
        Pv = torch.empty(max(z["nnz_Pv"], 1), **f64)
        Pp = torch.empty(max(z["nnz_Pp"], 1), **f64)
        Ac = torch.empty(max(z["nnz_Ac"], 1), **f64)
        Bc = torch.empty(max(z["nnz_Bc"], 1), **f64)
        L.pattern.setup(prm_mixed, Pv.data_ptr(), Pp.data_ptr())
        L.pattern.rap(Pv.data_ptr(), Pp.data_ptr(), Ac.data_ptr(), Bc.data_ptr(), mixed=True)
        torch.cuda.synchronize()
        d = {}
        for name, t, nnz in (("Pv", Pv, "nnz_Pv"), ("Pp", Pp, "nnz_Pp"), ("Ac", Ac, "nnz_Ac"),
                             ("Bc", Bc, "nnz_Bc")):
            a = t[:z[nnz]].cpu().numpy()
            b = getattr(L, name)[:z[nnz]].cpu().numpy()
            d[name] = float("%.3g" % _relfro(a, b))
        out.append(d)
    return dict(levels=out, max=max(v for d in out for v in d.values()))


def run_standard(args, E, synth, torch):
    """One hierarchy workload: the FP64 build timed (the headline), the
    mixed-precision form beside it, the CPU oracle in a child process, and the
    accuracy of both against the oracle and against each other."""
    wl = WORKLOADS[args.workload]
    ata = bool(args.energy_ata)
    child = None
    if not args.no_cpu_baseline:
        child, child_out = start_oracle_child(args)
        log(f"[bench] CPU oracle baseline started in a child process (pid {child.pid})")
    t0 = time.perf_counter()
    system = wl["make"](synth)
    log(f"[bench] generated {args.workload}: dofs={system.dofs} in {time.perf_counter() - t0:.1f}s")
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    prm64 = E.params(wl["tau1_v"], wl["tau1_p"], 1.5e-3, wl["iters"], mixed=False, energy_ata=ata,
                     staged=args.tiled)
    prmx = E.params(wl["tau1_v"], wl["tau1_p"], 1.5e-3, wl["iters"], mixed=True, energy_ata=ata,
                    staged=args.tiled)
    H64 = E.Hierarchy(system, wl["nlevels"], prm64, min_dofs=wl["min_dofs"])
    torch.cuda.synchronize()
    prof = not args.no_profile
    elapsed, lat, launches = timed_builds(H64, args.steps, args.warmup, torch, "fp64",
                                          profile=prof)
    ms_per_step = elapsed / args.steps * 1e3
    levels = [L.pattern.sizes for L in H64.levels]
    p_nnz_iters = H64.p_nnz() * wl["iters"]
    p_nnz_expanded = sum(system.dim * z["nnz_Pv"] + z["nnz_Pp"] for z in levels) * wl["iters"]
    value = p_nnz_iters / (elapsed / args.steps)
    roof = spmm_roofline(launches, elapsed * 1e3) if prof else None

    phases = {}
    if prof:
        H64.close()
        E.profile_enable(True)
        E.profile_collect()
        H64.build()
        torch.cuda.synchronize()
        phases = E.profile_collect()
        E.profile_enable(False)

    def resetup_ms(H, prm, reps):
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            H.resetup(prm=prm)
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        for L in H.levels:
            E.sync_report(L.report)
        return sorted(ts)[len(ts) // 2]

    # the mixed-precision form: numeric re-setups (a new Picard
    # linearisation) on the patterns and drop masks of the FP64 pass, FP32
    # masked products and RAP, FP64 projection and CG scalars; timed beside
    # the FP64 re-setup of the same hierarchy, its whole chain compared with
    # the FP64 values
    reps = max(3, args.steps)
    inc64 = resetup_ms(H64, prm64, reps)
    ref64 = gpu_reference(H64, E)
    incx = resetup_ms(H64, prmx, reps)
    chained = accuracy(H64, ref64, "GPU FP64 hierarchy (matches the oracle to 1e-10); the mixed "
                                   "re-setup runs on its patterns, level l+1 on the mixed "
                                   "level l's coarse operator (chained)")
    resetup_ms(H64, prm64, 1)      # FP64 values again
    same_in = same_input_mixed(H64, prmx, torch)
    resetup_ms(H64, prm64, 1)

    # a fresh mixed build: its coarse levels' drop decisions are taken on
    # FP32-accumulated coarse operators, so an entry within ~1e-7 of the drop
    # threshold can flip; the flips are counted against the FP64 build
    Hx = E.Hierarchy(system, wl["nlevels"], prmx, min_dofs=wl["min_dofs"])
    nx = max(1, min(args.steps, 3))
    x_el, _, _ = timed_builds(Hx, nx, 1, torch, "mixed build")
    x_ms = x_el / nx * 1e3
    flips = []
    for La, Lb in zip(Hx.levels, H64.levels):
        f = {}
        for nm, what in (("keep_v", E.VIEW_KEEPV), ("keep_p", E.VIEW_KEEPP)):
            a = La.pattern.array_host(what, "u1")
            b = Lb.pattern.array_host(what, "u1")
            f[nm] = int((a != b).sum()) if a.size == b.size else None
        flips.append(f)
    fresh = dict(ms_per_step=x_ms, value=Hx.p_nnz() * wl["iters"] / (x_ms * 1e-3),
                 drop_decisions_differing_from_fp64=flips,
                 accuracy=accuracy(Hx, ref64, "GPU FP64 hierarchy; every level of the fresh "
                                              "mixed build on its own patterns"))
    Hx.close()
    mixed_obj = dict(
        what="numeric re-setup of every level (emin_setup + emin_rap) on the FP64 pass's "
             "patterns: FP32 masked products and RAP with FP32 accumulation, FP64 projection "
             "and CG scalars",
        resetup_ms=incx, fp64_resetup_ms=inc64, speedup_over_fp64_resetup=inc64 / incx,
        value=p_nnz_iters / (incx * 1e-3),
        accuracy=dict(chained=chained, same_input=same_in),
        fresh_mixed_build=fresh)

    copy_gbs = copy_bandwidth(torch)
    if roof is not None:
        roof["copy_gbs"] = round(copy_gbs, 1)
        roof["frac_of_copy"] = round(roof["achieved"] / copy_gbs, 4)
        roof["traffic"] = load_traffic("k_spmm", args.workload, "fp64" + ("_ata" if ata else ""))
        if roof["traffic"] is None:
            roof["traffic_note"] = ("no counter record in profiles/ for this workload and the "
                                    "current source of the masked product")

    cpu = None
    acc = None
    if child is not None:
        log("[bench] waiting for the CPU oracle child")
        cpu, refs = finish_oracle_child(child, child_out, p_nnz_iters)
        if refs is not None:
            acc = accuracy(H64, refs, "FP64 oracle (chained hierarchy, levels with equal "
                                      "patterns)")
    breakdown = {k: dict(launches=v["launches"], ms=round(v["ms"], 3))
                 for k, v in phases.items()}
    # the other kernel classes with an algorithmic byte count, over one build:
    # the numeric sparse products (B B^T and the Galerkin products, 12 bytes
    # per entry of A, B and C plus the row pointers) and the CG update (44
    # bytes per pattern entry and 20 per row)
    other_roofs = []
    for kind, kernel, bound in (
            ("spgemm", "k_spgemm_num (numeric B B^T and RAP products), every launch of a build",
             "latency (LDS accumulation of gathered B rows)"),
            ("update", "k_update (projection and CG update), every launch of a build", "hbm")):
        v = phases.get(kind)
        if v and v["ms"] > 0 and v.get("bytes", 0) > 0:
            ach = v["bytes"] / (v["ms"] * 1e-3) / 1e9
            other_roofs.append(dict(kernel=kernel, bound=bound, achieved=round(ach, 1),
                                    peak=HBM_PEAK_GBS, unit="GB/s",
                                    frac=round(ach / HBM_PEAK_GBS, 4),
                                    algorithmic_bytes=round(v["bytes"]),
                                    ms_per_build=round(v["ms"], 3), launches=v["launches"]))
    H64.close()
    return {
        "metric": "EMIN setup P-nnz*iters/s",
        "value": value,
        "unit": "P-nnz*iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": wl["desc"], "dofs": system.dofs,
                   "levels": len(levels) + 1, "iters": wl["iters"], "tau1_v": wl["tau1_v"],
                   "tau1_p": wl["tau1_p"], "tau2_sq": 1.5e-3, "precision": "fp64",
                   "energy_v": "A^T A" if ata else "(A + A^T)/2"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "accuracy": acc,
        "fp64_plain": dict(ms_per_step=ms_per_step, value=value, resetup_ms=inc64),
        "mixed": mixed_obj,
        "p50_ms": pct(lat, 50) * 1e3,
        "p99_ms": pct(lat, 99) * 1e3,
        "p_nnz_iters": p_nnz_iters,
        "p_nnz_iters_expanded_dxPv": p_nnz_expanded,
        "incremental_setup": {"ms": inc64, "value": p_nnz_iters / (inc64 * 1e-3),
                              "what": "FP64 emin_setup + emin_rap on all levels, patterns "
                                      "reused"},
        "kernel_ms_one_build": breakdown,
        "rooflines_other": other_roofs,
        "level_sizes": [{k: z[k] for k in ("n_v", "n_p", "n_vc", "n_pc", "nnz_Pv", "nnz_Pp",
                                             "nnz_Mv", "nnz_Mp", "nnz_Ac", "nnz_Bc")}
                        for z in levels],
    }


if __name__ == "__main__":
    main()
