"""Benchmark of the HIP solve loop on one MI355X.

Default workload: uniform random 3-CNF, n = 20000 variables, m = 86000 clauses
(ratio 4.3), 64 restarts solved together, 2000 Adam steps (lr 1e-4), rounding
and unsat count every 50 steps.  One benchmark step = one complete solve of
that batch (inputs resident in HBM; loading the instance is timed apart).

Printed: one JSON line with fwd+bwd literal nonzeros per second (2 L R T per
solve), the roofline of the dominant kernel (algorithmic bytes per launch /
average launch time from HIP events), and the FP64 CPU oracle timed on a
bounded sample of the same workload on this host.  The default line also
carries the same 64 restarts solved one at a time against the batched solve
(at equal per-restart cost), the structured workload (n = 500000, m = 2.5M,
one restart) and the
serving workload (512 Poisson requests through the continuous-batching
server: instances/s, p50/p99 latency, against the plain one-at-a-time loop).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_bytes(n, m, L, R, weighted=False):
    """Algorithmic bytes per launch (index arrays once, state per restart)."""
    fwd = 4 * L + 4 * (m + 1) + R * (4 * n + 4 * m)      # literals, offsets, x gather, a write
    if weighted:
        fwd += 8 * m                                     # clause weights, once
    bwd = 4 * L + 4 * (n + 1) + R * (4 * m + 24 * n)     # occurrences, offsets, a gather, x/m/v r+w
    return fwd, bwd


def kernels_sha():
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.hpp", "plan.cpp", "plan.hpp"):
        with open(os.path.join(ROOT, "paper_2402_03640_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_record(config, schedule, kernel_key):
    """HBM bytes per launch from the committed rocprofv3 counter summary
    (profiles/traffic.json), if it was taken on the current kernel sources
    with the same schedule; None otherwise."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        rec = json.load(open(p))
    except Exception:
        return None
    if rec.get("kernels_sha") != kernels_sha():
        return None
    c = rec.get("configs", {}).get(config, {}).get(str(schedule))
    if not c:
        return None
    k = c.get("kernels", {}).get(kernel_key)
    return None if not k else round(k["hbm_bytes_per_launch"])


def counters_summary(dirs):
    """Summarise rocprofv3 counter runs of ``--kernels-only``.

    Each directory is the ``-d`` of one ``rocprofv3 --pmc <COUNTER>
    --kernel-trace -f csv -o pmc`` run, named pmc_<config>_<schedule>_<COUNTER>.
    The counter of the 256 MiB calibration copy in the same run gives the
    scale factor (bytes the copy must move / bytes the counter reports); the
    forward and backward kernels' per-dispatch averages are scaled by it.
    Writes profiles/traffic.json and prints the text summary."""
    import csv
    import glob
    copy_bytes = 256 * 2 ** 20
    runs = {}
    for d in dirs:
        base = os.path.basename(os.path.normpath(d))
        parts = base.split("_")
        if len(parts) < 4 or parts[0] != "pmc":
            continue
        counter = "_".join(parts[-2:])
        config, sched = "_".join(parts[1:-3]), parts[-3]
        files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        if not files:
            continue
        rows = list(csv.DictReader(open(files[0])))
        copies = [float(r["Counter_Value"]) for r in rows if "k_copy" in r["Kernel_Name"]]
        gathers = [float(r["Counter_Value"]) for r in rows if "k_gather" in r["Kernel_Name"]]
        per = {}
        for r in rows:
            name = r["Kernel_Name"]
            key = "fwd" if ("k_fwd<" in name or "k_fwd_nt<" in name) else ("bwd" if "k_bwd<" in name else None)
            if key:
                per.setdefault(key, [name, []])[1].append(float(r["Counter_Value"]))
        runs.setdefault((config, sched), {})[counter] = (max(copies) if copies else None, per,
                                                         max(gathers) if gathers else None)
    out = {"kernels_sha": kernels_sha(),
           "method": "rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) --kernel-trace, KiB per dispatch averaged "
                     "over launches, each scaled by (256 MiB / the counter's reading for the project's 256 MiB "
                     "streaming copy made in the same run); a cold 128-byte gather checks the FETCH factor",
           "configs": {}}
    base = os.path.dirname(os.path.normpath(dirs[0])) if dirs else "."
    lines = ["# HBM traffic per launch from rocprofv3 counters (calibrated)",
             "# commands (one run per counter, config and schedule):",
             f"#   rocprofv3 --pmc FETCH_SIZE --kernel-trace -f csv -d {base}/pmc_<cfg>_<sched>_FETCH_SIZE -o pmc "
             "-- python -u bench.py --config <cfg> --kernels-only --kernel-iters 20 --schedule <sched>",
             "#   (the same with WRITE_SIZE)",
             f"#   python bench.py --counters-summary {base}/pmc_<cfg>_<sched>_<counter> ...",
             "# columns: config, schedule, kernel, launches, FETCH KiB avg, WRITE KiB avg, FETCH factor, "
             "WRITE factor, calibrated MB per launch, algorithmic MB per launch"]
    for (config, sched), ctr in sorted(runs.items()):
        if "FETCH_SIZE" not in ctr or "WRITE_SIZE" not in ctr:
            continue
        import paper_2402_03640_amd as hm
        wl = make_workload(config)
        L = int(hm.Plan(wl["n"], wl["lits"]).nnz)  # canonical literal count (host-only plan)
        fb, bb = kernel_bytes(wl["n"], wl["m"], L, wl["R"], wl["weights"] is not None)
        fcopy, fper, fgat = ctr["FETCH_SIZE"]
        wcopy, wper, _ = ctr["WRITE_SIZE"]
        ff = copy_bytes / (fcopy * 1024) if fcopy else None
        wf = copy_bytes / (wcopy * 1024) if wcopy else None
        # second point: the cold gather fetches about 94% of its 512 MiB of
        # rows as distinct lines (16 MiB of indices on top): its scaled reading
        # should come out near 0.94 * 512 + 16 MiB
        gat = fgat * 1024 * ff / 2 ** 20 if (fgat and ff) else None
        rec = {"fetch_factor": ff, "write_factor": wf, "gather_check_mib": gat, "kernels": {}}
        if gat is not None:
            lines.append(f"# {config} {sched}: cold 128-byte gather, FETCH scaled by the copy factor: {gat:.0f} MiB "
                         f"(expected about {0.94 * 512 + 16:.0f} MiB of distinct lines)")
        for key, alg in (("fwd", fb), ("bwd", bb)):
            if key not in fper or key not in wper or ff is None or wf is None:
                continue
            name, fv = fper[key]
            wv = wper[key][1]
            fk, wk = sum(fv) / len(fv), sum(wv) / len(wv)
            hbm = (fk * ff + wk * wf) * 1024
            rec["kernels"][key] = {"name": name, "launches": len(fv), "fetch_kib": fk, "write_kib": wk,
                                   "hbm_bytes_per_launch": hbm, "algorithmic_bytes": alg}
            lines.append(f"{config} {sched} {name[:60]} {len(fv)} {fk:.1f} {wk:.1f} {ff:.3f} {wf:.3f} "
                         f"{hbm / 1e6:.2f} {alg / 1e6:.2f}")
        out["configs"].setdefault(config, {})[sched] = rec
    with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print("\n".join(lines))


# one-restart schedules compared over instance sizes: the uniform bitset
# entry, the 16-column one-row and multi-lane entries, the slot entries
SIZE_SWEEP_SCHEDULES = (37, 38, 39, 41, 42)


def size_sweep(iters):
    """Step time of the one-restart schedules (their default rows per unit)
    on uniform 3- and 5-CNF and skewed instances of growing size, best of
    three hms_time_kernels runs each."""
    import cnfgen
    import paper_2402_03640_amd as hm
    insts = [(f"3-CNF n={n} m={int(4.3 * n)}", n, cnfgen.uniform_kcnf(n, int(4.3 * n), 3, seed=n))
             for n in (2000, 5000, 20000, 60000, 200000)]
    insts += [(f"5-CNF n={n} m={17 * n}", n, cnfgen.uniform_kcnf(n, 17 * n, 5, seed=n)) for n in (4000, 30000)]
    insts += [(f"structured n={n} m={5 * n}", n, cnfgen.structured_cnf(n, 5 * n, seed=3)) for n in (100000, 500000)]
    print(f"# one-restart schedules over instance sizes: hms_time_kernels, {iters} launches, best of three\n"
          f"# command: python -u bench.py --size-sweep --kernel-iters {iters}\n"
          f"# columns: instance, nonzeros, then per table entry: step us (forward us / backward with combine us)",
          flush=True)
    for name, n, lits in insts:
        cnf = hm.load_cnf(n, lits)
        cols = []
        for sc in SIZE_SWEEP_SCHEDULES:
            best = min((hm.time_kernels(cnf, restarts=1, iters=iters, schedule=sc) for _ in range(3)),
                       key=lambda t: t[2])
            cols.append(f"{sc}: {best[2] * 1e3:6.2f} ({best[0] * 1e3:5.2f}/{best[1] * 1e3:5.2f})")
        print(f"{name:28s} {cnf.info['nnz']:9d}  " + "  ".join(cols), flush=True)
        cnf.free()


def sweep(cnf, wl, iters):
    """Time every schedule the autotuner considers (hms_time_kernels, HIP events)."""
    import paper_2402_03640_amd as hm
    R = wl["R"]
    codes = hm.tune_candidates(R, hm.LOSS_UNSAT) + [hm.RESIDENT]
    res = []
    print(f"# schedule sweep of {wl['name']} ({wl['desc']}): hms_time_kernels, {iters} launches each\n"
          f"# command: python -u bench.py --config {wl['name']} --sweep --kernel-iters {iters}\n"
          f"# columns: schedule id, table index, rows per unit, fwd us, bwd us, step us", flush=True)
    for code in codes:
        try:
            f, b, st = hm.time_kernels(cnf, restarts=R, iters=iters, lr=1e-4, schedule=code)
        except hm.HipMsatError as e:
            print(f"{code:6d} {code & 0xff:3d} {code >> 8:3d}  skipped: {e}", flush=True)
            continue
        res.append((st, code))
        print(f"{code:6d} {code & 0xff:3d} {code >> 8:3d} {f * 1e3:8.2f} {b * 1e3:8.2f} {st * 1e3:8.2f}",
              flush=True)
    res.sort()
    print("# fastest: " + ", ".join(f"{c} ({t * 1e3:.2f} us)" for t, c in res[:5]), flush=True)


def copy_bandwidth(nbytes=1 << 30, iters=20):
    """Achievable HBM bandwidth: the project's streaming-copy kernel (probe
    library) over `nbytes`, bytes read + bytes written per second, HIP events."""
    import torch

    from paper_2402_03640_amd import probe
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    ms = probe.copy_ms(src, dst, iters)
    del src, dst
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


# gather probe points: (row bytes, footprint bytes); rows of 4 B are the
# one-restart gathers, 32 B eight restarts, 128 B the 32-restart groups of the
# headline; 2 MiB sits in an XCD's L2, 22 MiB is the headline's adjoint array
# (in the 256 MB Infinity Cache), 4 GiB is beyond every cache
GATHER_POINTS = [(rb, fp) for rb in (4, 32, 128) for fp in (2 << 20, 22 << 20, 64 << 20, 4 << 30)]


def gather_bandwidth(row_bytes, footprint, iters=10, seed=0):
    """The project's gather-sum probe: random rows of `row_bytes` from a
    `footprint`-byte array, the best of its lane and rows-per-output shapes.
    Returns (gathered GB/s, total GB/s with the index and output bytes, ms
    per launch, the best shape)."""
    import torch

    from paper_2402_03640_amd import probe
    W = row_bytes // 4
    rows = footprint // row_bytes
    gathered = (512 << 20) if row_bytes >= 32 else (128 << 20)  # gathered bytes per launch
    n_idx = gathered // row_bytes
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    src = torch.ones((rows, W), dtype=torch.float32, device="cuda")
    idx = torch.randint(0, rows, (n_idx,), dtype=torch.int32, device="cuda", generator=g)
    out = torch.empty((n_idx // 8, W), dtype=torch.float32, device="cuda")
    best = None
    for vec, deg in probe.GATHER_SHAPES:
        if vec > W:
            continue
        ms = probe.gather_ms(src, idx, out, deg=deg, vec=vec, iters=iters)
        if best is None or ms < best[0]:
            best = (ms, vec, deg)
    ms, vec, deg = best
    total = gathered + n_idx * 4 + (n_idx // deg) * W * 4
    del src, idx, out
    return gathered / (ms * 1e-3) / 1e9, total / (ms * 1e-3) / 1e9, ms, f"{vec} floats per lane, {deg} rows per output"


def pattern_floors(n, m, L, R, copy_gbps):
    """Floors of the two sparse passes from the probes: each pass's gathered
    bytes (L R 4: one row of the gathered array per literal, all restarts) at
    the gather probe's rate for that array's row size and footprint, plus its
    streamed bytes at the copy rate.  Rows are 4 min(R, 32) bytes (a restart
    group of up to 32 restarts; 4 bytes at one restart)."""
    rp = 1
    while rp < R and rp < 32:
        rp *= 2
    rb = 4 * rp
    gathered = 4.0 * L * R
    out = {}
    # forward: gathers t ([n + 1][R]); streams the literal entries and writes the adjoint
    # backward: gathers the adjoint ([m][R]); streams the occurrence entries, x, m, v (read and
    # write) and writes t
    for name, foot, streamed in (("fwd", 4 * (n + 1) * R, 4 * L + 4 * (m + 1) + 4 * m * R),
                                 ("bwd", 4 * m * R, 4 * L + 4 * (n + 1) + 28 * n * R)):
        gg, _, _, shape = gather_bandwidth(rb, max(foot // rb * rb, rb * 16), iters=10)
        out[name] = {"gather_row_bytes": rb, "gather_footprint_bytes": foot, "gather_GBps": round(gg, 1),
                     "gather_shape": shape,
                     "floor_us": round((gathered / (gg * 1e9) + streamed / (copy_gbps * 1e9)) * 1e6, 3)}
    return out


def probe_table():
    """Print the copy and gather ceilings (``--probe``)."""
    print("# bandwidth probes on this GPU (libhipmsat_probe.so, HIP events)\n"
          "# command: python -u bench.py --probe\n"
          f"copy 1 GiB: {copy_bandwidth():.0f} GB/s (read + write)\n"
          "# gather-sum of random rows, best of the probe's shapes: row bytes, footprint MiB, gathered GB/s, "
          "total GB/s (+ indices and outputs), us per launch, shape", flush=True)
    for rb, fp in GATHER_POINTS:
        gg, tt, ms, shape = gather_bandwidth(rb, fp)
        print(f"gather {rb:4d} {fp >> 20:6d} {gg:8.0f} {tt:8.0f} {ms * 1e3:9.1f}  {shape}", flush=True)
    from paper_2402_03640_amd import probe
    print("# synchronisation between two passes: a grid barrier inside one cooperative launch (agent-scope\n"
          "# release/acquire on one counter) vs one more dependent launch; blocks of 256 threads, us each",
          flush=True)
    for blocks in (8, 64, 256, 512, 1024):
        us, gave = probe.grid_barrier_us(blocks)
        print(f"grid barrier {blocks:5d} blocks {us:8.2f} us" + ("  (a bounded wait gave up)" if gave else ""),
              flush=True)
    for blocks in (256, 1024):
        for graph in (False, True):
            print(f"launch gap   {blocks:5d} blocks {probe.launch_gap_us(blocks, graph=graph):8.2f} us  "
                  f"({'graph replay' if graph else 'stream launches'})", flush=True)


def make_workload(name):
    import numpy as np

    import cnfgen
    if name == "cfg2":
        n, m, R, T, K = 20000, 86000, 64, 2000, 50
        lits = cnfgen.uniform_kcnf(n, m, 3, seed=2)
        desc = ("uniform random 3-CNF n=20000 m=86000 (ratio 4.3), 64 restarts in one solve, "
                "2000 Adam steps lr 1e-4, round+count every 50")
    elif name == "cfg2-weighted":
        n, m, R, T, K = 20000, 86000, 64, 2000, 50
        lits = cnfgen.uniform_kcnf(n, m, 3, seed=2)
        desc = ("weighted MaxSAT: the uniform 3-CNF n=20000 m=86000 with clause weights U{1..100}, 64 restarts, "
                "2000 Adam steps lr 1e-4, round+count every 50")
    elif name == "cfg2-plain":
        n, m, R, T, K = 20000, 86000, 1, 2000, 50
        lits = cnfgen.uniform_kcnf(n, m, 3, seed=2)
        desc = "uniform random 3-CNF n=20000 m=86000, one restart, 2000 Adam steps, K=50"
    elif name == "cfg1":
        n, m, R, T, K = 50, 215, 1, 1000, 1
        lits = cnfgen.uniform_kcnf(n, m, 3, seed=1)
        desc = "uniform random 3-CNF n=50 m=215, one restart, 1000 Adam steps, K=1"
    elif name == "cfg3":
        n, m, R, T, K = 500000, 2500000, 1, 200, 50
        lits = cnfgen.structured_cnf(n, m, seed=3)
        desc = ("structured CNF n=500000 m=2.5M, length 2+Geometric(0.4) capped at 12, Zipf(1.1) "
                "occurrences, one restart, 200 Adam steps, K=50")
    elif name == "cfg3-r8":
        n, m, R, T, K = 500000, 2500000, 8, 200, 50
        lits = cnfgen.structured_cnf(n, m, seed=3)
        desc = ("structured CNF n=500000 m=2.5M as above with 8 restarts (state and adjoint past the 256 MB "
                "Infinity Cache), 200 Adam steps, K=50")
    elif name == "cfg4":
        n, m, R, T, K = 1000, 4200, 16, 1000, 1
        lits = cnfgen.mixed_kcnf(n, m, seed=4)
        desc = "mixed 2/3/4-CNF n=1000 m=4200, 16 restarts, 1000 Adam steps, K=1"
    else:
        raise SystemExit(f"unknown config {name}")
    weights = None
    if name.endswith("-weighted"):
        weights = np.random.default_rng(20).integers(1, 101, size=m).astype(np.int64)
    # uniform random clauses: the probes' uniform random rows model their gathers
    uniform = name.startswith("cfg2") or name in ("cfg1", "cfg4")
    return dict(name=name, n=n, m=m, R=R, T=T, K=K, lits=lits, desc=desc, weights=weights, uniform=uniform)


# the structured workload's schedule: table entry 41 (one lane per row, two
# clause tiles per forward wavefront, occurrence slots: the forward leaves each
# occurrence's adjoint where the backward reads it in entry order), 64 rows per
# unit, which the untimed rule takes for it (the sweep under profiles/sweeps)
STRUCTURED_SCHEDULE = 41 | (64 << 8)


def plain_vs_batched_record(cnf, wl, code):
    """Plain against batched restarts on the headline instance: the R
    restarts one solve each (restart r is the one-restart solve with seed r,
    under the untimed one-restart schedule) against the batched solve of all
    R, wall time with the solves' own device time beside it, and whether every
    restart reaches the same best cost at the same step either way."""
    import numpy as np
    import torch

    import paper_2402_03640_amd as hm
    R, T, K = wl["R"], wl["T"], wl["K"]
    kw = dict(steps=T, eval_every=K, lr=1e-4)
    hm.solve(cnf, restarts=1, seed=0, autotune=False, **kw)  # warm the one-restart code objects
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = [hm.solve(cnf, restarts=1, seed=r, autotune=False, **kw) for r in range(R)]
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    batched = hm.solve(cnf, restarts=R, seed=0, schedule=code, **kw)
    torch.cuda.synchronize()
    batched_s = time.perf_counter() - t0
    pb = np.array([p.best_cost for p in plain])
    ps = np.array([p.best_step for p in plain])
    equal = bool(np.array_equal(pb, batched.restart_best) and np.array_equal(ps, batched.restart_step))
    return {"restarts": R, "plain_schedule": plain[0].schedule, "batched_schedule": batched.schedule,
            "plain_s": round(plain_s, 4), "plain_device_s": round(sum(p.device_ms for p in plain) / 1e3, 4),
            "batched_s": round(batched_s, 4), "batched_device_s": round(batched.device_ms / 1e3, 4),
            "restarts_per_s_plain": round(R / plain_s, 2), "restarts_per_s_batched": round(R / batched_s, 2),
            "speedup": round(plain_s / batched_s, 2), "equal_cost": equal, "best_cost": int(batched.best_cost)}


def structured_record(kernel_iters=100, solves=3):
    """The largest workload (structured n=500000, m=2.5M, one restart, 200
    Adam steps, count every 50) timed as the headline is: µs per gradient step
    over whole solves (HIP events), and the forward and backward (with the
    heavy-row combine) kernels against the HBM roofline."""
    import numpy as np

    import paper_2402_03640_amd as hm
    wl = make_workload("cfg3")
    cnf = hm.load_cnf(wl["n"], wl["lits"])
    L = cnf.info["nnz"]
    kw = dict(steps=wl["T"], restarts=1, eval_every=wl["K"], seed=0, lr=1e-4, schedule=STRUCTURED_SCHEDULE)
    hm.solve(cnf, **kw)  # warm
    dev = [hm.solve(cnf, **kw).device_ms for _ in range(solves)]
    f, b, st = hm.time_kernels(cnf, restarts=1, iters=kernel_iters, lr=1e-4, schedule=STRUCTURED_SCHEDULE)
    fb, bb = kernel_bytes(wl["n"], wl["m"], L, 1)
    us = 1e3 * float(np.median(dev)) / wl["T"]
    cnf.free()
    return {"workload": wl["desc"], "nnz": int(L), "schedule": STRUCTURED_SCHEDULE,
            "us_per_grad_step": round(us, 3), "nnz_per_s": 2.0 * L * wl["T"] / (float(np.median(dev)) * 1e-3),
            "fwd_us": round(f * 1e3, 3), "bwd_with_combine_us": round(b * 1e3, 3),
            "fwd_frac": round(fb / (f * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
            "bwd_frac": round(bb / (b * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
            "algorithmic_bytes": {"fwd": fb, "bwd": bb}}


def cpu_baseline(wl, L, max_threads=16, sample_steps=None, min_wall=2.0):
    """The FP64 oracle on this host, on a bounded sample of the workload
    (repeated until it has run at least ``min_wall`` seconds when the whole
    workload is tiny)."""
    import oracle as O
    oracle_lib = O.build(force=False)
    del oracle_lib
    oc = O.OracleCNF(wl["n"], wl["lits"], weights=wl["weights"])
    R = wl["R"]
    threads = max(1, min(os.cpu_count() or 1, max_threads, R))  # OpenMP over restarts
    if sample_steps is None:
        # about 6e10 literal visits: 10-30 s of the oracle on 8-16 host cores
        sample_steps = min(wl["T"], max(1, int(6.0e10 / max(1, 2 * L * R))))
    reps = 0
    t0 = time.perf_counter()
    while True:
        oc.solve(steps=sample_steps, restarts=R, eval_every=wl["K"], seed=reps, lr=1e-4, threads=threads)
        reps += 1
        dt = time.perf_counter() - t0
        if dt >= min_wall:
            break
    nnz = 2.0 * L * R * sample_steps * reps
    return {"value": nnz / dt, "unit": "nnz/s", "cores": threads, "kind": "oracle",
            "sample": f"{reps} x ({R} restarts x {sample_steps} of {wl['T']} steps, eval every {wl['K']}), "
                      f"FP64, OpenMP over restarts on {threads} threads, {dt:.2f} s wall",
            "cpu_model": host_cpu_model(), "host_cpus": os.cpu_count()}


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def batch_record(groups=((16, 15000, 60000), (32, 15000, 60000), (16, 60000, 200000)), steps=1000):
    """Grouped batches (hms_solve_batch: instances of uneven size in one
    launch per kernel per step) against one hms_solve after another, on
    uniform 3-CNF one-restart instances of log-uniform size, 1000 Adam steps,
    K=50 (plans built beforehand; the batch timed twice, the faster kept);
    each batched result must equal its solo result."""
    import numpy as np
    import torch

    import cnfgen
    import paper_2402_03640_amd as hm
    out = []
    for gi, (count, n_lo, n_hi) in enumerate(groups):
        rng = np.random.default_rng(40 + gi)
        ns = [int(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))) for _ in range(count)]
        cnfs = [hm.load_cnf(n, cnfgen.uniform_kcnf(n, int(4.3 * n), 3, seed=1000 * gi + i)) for i, n in enumerate(ns)]
        kw = dict(steps=steps, restarts=1, eval_every=50, lr=1e-4)
        seeds = list(range(count))
        hm.solve_batch(cnfs[:2], seeds=seeds[:2], **kw)  # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solo = [hm.solve(c, seed=s, autotune=False, **kw) for c, s in zip(cnfs, seeds)]
        torch.cuda.synchronize()
        solo_s = time.perf_counter() - t0
        batch_s = float("inf")
        for _ in range(2):  # the first call of a group also grows the allocator's pool
            t0 = time.perf_counter()
            batch = hm.solve_batch(cnfs, seeds=seeds, **kw)
            torch.cuda.synchronize()
            batch_s = min(batch_s, time.perf_counter() - t0)
        equal = all(a.best_cost == b.best_cost and a.best_step == b.best_step
                    and np.array_equal(a.best_assignment, b.best_assignment) for a, b in zip(solo, batch))
        out.append({"instances": count, "n_range": [n_lo, n_hi], "nnz": int(sum(c.info["nnz"] for c in cnfs)),
                    "batch_schedule": batch[0].schedule, "solo_s": round(solo_s, 4), "batch_s": round(batch_s, 4),
                    "instances_per_s_solo": round(count / solo_s, 1), "instances_per_s_batch": round(count / batch_s, 1),
                    "speedup": round(solo_s / batch_s, 2), "equal": equal})
        log(f"[batch] {out[-1]}")
        for c in cnfs:
            c.free()
    return {"metric": "instances/s (grouped batches vs one solve after another)", "steps": steps,
            "workload": "uniform random 3-CNF, one restart, n log-uniform in each range, m = 4.3 n, 1000 Adam steps, "
                        "K=50", "groups": out}


def serve_bench(args):
    """Serving workload as its own bench line."""
    print(json.dumps(serve_record(args)), flush=True)


def serve_record(args):
    """Serving workload: Poisson arrivals replayed in real time into the
    continuous-batching server (at the workload's 200 req/s and again at 80
    req/s, below capacity), then the same instances one at a time in arrival
    order, with the host plan build and the solve timed apart."""
    import numpy as np
    import torch

    import cnfgen
    import paper_2402_03640_amd as hm
    from paper_2402_03640_amd.serve import Server, percentile

    reqs = cnfgen.serving_stream(args.serve_requests, seed=5)
    log(f"[serve] generating {len(reqs)} instances ...")
    data = []
    for i, r in enumerate(reqs):
        data.append(r.cnf())
        if i % 64 == 63:
            log(f"[serve] generated {i + 1}")
    L_tot = int(sum(int(np.count_nonzero(d)) for d in data))
    T = args.serve_steps
    params = [dict(steps=T, restarts=1, eval_every=50, seed=r.index, lr=1e-4, autotune=False)
              for r in reqs]
    # warm the code objects on a small instance
    c = hm.load_cnf(reqs[0].n, data[0])
    hm.solve(c, **params[0])
    c.free()
    torch.cuda.synchronize()

    def served(scale):
        """Replay the arrivals with their times multiplied by `scale`."""
        srv = Server(workers=args.serve_workers)
        t0 = time.perf_counter()
        futs = []
        for r, lits, p in zip(reqs, data, params):
            target = t0 + scale * r.arrival_s
            while True:
                now = time.perf_counter()
                if now >= target:
                    break
                time.sleep(min(target - now, 0.002))
            futs.append(srv.submit(r.n, lits, arrival=target, **p))
        res = [f.result() for f in futs]
        srv.close()
        span = max(x.done for x in res) - (t0 + scale * reqs[0].arrival_s)
        lat = [x.latency for x in res]
        return res, span, lat

    rate = len(reqs) / reqs[-1].arrival_s
    log(f"[serve] served run at {rate:.0f} req/s ...")
    res, span, lat = served(1.0)
    served_ips = len(res) / span
    log(f"[serve] served {len(res)} in {span:.3f} s, p50 {percentile(lat, 50)*1e3:.1f} ms, "
        f"p99 {percentile(lat, 99)*1e3:.1f} ms")
    low = 80.0
    log(f"[serve] served run at {low:.0f} req/s (arrival times scaled by {rate / low:.2f}) ...")
    res_lo, span_lo, lat_lo = served(rate / low)
    log(f"[serve] at {low:.0f} req/s: {len(res_lo) / span_lo:.1f} inst/s, p50 {percentile(lat_lo, 50)*1e3:.1f} ms, "
        f"p99 {percentile(lat_lo, 99)*1e3:.1f} ms")
    log("[serve] plain run (one at a time, arrival order; plan build and solve timed apart) ...")
    t1 = time.perf_counter()
    plain = []
    build_s, solve_s, threads = [], [], 1
    for r, lits, p in zip(reqs, data, params):
        a = time.perf_counter()
        c = hm.load_cnf(r.n, lits)
        b = time.perf_counter()
        threads = max(threads, c.info["plan_threads"])
        plain.append(hm.solve(c, **p))
        e = time.perf_counter()
        c.free()
        build_s.append(b - a)
        solve_s.append(e - b)
    plain_span = time.perf_counter() - t1
    plain_ips = len(plain) / plain_span
    dev_ips = len(plain) / sum(solve_s)
    same = all(int(a.best_cost) == int(b.output.best_cost) and
               np.array_equal(a.best_assignment, b.output.best_assignment) for a, b in zip(plain, res))
    same_lo = all(int(a.best_cost) == int(b.output.best_cost) and
                  np.array_equal(a.best_assignment, b.output.best_assignment) for a, b in zip(plain, res_lo))
    log(f"[serve] plain {plain_span:.3f} s ({plain_ips:.1f} inst/s): plan builds {sum(build_s):.3f} s, "
        f"solves {sum(solve_s):.3f} s ({dev_ips:.1f} inst/s without the builds); results identical: {same}, {same_lo}")
    out = {
        "metric": "instances/s (served, continuous batching)",
        "value": served_ips, "unit": "instances/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": 1e3 * span, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{len(reqs)} random k-CNF requests (k in 3..5, n log-uniform "
                               f"100..200000, m = n U(3.5,5) 2^k/8), Poisson {rate:.0f}/s, {T} Adam steps, "
                               f"eval every 50", "total_literals": L_tot,
                   "workers": args.serve_workers, "plain_plan_threads": threads},
        "latency_ms": {"p50": 1e3 * percentile(lat, 50), "p99": 1e3 * percentile(lat, 99),
                       "max": 1e3 * max(lat)},
        "below_capacity": {"offered_req_per_s": low, "instances_per_s": len(res_lo) / span_lo,
                           "latency_ms": {"p50": 1e3 * percentile(lat_lo, 50), "p99": 1e3 * percentile(lat_lo, 99),
                                          "max": 1e3 * max(lat_lo)}},
        "plain": {"instances_per_s": plain_ips, "p50_solve_ms": 1e3 * percentile(solve_s, 50),
                  "total_s": plain_span, "plan_build_s": sum(build_s), "solve_s": sum(solve_s),
                  "device_only_instances_per_s": dev_ips},
        "speedup_vs_plain": served_ips / plain_ips,
        "speedup_vs_plain_device_only": served_ips / dev_ips,
        "equal_cost": bool(same and same_lo),
        "fwd_bwd_nnz_per_s_served": 2.0 * L_tot * T / span,
    }
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed solves")
    ap.add_argument("--warmup", type=int, default=1, help="untimed solves")
    ap.add_argument("--config", default="cfg2")
    ap.add_argument("--schedule", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true",
                    help="leave out the plain-restarts record (64 one-restart solves) of the default line")
    ap.add_argument("--no-structured", action="store_true",
                    help="leave out the structured-workload record of the default line")
    ap.add_argument("--no-serving", action="store_true",
                    help="leave out the serving record (512 Poisson requests) of the default line")
    ap.add_argument("--kernel-iters", type=int, default=200)
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-steps", type=int, default=1000)
    ap.add_argument("--serve-workers", type=int, default=16)
    ap.add_argument("--sweep", action="store_true", help="time every candidate schedule and exit")
    ap.add_argument("--size-sweep", action="store_true",
                    help="time the one-restart schedules over instance sizes and exit")
    ap.add_argument("--tune-iters", type=int, default=20)
    ap.add_argument("--counters-summary", nargs="*", default=None, metavar="DIR",
                    help="summarise rocprofv3 counter runs of --kernels-only into profiles/traffic.json")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only time the forward/backward kernels (for counter runs), after a "
                         "256 MiB device copy used to calibrate the byte counters")
    ap.add_argument("--probe", action="store_true", help="print the copy and gather bandwidth ceilings and exit")
    args = ap.parse_args()
    if args.counters_summary is not None:
        counters_summary(args.counters_summary)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the solve loop is benchmarked on a single MI355X; "
              "restarts and instances shard across GPUs without communication, "
              "no multi-GPU figure is produced.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2402_03640_amd as hm

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.probe:
        probe_table()
        return
    if args.size_sweep:
        size_sweep(args.kernel_iters)
        return
    if args.config == "serve":
        serve_bench(args)
        return
    if args.config == "batch":
        print(json.dumps(batch_record()), flush=True)
        return
    wl = make_workload(args.config)
    log(f"[bench] workload {wl['name']}: {wl['desc']}")
    t0 = time.perf_counter()
    cnf = hm.load_cnf(wl["n"], wl["lits"], weights=wl["weights"])
    torch.cuda.synchronize()
    load_s = time.perf_counter() - t0
    L = cnf.info["nnz"]
    n, m, R, T, K = wl["n"], wl["m"], wl["R"], wl["T"], wl["K"]
    log(f"[bench] loaded: L={L} heavy={cnf.info['n_heavy']} in {load_s:.3f} s")

    if args.sweep:
        sweep(cnf, wl, args.kernel_iters)
        return
    code = args.schedule
    if code == 0:
        # one tuning pass (outside the timed region); the solves use its choice
        code, tms = hm.tune(cnf, restarts=R, iters=args.tune_iters, eval_every=K)
        log(f"[bench] tuned schedule {code} ({tms * 1e3:.2f} us per step)")
    kw = dict(steps=T, restarts=R, eval_every=K, seed=0, lr=1e-4, schedule=code)
    if args.kernels_only:
        from paper_2402_03640_amd import probe
        src = torch.ones(64 * 2 ** 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        probe.copy_ms(src, dst, 1)  # calibration: each launch reads 256 MiB and writes 256 MiB
        # a second point: 512 MiB of random 128-byte rows from a 4 GiB array
        # (about 94% of them distinct lines), plus 16 MiB of indices, per launch
        gather_bandwidth(128, 4 << 30, iters=1)
        torch.cuda.synchronize()
        f, b, st = hm.time_kernels(cnf, restarts=R, iters=args.kernel_iters, lr=1e-4, schedule=code)
        fb, bb = kernel_bytes(n, m, L, R, wl['weights'] is not None)
        print(json.dumps({"config": wl["name"], "schedule": code, "fwd_us": f * 1e3, "bwd_us": b * 1e3,
                          "step_us": st * 1e3, "fwd_bytes": fb, "bwd_bytes": bb,
                          "kernel_iters": args.kernel_iters,
                          "calibration_copy_bytes": 2 * 4 * src.numel()}),
              flush=True)
        return
    for i in range(args.warmup):
        r = hm.solve(cnf, **kw)
        log(f"[bench] warmup {i}: best {r.best_cost} device {r.device_ms:.2f} ms")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dev_ms = []
    best = []
    for i in range(args.steps):
        r = hm.solve(cnf, **kw)
        dev_ms.append(r.device_ms)
        best.append(r.best_cost)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"[bench] timed {args.steps} solves: {wall:.3f} s, best {best}, schedule {r.schedule}")
    ms_per_solve = 1e3 * wall / args.steps
    nnz_per_solve = 2.0 * L * R * T
    value = nnz_per_solve * args.steps / wall

    fwd_ms, bwd_ms, step_ms = hm.time_kernels(cnf, restarts=R, iters=args.kernel_iters, lr=1e-4,
                                              schedule=code)
    fb, bb = kernel_bytes(n, m, L, R, wl['weights'] is not None)
    log(f"[bench] kernels: fwd {fwd_ms*1e3:.2f} us, bwd {bwd_ms*1e3:.2f} us, step {step_ms*1e3:.2f} us")
    if fwd_ms <= 0 or bwd_ms <= 0:
        # resident schedule: the whole loop is one launch with the state in LDS;
        # per-kernel HBM bytes do not describe it
        roof = None
    else:
        if bwd_ms >= fwd_ms:
            dom, dbytes, dms, key = "backward (transposed sums + Adam)", bb, bwd_ms, "bwd"
            oname, obytes, oms = "forward", fb, fwd_ms
        else:
            dom, dbytes, dms, key = "forward (scores + mask + adjoint)", fb, fwd_ms, "fwd"
            oname, obytes, oms = "backward", bb, bwd_ms
        achieved = dbytes / (dms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4),
                "traffic": traffic_record(wl["name"], r.schedule, key),
                "kernel": dom, "algorithmic_bytes_per_launch": dbytes,
                "avg_launch_us": round(dms * 1e3, 3),
                "other_kernel": {"name": oname, "avg_launch_us": round(oms * 1e3, 3),
                                 "algorithmic_bytes_per_launch": obytes,
                                 "achieved_GBps": round(obytes / (oms * 1e-3) / 1e9, 1)}}
    step_bytes = fb + bb
    copy_gbps = copy_bandwidth()
    log(f"[bench] device copy (project kernel): {copy_gbps:.0f} GB/s (read + write)")
    floors = None
    if roof is not None:
        roof["frac_of_copy"] = round(roof["achieved"] / copy_gbps, 4)
        if wl["uniform"]:
            floors = pattern_floors(n, m, L, R, copy_gbps)
            roof["pattern_floor_us"] = floors[key]["floor_us"]
            roof["frac_of_pattern_floor"] = round(floors[key]["floor_us"] / roof["avg_launch_us"], 4)
            log(f"[bench] pattern floors: {floors}")
    out = {
        "metric": "fwd+bwd literal nnz/s",
        "value": value,
        "unit": "nnz/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_solve,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "n": n, "m": m, "nnz": L, "restarts": R,
                   "grad_steps_per_solve": T, "eval_every": K, "schedule": r.schedule},
        "roofline": roof,
        "effective_GBps_per_step": round(step_bytes / (step_ms * 1e-3) / 1e9, 1),
        "copy_GBps": round(copy_gbps, 1),
        "ceilings": {"copy_GBps": round(copy_gbps, 1), "copy_kernel": "project streaming copy (probe library)",
                     "pattern_floors": floors},
        "device_ms_per_solve": round(float(np.median(dev_ms)), 3),
        "us_per_grad_step": round(1e3 * float(np.median(dev_ms)) / max(T, 1), 3),
        "best_cost": int(min(best)),
        "load_s": round(load_s, 4),
    }
    # the sub-records report a failure in the line instead of losing it
    if args.config == "cfg2" and not args.no_plain:
        log("[bench] plain restarts: 64 one-restart solves against the batched solve ...")
        try:
            out["plain_vs_batched"] = plain_vs_batched_record(cnf, wl, code)
        except Exception as e:  # noqa: BLE001
            out["plain_vs_batched"] = {"error": f"{type(e).__name__}: {e}"}
        log(f"[bench] plain vs batched: {out['plain_vs_batched']}")
    if args.config == "cfg2" and not args.no_structured:
        log("[bench] the structured workload (n=500000, m=2.5M) ...")
        try:
            out["structured"] = structured_record()
        except Exception as e:  # noqa: BLE001
            out["structured"] = {"error": f"{type(e).__name__}: {e}"}
        log(f"[bench] structured: {out['structured']}")
    if args.config == "cfg2" and not args.no_serving:
        log("[bench] the serving workload (512 Poisson requests) ...")
        try:
            sv = serve_record(args)
            out["serving"] = {k: sv[k] for k in ("metric", "value", "unit", "latency_ms", "below_capacity", "plain",
                                                 "speedup_vs_plain", "speedup_vs_plain_device_only", "equal_cost",
                                                 "fwd_bwd_nnz_per_s_served")}
            out["serving"]["workload"] = sv["config"]["workload"]
        except Exception as e:  # noqa: BLE001
            out["serving"] = {"error": f"{type(e).__name__}: {e}"}
        log(f"[bench] serving: {out['serving']}")
    if not args.no_cpu:
        log("[bench] timing the FP64 oracle on the host ...")
        out["cpu_baseline"] = cpu_baseline(wl, L)
        log(f"[bench] oracle: {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
