"""Benchmark: point-edge tests per second of the grid-filtered PIP + P2P refinement.

One step is one query batch through the whole per-batch path (cell hash, stable sort,
gather/rebase, work items, refinement, FP64 recheck, output) for BOTH operations:
  PIP  configuration 3: 50M points against 5,000 Voronoi polygons (holes, up to
       50,000 vertices), grid 512 x 512 of 1/512 cells (the fastest of the cell-size sweep);
  P2P  configuration 4: 200M points against 200,000 random-walk polylines, D = 100 m,
       grid 400 x 400 of 100 m cells;
in the mixed-precision form.  The grids (MBBs, rasterised candidate lists) are built
once per geometry set and stay resident, as in a serving deployment; their build time
is reported separately.  Inputs are resident in HBM before the timed region starts.

Printed: ONE JSON line (rank 0).  Runs on one GPU; --gpus above 1 exits.
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "point-edge tests/sec (PIP, P2P) vs FP32-ALU roofline; serving p50/p99 latency"
FP32_PEAK = 157.3e12  # MI355X vector FP32, TFLOP/s (published)
FP64_PEAK = 78.6e12   # MI355X vector FP64
F_PIP = 6             # algorithmic FLOP per PIP point-edge test
F_P2P = 14            # algorithmic FLOP per P2P point-segment test
KERNEL_SRC = os.path.join(ROOT, "paper_1403_0802_amd", "csrc", "gp_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def load_traffic(kernel: str, workload: str):
    """HBM bytes per launch from rocprofv3 FETCH_SIZE/WRITE_SIZE runs, if they were taken
    on the current kernel source (else None)."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    e = t.get(kernel)
    if not e or e.get("kernel_source_sha") != kernel_hash() or e.get("workload") != workload:
        return None
    return e.get("hbm_bytes_per_launch")


COPY_PROBE_BYTES = 1 << 30


def _pmc_rows(path):
    import csv
    return list(csv.DictReader(open(path)))


def write_traffic(fetch_csv: str, write_csv: str):
    """HBM bytes per launch of the refinement kernels from rocprofv3 --pmc counter files
    (FETCH_SIZE and WRITE_SIZE, KiB per dispatch), each scaled by what the same counter
    reads for the plain 1 GiB copy of --copy-probe."""
    out = {}
    per = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = [r for r in _pmc_rows(path) if r.get("Counter_Name") == counter]
        # the probe is the largest copy dispatch (it reads and writes 1 GiB)
        copy = [float(r["Counter_Value"]) for r in rows if "copybuffer" in r["Kernel_Name"].lower()]
        copy = [c for c in copy if c > 0.25 * COPY_PROBE_BYTES / 1024]
        factor = (max(copy) * 1024.0 / COPY_PROBE_BYTES) if copy else None
        per[counter] = {"copy_factor": factor}
        for r in rows:
            name = r["Kernel_Name"]
            for k in ("k_p2pmix_pre", "k_p2pmix", "k_pipmix_pre", "k_pipmix", "k_p2p64", "k_pip64"):
                if f"gp::{k}<" in name:
                    per[counter].setdefault(k, []).append(float(r["Counter_Value"]))
    for k in ("k_p2pmix_pre", "k_p2pmix", "k_pipmix_pre", "k_pipmix", "k_p2p64", "k_pip64"):
        f = per["FETCH_SIZE"].get(k)
        w = per["WRITE_SIZE"].get(k)
        ff, wf = per["FETCH_SIZE"]["copy_factor"], per["WRITE_SIZE"]["copy_factor"]
        if not f or not w or not ff or not wf:
            continue
        fb = float(np.median(f)) * 1024.0 / ff
        wb = float(np.median(w)) * 1024.0 / wf
        out[k] = {"kernel_source_sha": kernel_hash(),
                  "workload": WORKLOAD_NAME,
                  "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
                  "hbm_bytes_per_launch": fb + wb,
                  "copy_factor_fetch": ff, "copy_factor_write": wf,
                  "launches": len(f)}
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    json.dump(out, open(TRAFFIC_FILE, "w"), indent=1, sort_keys=True)
    print(json.dumps(out, indent=1))


WORKLOAD_NAME = "C3 PIP 50M pts x 5000 polygons + C4 P2P 200M pts x 200000 polylines, mixed"
# The grids of the step (the full-size parity tests build the same ones).  PIP: 1/512, the
# fastest PIP query of the cell-size sweep (bench.py --cell-sweep), with build-time
# per-(cell, polygon) edge records (prestage).  P2P: 100 m cells with
# build-time segment records (prestage), an index structure like the candidate lists;
# detail.p2p_plain_grid runs the grid without them.
PIP_GRID = dict(cell_size=1 / 512, nx=512, ny=512, prestage=1)
P2P_GRID = dict(cell_size=100.0, radius_D=100.0, nx=400, ny=400, prestage=1)
# the server's P2P grid: the same extent in 200 m cells
SERVE_P2P_GRID = dict(cell_size=200.0, nx=200, ny=200)


def build_workloads(scale: float):
    from paper_1403_0802_amd import synth
    t0 = time.time()
    geom3, info3 = synth.config3_geometry()
    p3 = synth.GridParams(**PIP_GRID)
    n3 = int(50_000_000 * scale)
    px3, py3 = synth.config3_points(n3)
    geom4 = synth.config4_geometry()
    p4 = synth.GridParams(**P2P_GRID)
    n4 = int(200_000_000 * scale)
    px4, py4 = synth.config4_points(n4)
    log(f"[bench] inputs generated in {time.time() - t0:.1f}s: C3 {n3} pts / "
        f"{geom3.n_vertices} verts, C4 {n4} pts / {geom4.n_vertices} verts")
    return (geom3, p3, px3, py3), (geom4, p4, px4, py4)


def cpu_baseline(c3, c4, budget_s: float, step_tests):
    """The CPU oracle as it stands (grid-filtered, FP64, OpenMP over points) on a seeded
    random sample of each workload's points, with 1 thread (the paper's single-core
    "SC" setting) and with every host thread ("MC"), median of 3 runs each.  Sample sizes
    are set from a short calibration run so the twelve runs take about budget_s.  The
    rate of each setting is that of the step's own mix: step_tests = (PIP tests, P2P
    tests) of one step, done at the sampled PIP and P2P rates."""
    import oracle
    lib = oracle.load()
    threads = len(os.sched_getaffinity(0))
    geom3, p3, px3, py3 = c3
    geom4, p4, px4, py4 = c4
    g3 = oracle.build_grid(geom3, p3, lib)
    g4 = oracle.build_grid(geom4, p4, lib)
    rng = np.random.default_rng(14030805)
    per_run = budget_s / 12.0
    out = {}
    for name, geom, g, px, py in (("pip", geom3, g3, px3, py3), ("p2p", geom4, g4, px4, py4)):
        # a seeded random sample (not a prefix), large enough for any run below
        order = rng.choice(len(px), min(len(px), 8_000_000), replace=False)

        def run(m, nthreads):
            sx, sy = px[order[:m]], py[order[:m]]
            t0 = time.perf_counter()
            if name == "pip":
                oracle.pip(geom, sx, sy, g, nthreads, lib)
            else:
                oracle.p2p(geom, sx, sy, p4.radius_D, g, nthreads, lib)
            return time.perf_counter() - t0

        row = {}
        for mode, nthreads in (("sc", 1), ("mc", threads)):
            m = 4_000 if nthreads == 1 else 40_000
            dt = run(m, nthreads)  # calibration
            m = int(min(len(order), max(m, m * per_run / max(dt, 1e-4))))
            times = sorted(run(m, nthreads) for _ in range(3))
            tests = oracle.test_count(g, px[order[:m]], py[order[:m]], lib)
            row[mode] = {"points": m, "tests": tests, "threads": nthreads,
                         "seconds_median": times[1], "tests_per_s": tests / times[1],
                         "points_per_s": m / times[1]}
            log(f"[bench] oracle {name} {mode}: {m} points, {tests / times[1]:.3g} tests/s")
        out[name] = row
    tp, tq = step_tests

    def mix_rate(mode):  # tests/s of one step's mix of PIP and P2P tests
        return (tp + tq) / (tp / out["pip"][mode]["tests_per_s"] + tq / out["p2p"][mode]["tests_per_s"])

    return {
        "value": mix_rate("mc"),
        "unit": "tests/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"seeded random samples of the step's points: {out['pip']['mc']['points']} "
                   f"C3 points (PIP) and {out['p2p']['mc']['points']} C4 points (P2P) on all "
                   f"{threads} host threads (value), {out['pip']['sc']['points']} and "
                   f"{out['p2p']['sc']['points']} on 1 thread (sc); FP64 oracle with its own "
                   f"grid (same cells), OpenMP over points, median of 3 runs each; rates "
                   f"weighted by one step's PIP and P2P test counts"),
        "sc_value": mix_rate("sc"),
        "step_seconds_mc": tp / out["pip"]["mc"]["tests_per_s"] + tq / out["p2p"]["mc"]["tests_per_s"],
        "modes": out,
    }


def cpu_simd_run(c3, c4, budget_s: float):
    """The host implementation in the paper's four CPU modes (single core / all cores,
    scalar / AVX-512), on prefixes of the same point sets sized for about budget_s/8 of
    refinement each; rates are tests per second of refinement."""
    from paper_1403_0802_amd import cpu
    threads = len(os.sched_getaffinity(0))
    out = {"simd_available": cpu.gp_cpu_has_simd(), "threads": threads, "modes": {}}
    per = budget_s / 8
    for mode in ("sc", "mc", "sc_simd", "mc_simd"):
        row = {}
        for name, (geom, p, px, py), m0 in (("pip", c3, 20_000), ("p2p", c4, 20_000)):
            _, _, st = cpu.gp_cpu_join(name, geom, p, px[:m0], py[:m0], mode, threads)
            rate = st["tests"] / max(st["ms_refine"] / 1e3, 1e-6)
            per_pt = max(st["tests"] / m0, 1.0)
            m = int(min(len(px), max(m0, per * rate / per_pt)))
            _, _, st = cpu.gp_cpu_join(name, geom, p, px[:m], py[:m], mode, threads)
            row[name] = {"points": m, "tests": st["tests"], "ms_refine": st["ms_refine"],
                         "tests_per_s": st["tests"] / max(st["ms_refine"] / 1e3, 1e-9),
                         "simd": st["simd"], "threads": st["threads"]}
        out["modes"][mode] = row
        log(f"[bench] cpu {mode}: pip {row['pip']['tests_per_s']:.3g} tests/s, "
            f"p2p {row['p2p']['tests_per_s']:.3g} tests/s")
    return out


def autotune_small_run(gp, torch):
    """The autotuner on the two small configurations (PIP C1, 50K points; P2P C2, 1M
    points), whose points per cell are far from the full-size workloads the library
    defaults come from: the query time with the default and with the tuned configuration
    (median of 7 after one untimed query), and the winner."""
    from paper_1403_0802_amd import synth
    dev = torch.device("cuda")
    rows = {}
    for w in (synth.config1(), synth.config2()):
        grid = gp.gp_build_grid(w.kind, w.geom, w.params)
        x = torch.from_numpy(np.ascontiguousarray(w.px)).to(dev)
        y = torch.from_numpy(np.ascontiguousarray(w.py)).to(dev)
        oid = torch.empty(x.numel(), dtype=torch.int32, device=dev)
        od = torch.empty(x.numel(), dtype=torch.float64, device=dev)
        ws = gp.new_workspace(grid, x.numel(), "mixed")

        def query(st):
            if w.kind == "pip":
                return gp.gp_pip(grid, x, y, oid, "mixed", ws, None, st)
            return gp.gp_p2p(grid, x, y, oid, od, "mixed", ws, None, st)

        def timed():
            query(False)
            return float(np.median([query(True)["ms_total"] for _ in range(7)]))

        gp.gp_reset_tuning(grid, "mixed")
        t_default = timed()
        tuning, _ = gp.gp_autotune(grid, "mixed", x, y, ws)
        t_tuned = timed()
        rows[w.name] = {"points": x.numel(), "default_ms": t_default, "tuned_ms": t_tuned,
                        "tuning": tuning}
        log(f"[bench] autotune {w.name}: default {t_default:.3f} ms, tuned {t_tuned:.3f} ms")
        del grid, ws
    return rows


def serving_run(gp, torch, grid3, grid4, pools, n_requests: int, n_warmup: int, precision: str,
                n_slots=4, slot_points=1 << 22, mem_budget=24 << 30):
    """Configuration 5: a Poisson stream of mixed PIP/P2P requests (log-uniform 1K-4M
    points, kinds 50/50) against the resident grids.  Each request's payload is its own
    seeded random draw from the configuration's resident point set (pools: the 50M C3
    and 200M C4 points the C3/C4 generators drew), so no two requests share a payload
    and none repeats a warm-up request.  The warm-up requests run back to back (they
    capture the graphs) and give the sustained rate; the timed requests then arrive as
    a Poisson stream at 70% of it.  Latency is submit -> results visible, measured inside
    the server.  A sample of the timed requests is rerun through the direct entry points
    and must give the same bits."""
    from paper_1403_0802_amd import synth
    dev = torch.device("cuda")
    stream = synth.serving_stream(n_warmup + n_requests, rate_per_s=1.0)
    gen = torch.Generator(device=dev)
    gen.manual_seed(14030805)

    def payload(kind, n):
        x, y = pools[kind]
        idx = torch.randint(0, x.numel(), (n,), device=dev, generator=gen)
        return x[idx], y[idx]

    data, outs = [], []
    for (_, kind, n, _) in stream:
        x, y = payload(kind, n)
        data.append((kind, x, y))
        oid = torch.empty(n, dtype=torch.int32, device=dev)
        od = torch.empty(n, dtype=torch.float64, device=dev) if kind == "p2p" else None
        outs.append((oid, od))
    torch.cuda.synchronize()
    warm, timed = list(zip(data, outs))[:n_warmup], list(zip(data, outs))[n_warmup:]
    srv = gp.Server(grid3, grid4, n_slots=n_slots, slot_points=slot_points,
                    mem_budget=mem_budget, precision=precision, inputs_on_device=True,
                    use_graphs=True)
    t0 = time.perf_counter()
    for t in [srv.submit(k, x, y, o[0], o[1]) for (k, x, y), o in warm]:
        srv.wait(t)
    warm_s = time.perf_counter() - t0
    rate_pts = sum(x.numel() for (_, x, _), _ in warm) / warm_s
    mean_pts = float(np.mean([x.numel() for (_, x, _), _ in timed]))
    lam = 0.7 * rate_pts / mean_pts
    log(f"[bench] serving warm-up: {n_warmup} requests in {warm_s:.2f}s, sustained "
        f"{rate_pts:.3g} points/s; offering {lam:.1f} requests/s")
    srv.reset_stats()
    arrivals = np.cumsum(np.random.default_rng(5).exponential(1.0 / lam, len(timed)))
    t_start = time.perf_counter()
    tickets = []
    for ((k, x, y), o), ta in zip(timed, arrivals):
        now = time.perf_counter() - t_start
        if ta > now:
            time.sleep(ta - now)
        tickets.append(srv.submit(k, x, y, o[0], o[1]))
    for t in tickets:
        srv.wait(t)
    wall = time.perf_counter() - t_start
    st = srv.stats()
    srv.close()
    # a sample of the timed requests, rerun alone through the direct entry points
    rng = np.random.default_rng(7)
    same = True
    sample = rng.choice(len(timed), min(24, len(timed)), replace=False)
    for i in sample:
        (k, x, y), (oid, od) = timed[i]
        r = gp.run(grid3 if k == "pip" else grid4, x, y, precision)
        if k == "pip":
            same &= bool(torch.equal(r, oid))
        else:
            same &= bool(torch.equal(r[0], oid) and torch.equal(r[1], od))
    del data, outs, warm, timed
    torch.cuda.empty_cache()
    return {"requests": len(tickets), "warmup_requests": n_warmup,
            "offered_req_per_s": lam, "sustained_pts_per_s": rate_pts,
            "wall_s": wall, "p50_us": st["p50_us"], "p99_us": st["p99_us"],
            "mean_us": st["mean_us"], "max_us": st["max_us"],
            "latency_samples": st["latency_samples"], "completed": st["completed"],
            "failed": st["failed"], "points_per_s": st["points_per_s"],
            "tests_per_s": st["tests_per_s"], "graph_replays": st["graph_replays"],
            "max_in_flight_requests": st["max_in_flight"],
            "max_in_flight_chunks": st["max_chunks_in_flight"],
            "deferred_for_memory": st["deferred_for_memory"],
            "peak_bytes_in_use": st["peak_bytes_in_use"], "arena_bytes": st["arena_bytes"],
            "slots": n_slots, "slot_points": slot_points,
            "sample_equal_to_direct_calls": {"requests": len(sample), "equal": same},
            "payloads": "per request, a seeded random draw (torch.randint on the device) "
                        "from the resident C3 / C4 point sets"}


def cell_sweep(gp, torch, dev, c3, c4, which="both"):
    """The filter-versus-refine trade-off (Sec. III.A): query time, candidate pairs, tests
    and grid memory at five cell sizes around each configuration's default, on the full
    point sets, mixed form, default kernel tuning; `which` is "pip", "p2p" or "both"."""
    out = {}
    for name, kind, (geom, p, px, py), sizes in (
            ("pip_c3", "pip", c3, [1 / 128, 1 / 256, 1 / 512, 1 / 1024, 1 / 2048]),
            ("p2p_c4", "p2p", c4, [25.0, 50.0, 100.0, 200.0, 400.0])):
        if which not in ("both", kind):
            continue
        if kind == "p2p":
            # the sweep is over the filter; build-time segment records (20 B per cell and
            # candidate segment: about 100 GB at 25 m cells) stay out of it
            p = dataclasses.replace(p, prestage=0)
        x, y = torch.from_numpy(px).to(dev), torch.from_numpy(py).to(dev)
        t0 = time.perf_counter()
        best, rows = gp.gp_sweep_cell_size(kind, geom, p, sizes, x, y, "mixed")
        log(f"[bench] {name} sweep {time.perf_counter() - t0:.1f}s best {best}")
        out[name] = {"default_cell_size": p.cell_size, "best_cell_size": best, "rows": rows}
        del x, y
        torch.cuda.empty_cache()
    print(json.dumps({"cell_sweep": out, "workload": WORKLOAD_NAME}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=float, default=1.0, help="fraction of the point counts")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="timed requests of the serving run (after the warm-up ones)")
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--filters", action="store_true",
                    help="also measure the P2P segment filter (a work filter beyond the "
                         "paper's method)")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-cpu-simd", action="store_true",
                    help="skip the host SIMD/multi-core implementation's four modes")
    ap.add_argument("--no-classes", action="store_true",
                    help="skip the grid-option measurements (cell classes, segment filter, prestage)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run one plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--cell-sweep", nargs="?", const="both", choices=("pip", "p2p", "both"),
                    help="instead of the step: sweep the cell size of both grids on the full "
                         "workloads (gp_sweep_cell_size) and print one JSON line")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic.json from two rocprofv3 --pmc counter "
                         "CSVs of a --copy-probe run, then exit")
    args = ap.parse_args()
    if args.traffic_from:
        write_traffic(*args.traffic_from)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (every "
              "point's result depends only on the point and the resident grid, so points "
              "would be split across GPUs by cell, each GPU holding the whole grid)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1403_0802_amd import gp

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    c3, c4 = build_workloads(args.scale)
    geom3, p3, px3, py3 = c3
    geom4, p4, px4, py4 = c4
    if args.cell_sweep:
        cell_sweep(gp, torch, dev, c3, c4, args.cell_sweep)
        return
    t0 = time.perf_counter()
    grid3 = gp.gp_build_grid("pip", geom3, p3)
    t1 = time.perf_counter()
    grid4 = gp.gp_build_grid("p2p", geom4, p4)
    t2 = time.perf_counter()
    build_ms = {"pip": 1e3 * (t1 - t0), "p2p": 1e3 * (t2 - t1)}
    x3, y3 = torch.from_numpy(px3).to(dev), torch.from_numpy(py3).to(dev)
    x4, y4 = torch.from_numpy(px4).to(dev), torch.from_numpy(py4).to(dev)
    del px3, py3
    prec = "mixed"
    ws3 = gp.new_workspace(grid3, x3.numel(), "mixed")
    ws4 = gp.new_workspace(grid4, x4.numel(), "mixed")
    id3 = torch.empty(x3.numel(), dtype=torch.int32, device=dev)
    id4 = torch.empty(x4.numel(), dtype=torch.int32, device=dev)
    d4 = torch.empty(x4.numel(), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    if args.copy_probe:
        src = torch.ones(COPY_PROBE_BYTES // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_autotune:
        # The autotuner times each kernel configuration.  PIP queries take milliseconds,
        # so it tunes on the full workload.  For P2P it tunes on a sample that keeps
        # every point of one cell in 16 (cells whose column and row are both multiples
        # of 4), so points per cell -- what the tile shape trades against -- are those
        # of the full workload.
        def cell_sample(x, y, p):
            cx = torch.floor((x - p.x0) / p.cell_size).to(torch.int64)
            cy = torch.floor((y - p.y0) / p.cell_size).to(torch.int64)
            m = (cx % 4 == 0) & (cy % 4 == 0)
            return x[m].contiguous(), y[m].contiguous()
        log("[bench] autotune pip on", x3.numel(), "points",
            gp.gp_autotune(grid3, prec, x3, y3, ws3))
        sx, sy = cell_sample(x4, y4, p4)
        log("[bench] autotune p2p on", sx.numel(), "points",
            gp.gp_autotune(grid4, prec, sx, sy, ws4))
        del sx, sy
        # the sample's winner must also beat the library default on the full workload
        # (configurations within noise of each other can swap places at full size)
        for grid, run1 in ((grid3, lambda: gp.gp_pip(grid3, x3, y3, id3, prec, ws3, stream, True)),
                           (grid4, lambda: gp.gp_p2p(grid4, x4, y4, id4, d4, prec, ws4, stream, True))):
            tuned = gp.gp_get_tuning(grid, prec)
            t_tuned = min(run1()["ms_total"] for _ in range(2))
            gp.gp_reset_tuning(grid, prec)
            default = gp.gp_get_tuning(grid, prec)
            t_default = min(run1()["ms_total"] for _ in range(2))
            if t_tuned < t_default:
                gp.gp_set_tuning(grid, prec, **tuned)
            log("[bench] full-size check: tuned %.2f ms, default %.2f ms -> %s" % (
                t_tuned, t_default, gp.gp_get_tuning(grid, prec)))

    def step(stats):
        a = gp.gp_pip(grid3, x3, y3, id3, prec, ws3, stream, stats)
        b = gp.gp_p2p(grid4, x4, y4, id4, d4, prec, ws4, stream, stats)
        return a, b

    for i in range(args.warmup):
        step(False)
        log(f"[bench] warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    st_pip, st_p2p = [], []
    t_start = time.perf_counter()
    for i in range(args.steps):
        a, b = step(True)  # stats: hipEvents around each stage on this stream
        st_pip.append(a)
        st_p2p.append(b)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    log(f"[bench] {args.steps} timed steps in {t_total:.3f}s")
    ms_step = 1e3 * t_total / args.steps
    tests_pip = st_pip[0]["tests"]
    tests_p2p = st_p2p[0]["tests"]
    value = (tests_pip + tests_p2p) / (ms_step / 1e3)

    def avg(lst, key):
        return float(np.mean([s[key] for s in lst]))

    pip_ref = avg(st_pip, "ms_refine")
    p2p_ref = avg(st_p2p, "ms_refine")
    pip_flops = tests_pip * F_PIP / (pip_ref / 1e3)
    p2p_flops = tests_p2p * F_P2P / (p2p_ref / 1e3)
    dom = "p2p" if p2p_ref >= pip_ref else "pip"
    p2p_kernel = "k_p2pmix_pre" if getattr(p4, "prestage", 0) else "k_p2pmix"
    pip_kernel = "k_pipmix_pre" if getattr(p3, "prestage", 0) else "k_pipmix"
    dom_kernel = p2p_kernel if dom == "p2p" else pip_kernel
    achieved = p2p_flops if dom == "p2p" else pip_flops
    workload = WORKLOAD_NAME
    if args.scale != 1.0:
        workload += f" (points x{args.scale})"
    traffic = load_traffic(dom_kernel, workload)
    detail = {
        "pip": {"points": x3.numel(), "tests": tests_pip, "ms": avg(st_pip, "ms_total"),
                "points_per_s": x3.numel() / (avg(st_pip, "ms_total") / 1e3),
                "ms_pairing": avg(st_pip, "ms_pairing"), "ms_refine": pip_ref,
                "ms_recheck": avg(st_pip, "ms_recheck"), "n_rechecked": st_pip[0]["n_rechecked"],
                "n_items": st_pip[0]["n_items"], "refine_tflops": pip_flops / 1e12,
                "refine_frac_fp32": pip_flops / FP32_PEAK},
        "p2p": {"points": x4.numel(), "tests": tests_p2p, "ms": avg(st_p2p, "ms_total"),
                "points_per_s": x4.numel() / (avg(st_p2p, "ms_total") / 1e3),
                "ms_pairing": avg(st_p2p, "ms_pairing"), "ms_refine": p2p_ref,
                "ms_recheck": avg(st_p2p, "ms_recheck"), "n_rechecked": st_p2p[0]["n_rechecked"],
                "n_items": st_p2p[0]["n_items"], "refine_tflops": p2p_flops / 1e12,
                "refine_frac_fp32": p2p_flops / FP32_PEAK},
        "grid_build_ms": build_ms,
        "tuning": {"pip": gp.gp_get_tuning(grid3, prec), "p2p": gp.gp_get_tuning(grid4, prec)},
    }
    # Measured ceilings of this GPU (micro-kernels in the library): FP32 FMA with VGPR
    # operands (the form of the refinement loops) and with an SGPR operand, FP64 FMA, and
    # the mixed P2P test's instruction mix on register data.
    probes = {}
    for key, which, iters in (("fp32_fma_vgpr_tflops", 0, 20000), ("fp32_fma_sgpr_tflops", 4, 20000),
                              ("fp64_fma_tflops", 1, 10000),
                              ("p2p_test_sgpr_consts_tests_per_s", 3, 5000),
                              ("p2p_test_vgpr_tests_per_s", 5, 20000),
                              ("pip_test_vgpr_2x8_tests_per_s", 6, 5000),
                              ("pip_test_vgpr_4x4_tests_per_s", 7, 5000)):
        r, _ = gp.gp_probe_rate(which, iters)
        probes[key] = r / 1e12 if key.endswith("tflops") else r
    probes["p2p_refine_vs_vgpr_probe"] = (tests_p2p / (p2p_ref / 1e3)) / probes["p2p_test_vgpr_tests_per_s"]
    probes["pip_refine_vs_vgpr_probe"] = (tests_pip / (pip_ref / 1e3)) / max(
        probes["pip_test_vgpr_2x8_tests_per_s"], probes["pip_test_vgpr_4x4_tests_per_s"])
    detail["probes"] = probes
    # PIP with cell classes (Sec. III.A): points in cells wholly inside a polygon take its
    # id untested, cells outside are skipped; same ids, fewer tests (reported apart from
    # the headline, which runs every candidate test)
    if not args.no_classes:
        from paper_1403_0802_amd import synth
        p3c = synth.GridParams(**{**p3.__dict__, "cell_classes": 1})
        t0 = time.perf_counter()
        grid3c = gp.gp_build_grid("pip", geom3, p3c)
        build_c = 1e3 * (time.perf_counter() - t0)
        tune = gp.gp_get_tuning(grid3, prec)
        gp.gp_set_tuning(grid3c, prec, **{k: tune[k] for k in tune})
        id3c = torch.empty_like(id3)
        gp.gp_pip(grid3c, x3, y3, id3c, prec, ws3, stream, False)
        stc = [gp.gp_pip(grid3c, x3, y3, id3c, prec, ws3, stream, True) for _ in range(3)]
        info = grid3c.info()
        detail["pip_cell_classes"] = {
            "ms": avg(stc, "ms_total"), "ms_refine": avg(stc, "ms_refine"),
            "ms_without": avg(st_pip, "ms_total"), "tests": stc[0]["tests"],
            "tests_avoided": stc[0]["tests_avoided"],
            "ids_equal_unclassified": bool(torch.equal(id3c, id3)),
            "pairs": {"inside": info["n_pairs_inside"], "outside": info["n_pairs_outside"],
                      "boundary": info["n_pairs_boundary"]},
            "grid_build_ms": build_c}
        del grid3c, id3c
    # P2P with per-cell segment lists: segments that cannot come within D of a cell are
    # never tested; same ids and distances (reported apart from the headline)
    if args.filters:
        from paper_1403_0802_amd import synth
        p4f = synth.GridParams(**{**p4.__dict__, "segment_filter": 1})
        t0 = time.perf_counter()
        grid4f = gp.gp_build_grid("p2p", geom4, p4f)
        build_f = 1e3 * (time.perf_counter() - t0)
        tune = gp.gp_get_tuning(grid4, prec)
        gp.gp_set_tuning(grid4f, prec, **{k: tune[k] for k in tune})
        id4f = torch.empty_like(id4)
        d4f = torch.empty_like(d4)
        gp.gp_p2p(grid4f, x4, y4, id4f, d4f, prec, ws4, stream, False)
        stf = [gp.gp_p2p(grid4f, x4, y4, id4f, d4f, prec, ws4, stream, True) for _ in range(3)]
        info = grid4f.info()
        detail["p2p_segment_filter"] = {
            "ms": avg(stf, "ms_total"), "ms_refine": avg(stf, "ms_refine"),
            "ms_without": avg(st_p2p, "ms_total"), "tests": stf[0]["tests"],
            "tests_avoided": stf[0]["tests_avoided"],
            "refine_tests_per_s": stf[0]["tests"] / (avg(stf, "ms_refine") / 1e3),
            "same_as_unfiltered": bool(torch.equal(id4f, id4) and torch.equal(d4f, d4)),
            "segment_pairs": info["n_segment_pairs"], "grid_bytes": info["device_bytes"],
            "grid_build_ms": build_f}
        del grid4f, id4f, d4f
    # P2P on the grid without build-time segment records: the kernel stages every
    # segment's cell-relative record itself; same tests, same results
    if not args.no_classes:
        from paper_1403_0802_amd import synth
        p4p = synth.GridParams(**{**p4.__dict__, "prestage": 0})
        t0 = time.perf_counter()
        grid4p = gp.gp_build_grid("p2p", geom4, p4p)
        build_p = 1e3 * (time.perf_counter() - t0)
        tune = gp.gp_get_tuning(grid4, prec)
        gp.gp_set_tuning(grid4p, prec, **{k: tune[k] for k in tune})
        id4p = torch.empty_like(id4)
        d4p = torch.empty_like(d4)
        gp.gp_p2p(grid4p, x4, y4, id4p, d4p, prec, ws4, stream, False)
        stp = [gp.gp_p2p(grid4p, x4, y4, id4p, d4p, prec, ws4, stream, True) for _ in range(3)]
        detail["p2p_plain_grid"] = {
            "ms": avg(stp, "ms_total"), "ms_refine": avg(stp, "ms_refine"),
            "ms_refine_with_records": avg(st_p2p, "ms_refine"), "tests": stp[0]["tests"],
            "refine_tests_per_s": stp[0]["tests"] / (avg(stp, "ms_refine") / 1e3),
            "same_as_headline": bool(torch.equal(id4p, id4) and torch.equal(d4p, d4)),
            "grid_bytes": grid4p.info()["device_bytes"],
            "grid_bytes_with_records": grid4.info()["device_bytes"], "grid_build_ms": build_p}
        del grid4p, id4p, d4p
    # the FP64 form on the same inputs, for comparison
    if not args.no_fp64:
        del ws3, ws4
        torch.cuda.empty_cache()
        w3 = gp.new_workspace(grid3, x3.numel(), "fp64")
        w4 = gp.new_workspace(grid4, x4.numel(), "fp64")
        gp.gp_pip(grid3, x3, y3, id3, "fp64", w3, stream, False)
        gp.gp_p2p(grid4, x4, y4, id4, d4, "fp64", w4, stream, False)
        a = gp.gp_pip(grid3, x3, y3, id3, "fp64", w3, stream, True)
        b = gp.gp_p2p(grid4, x4, y4, id4, d4, "fp64", w4, stream, True)
        ms64 = a["ms_total"] + b["ms_total"]
        detail["fp64_form"] = {
            "tests_per_s": (tests_pip + tests_p2p) / (ms64 / 1e3), "ms_per_step": ms64,
            "pip_ms_refine": a["ms_refine"], "p2p_ms_refine": b["ms_refine"],
            "pip_refine_frac_fp64": tests_pip * F_PIP / (a["ms_refine"] / 1e3) / FP64_PEAK,
            "p2p_refine_frac_fp64": tests_p2p * F_P2P / (b["ms_refine"] / 1e3) / FP64_PEAK,
            "mixed_speedup": ms64 / ms_step}
        del w3, w4
        torch.cuda.empty_cache()
    if not args.no_serve:
        log("[bench] serving run")
        del id4, d4
        torch.cuda.empty_cache()
        pools = {"pip": (x3, y3), "p2p": (x4, y4)}
        # The server holds its own P2P grid, with the cell size that suits its requests
        # (1K-4M points, most of them far fewer points than cells: 200 m cells put more
        # points in each work item); the PIP grid is the headline's (coarser PIP cells
        # are slower at every request size).
        from paper_1403_0802_amd import synth
        p4s = synth.GridParams(**{**p4.__dict__, **SERVE_P2P_GRID})
        grid4s = gp.gp_build_grid("p2p", geom4, p4s)
        detail["serving"] = serving_run(gp, torch, grid3, grid4s, pools, args.serve_requests,
                                        args.serve_warmup, prec)
        detail["serving"]["grids"] = {
            "pip": {"cell_size": p3.cell_size, "prestage": int(p3.prestage)},
            "p2p": {"cell_size_m": p4s.cell_size, "prestage": int(p4s.prestage)}}
        del grid4s
        torch.cuda.empty_cache()
        s_ = detail["serving"]
        log(f"[bench] serving: {s_['requests']} requests, p50 {s_['p50_us']:.0f} us, "
            f"p99 {s_['p99_us']:.0f} us, {s_['points_per_s']:.3g} points/s, "
            f"peak {s_['max_in_flight_requests']} requests / {s_['max_in_flight_chunks']} chunks "
            f"in flight")
        # the same stream against the headline's grids, for comparison
        h_ = serving_run(gp, torch, grid3, grid4, pools, args.serve_requests,
                         args.serve_warmup, prec)
        detail["serving_headline_grids"] = {k: h_[k] for k in (
            "requests", "p50_us", "p99_us", "mean_us", "offered_req_per_s",
            "sustained_pts_per_s", "points_per_s", "sample_equal_to_direct_calls")}
        log(f"[bench] serving on the headline grids: p50 {h_['p50_us']:.0f} us, "
            f"p99 {h_['p99_us']:.0f} us")
    if not args.no_autotune:
        detail["autotune_small"] = autotune_small_run(gp, torch)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "tests/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded stand-ins for the paper's datasets)",
        "config": {"workload": workload, "pip_points": detail["pip"]["points"],
                   "p2p_points": detail["p2p"]["points"], "pip_polygons": geom3.n_features,
                   "p2p_polylines": geom4.n_features, "radius_D_m": 100.0,
                   "pip_grid": {"cell_size": p3.cell_size, "nx": p3.nx, "ny": p3.ny,
                                "prestage": int(getattr(p3, "prestage", 0)),
                                "note": "1/512 cells, the fastest PIP query of the cell-size "
                                        "sweep (the survey's C3 grid is 1/1024), with "
                                        "build-time per-(cell, polygon) edge records"},
                   "p2p_grid": {"cell_size_m": p4.cell_size, "nx": p4.nx, "ny": p4.ny,
                                "prestage": int(getattr(p4, "prestage", 0)),
                                "note": "with build-time per-(cell, segment) FP32 records"},
                   "precision": "mixed (FP32 cell-rebased + FP64 recheck)"},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": FP32_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / FP32_PEAK, "traffic": traffic,
                     "kernel": dom_kernel,
                     "flop_per_test": F_P2P if dom == "p2p" else F_PIP},
        "cpu_baseline": None,
        "detail": detail,
    }
    if not args.no_cpu:
        log("[bench] cpu baseline")
        out["cpu_baseline"] = cpu_baseline(c3, c4, args.cpu_budget, (tests_pip, tests_p2p))
        if not args.no_cpu_simd:
            log("[bench] cpu simd modes")
            detail["cpu_simd"] = cpu_simd_run(c3, c4, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
