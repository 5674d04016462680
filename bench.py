"""Benchmark of the fused ternary wetting LB step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp32]
                    [--workload cylinder_impact] [--only] [--no-cpu]
                    [--no-serving] [--serving-slice] [--serving-fp16dev] [--serving-full]
                    [--no-sweep] [--no-3d] [--only-3d] [--copy-calibration MIB]

Workload: the compound-drop / cylinder-impact lattice, 1024 x 2048 nodes,
staircase cylinder of radius 128 (We = 10, theta = 90 deg), FP32
populations.  A step is one full pass of the hot path: the fused
stream/bounce-back/moments/wetting/chemical-potential/force/collision kernel,
plus the device mass/NaN reduction every 100 steps.  FP32 lattices like this
one advance two steps per launch (the library's default; results are bitwise
those of one step per launch), so the dominant kernel is the two-step kernel
and a launch covers two steps.  Inputs are resident in HBM before timing
starts.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor peak
STORE = {"fp64": (8, 8), "fp32": (4, 4), "fp16dev": (None, 4)}
COUNTERS = os.path.join(ROOT, "profiles", "step_kernel_counters.json")
KERNEL_SRC = os.path.join(ROOT, "paper_1710_09534_amd", "csrc", "tlb_kernels.hip")


def pop_bytes(precision: str) -> float:
    """Algorithmic bytes per fluid node-step: 27 populations read and
    written once, 4 history scalars read and written once."""
    if precision == "fp16dev":
        pops = 16 * 2 + 11 * 4      # FP16 f^i_{k!=0}; FP32 rest populations and g
    else:
        pops = 27 * STORE[precision][0]
    return 2 * pops + 2 * 4 * STORE[precision][1]


def algorithmic_bytes(problem, precision: str) -> float:
    """Per launch: fluid nodes x per-node bytes + 1 byte of material id per node."""
    n = problem["nx"] * problem["ny"]
    fluid = int((problem["material"] == 0).sum())
    return fluid * pop_bytes(precision) + n * 1.0


def kernel_sha() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def steps_per_launch(problem, precision: str) -> int:
    """Steps one launch of the dominant kernel advances: 2 where the library
    uses its two-step kernel by default (FP32 storage, any lattice), else 1."""
    return 2 if precision == "fp32" else 1


def measured_traffic(precision: str):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 --pmc summary, if it was taken on the current kernel source."""
    try:
        d = json.load(open(COUNTERS))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha") != kernel_sha():
        return None
    e = d.get("precisions", {}).get(precision)
    if not e:
        return None
    return e.get("traffic_bytes_per_launch")


def make_problem(name: str, nx=None, ny=None):
    from paper_1710_09534_amd import workloads as W
    if name == "cylinder_impact":
        return W.cylinder_impact(We=10.0, theta=90.0, **({"nx": nx, "ny": ny} if nx else {}))
    if name == "sweep":
        return W.bandwidth_case(nx or 4096, ny or 4096)
    raise SystemExit("unknown workload %s" % name)


def time_precision(tlb, torch, problem, precision, steps, warmup):
    s = tlb.from_problem(problem, precision)
    s.set_check_interval(100)
    s.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # device time of the step kernel alone (HIP events on the solver's stream)
    kms = s.time_steps(max(20, steps // 5))
    m = s.mass()
    del s
    return dt, kms, m


def host_inclusive(tlb, torch, problem, precision, steps):
    """The same workload as a whole solve through the C ABI's host-side calls:
    from the host arrays (context creation, geometry, initial fields copied
    over PCIe, equilibrium initialisation) through `steps` steps to all ten
    fields copied back to host memory, timed on the host clock.  Not the
    benchmark's value, which has the inputs resident in HBM."""
    n = problem["nx"] * problem["ny"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = tlb.from_problem(problem, precision)
    s.set_check_interval(100)
    s.step(steps)
    s.read_fields()
    dt = time.perf_counter() - t0
    del s
    return {"precision": precision, "steps": steps, "seconds": round(dt, 4),
            "mlups": round(n * steps / dt / 1e6, 1)}


def bw_sweep_leg(tlb, torch, sizes=((1024, 2048), (2048, 2048), (4096, 4096)), steps=500):
    """The cylinder layout without a drop at three sizes and every storage
    precision: step-kernel time from HIP events on the solver's stream over
    `steps` launches, and the algorithmic bandwidth it implies.  The FP64
    and FP32 working sets exceed the 256 MB MALL at every size."""
    from paper_1710_09534_amd import workloads as W
    out = []
    for nx, ny in sizes:
        prob = W.bandwidth_case(nx, ny)
        n = nx * ny
        for prec in ("fp64", "fp32", "fp16dev"):
            s = tlb.from_problem(prob, prec)
            s.set_check_interval(0)
            s.time_steps(20)
            kms = s.time_steps(steps)
            del s
            torch.cuda.synchronize()
            gbs = algorithmic_bytes(prob, prec) / (kms * 1e-3) / 1e9
            out.append({"size": "%dx%d" % (nx, ny), "precision": prec,
                        "kernel_ms": round(kms, 4), "mlups": round(n / kms / 1e3, 1),
                        "algorithmic_gbs": round(gbs, 1),
                        "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)})
            print("# bw sweep %s %s %.4f ms %.0f MLUPS %.0f GB/s" %
                  (out[-1]["size"], prec, kms, out[-1]["mlups"], gbs), file=sys.stderr, flush=True)
    return out


def leg_3d(tlb, torch, steps=100):
    """The three-dimensional (D3Q19) step on the sphere-impact lattice
    (192 x 192 x 256, compound drop onto a staircase sphere): device time per
    step from HIP events, MLUPS and the algorithmic bandwidth (populations and
    history read and written once: 2 * (57 + 5) * s bytes per fluid node, plus
    1 byte of material per node)."""
    from paper_1710_09534_amd import workloads as W
    prob = W.sphere_impact3d()
    n = prob["nx"] * prob["ny"] * prob["nz"]
    fluid = int((prob["material"] == 0).sum())
    out = {"workload": "sphere_impact3d %dx%dx%d" % (prob["nx"], prob["ny"], prob["nz"])}
    for prec, s in (("fp32", 4), ("fp64", 8)):
        sol = tlb.from_problem3(prob, prec)
        sol.set_check_interval(0)
        sol.time_steps(5)
        kms = sol.time_steps(steps)
        del sol
        torch.cuda.synchronize()
        alg = fluid * 2 * (57 + 5) * s + n
        gbs = alg / (kms * 1e-3) / 1e9
        out[prec] = {"ms_per_step": round(kms, 4), "mlups": round(n / kms / 1e3, 1),
                     "algorithmic_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
        print("# 3-D %s: %.4f ms/step %.0f MLUPS %.0f GB/s" % (prec, kms, n / kms / 1e3, gbs),
              file=sys.stderr, flush=True)
    return out


def batching_leg(tlb, torch, precision="fp32", n_lattices=256, size=64, steps=200):
    """Many small lattices (the serving stream's most common size) advanced
    one at a time versus together in batched, graph-replayed launches (two
    steps per launch, the batch default for FP32, and one step per launch);
    the same lattices one at a time with the plain FP64 path are the
    reference."""
    from paper_1710_09534_amd import workloads as W
    rng = W.Rng(99)
    probs = [W.serving_request(W.Rng(rng.next_u64()), size, i % 3, (steps, steps))
             for i in range(n_lattices)]
    solvers = [tlb.from_problem(p, precision) for p in probs]
    for s in solvers:
        s.set_check_interval(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in solvers:
        s.step(steps)
    torch.cuda.synchronize()
    t_solo = time.perf_counter() - t0
    b = tlb.Batch(n_lattices)
    b.set(solvers)
    b.use_graph(48)
    b.step(50)
    b.sync()
    t0 = time.perf_counter()
    b.step(steps)
    b.sync()
    t_batch = time.perf_counter() - t0
    # the same batch with two-step strip heights from the batch autotuner
    rows = b.autotune_pair_rows(10)
    b.use_graph(48)
    b.step(50)
    b.sync()
    t0 = time.perf_counter()
    b.step(steps)
    b.sync()
    t_tuned = time.perf_counter() - t0
    # the same batch at one step per launch (its default for FP32 members is
    # two steps per launch)
    b.set_pair_rows(0)
    b.use_graph(48)
    b.step(48)
    b.sync()
    t0 = time.perf_counter()
    b.step(steps)
    b.sync()
    t_one = time.perf_counter() - t0
    del b, solvers
    solvers = [tlb.from_problem(p, "fp64") for p in probs]
    for s in solvers:
        s.set_check_interval(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in solvers:
        s.step(steps)
    torch.cuda.synchronize()
    t_fp64 = time.perf_counter() - t0
    del solvers
    nodes = n_lattices * size * size
    return {"lattices": n_lattices, "size": "%dx%d" % (size, size), "precision": precision,
            "steps": steps, "one_at_a_time_mlups": round(nodes * steps / t_solo / 1e6, 1),
            "pair_autotuned_rows": rows,
            "batched_autotuned_mlups": round(nodes * steps / t_tuned / 1e6, 1),
            "batched_mlups": round(nodes * steps / t_batch / 1e6, 1),
            "batched_one_step_per_launch_mlups": round(nodes * steps / t_one / 1e6, 1),
            "speedup": round(t_solo / t_batch, 2),
            "one_at_a_time_fp64_mlups": round(nodes * steps / t_fp64 / 1e6, 1),
            "speedup_vs_fp64": round(t_fp64 / t_batch, 2)}


def serving_leg(tlb, torch, precision="fp32", n_requests=120, steps=(1000, 4000),
                arena_gb=40.0, slots=64, quantum=250, calibrate_sequential=False,
                loads=(0.7, 1.2), sequential=True):
    """A seeded stream of independent drop solves (sizes 64^2..1024^2
    weighted 0.40/0.30/0.15/0.10/0.05, single/binary/compound drops, random
    angles and surface tensions) served with continuous batching under an
    HBM arena, at Poisson loads of 0.7x and 1.2x the measured capacity; and
    the same stream solved one request at a time by the plain FP64 path
    (FIFO, one request on the GPU at a time).  With calibrate_sequential the
    FP64 service time of each request is its size class's measured set-up
    time plus its steps times the class's measured time per step, instead
    of running every request.  loads: the Poisson loads to replay;
    sequential=False skips the one-at-a-time FP64 comparison."""
    from paper_1710_09534_amd import workloads as W
    stream = W.serving_stream(n_requests, seed=2026, steps=steps)
    probs = [f() for (_, _, f) in stream]
    work = sum(p["nx"] * p["ny"] * p["steps"] for p in probs)

    def run(arrivals, tag):
        srv = tlb.Server(int(arena_gb * (1 << 30)), max_slots=slots, precision=precision,
                         quantum=quantum)
        t0 = time.perf_counter()
        ids = []
        for p, ta in zip(probs, arrivals):
            now = time.perf_counter() - t0
            if ta > now:
                time.sleep(ta - now)
            ids.append(srv.submit(p, p["steps"], fields=0))
        last = time.perf_counter()
        for k, i in enumerate(ids):
            srv.wait(i, 1800.0)
            if time.perf_counter() - last > 30.0:
                last = time.perf_counter()
                print("# serving %s: %d/%d done at %.0f s" % (tag, k + 1, len(ids), last - t0),
                      file=sys.stderr, flush=True)
        makespan = time.perf_counter() - t0
        lat = np.array([srv.latency(i) for i in ids])
        st = srv.stats()
        srv.close()
        print("# serving %s: makespan %.1f s" % (tag, makespan), file=sys.stderr, flush=True)
        return makespan, lat, st

    # capacity: everything submitted at once
    makespan, lat, st = run([0.0] * len(probs), "capacity")
    cap = len(probs) / makespan
    out = {"requests": len(probs), "precision": precision, "steps_range": list(steps),
           "arena_gb": arena_gb, "slots": slots, "quantum": quantum,
           "capacity_req_per_s": round(cap, 2),
           "closed_batch_mlups": round(work / makespan / 1e6, 1)}
    for load in loads:
        tag = "load_%g" % load
        arr = W.poisson_arrivals(len(probs), load * cap, seed=7)
        makespan, lat, st = run(arr, tag)
        out[tag] = {"p50_s": round(float(np.percentile(lat, 50)), 4),
                    "p99_s": round(float(np.percentile(lat, 99)), 4),
                    "aggregate_mlups": round(work / makespan / 1e6, 1),
                    "failed": int(st["failed"])}

    if not sequential:
        return out

    def solo(p, nsteps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = tlb.from_problem(p, "fp64")
        s.set_check_interval(0)
        if nsteps:
            s.step(nsteps)
        s.mass()
        dt = time.perf_counter() - t0
        del s
        return dt

    if calibrate_sequential:
        # per size class: set-up (create, init, readout of the mass) and time
        # per step of the plain FP64 path on that size alone
        cal = {}
        for p in probs:
            n = p["nx"]
            if n in cal:
                continue
            t_set = solo(p, 0)
            t_run = solo(p, 400) - t_set
            cal[n] = (t_set, t_run / 400.0)
        service = [cal[p["nx"]][0] + cal[p["nx"]][1] * p["steps"] for p in probs]
        out["sequential_fp64_model"] = {str(k): {"setup_s": round(v[0], 4),
                                                 "ms_per_step": round(1e3 * v[1], 4)}
                                        for k, v in sorted(cal.items())}
    else:
        service = [solo(p, p["steps"]) for p in probs]
    for load in loads:
        tag = "load_%g" % load
        arr = W.poisson_arrivals(len(probs), load * cap, seed=7)
        fin, tts = 0.0, []
        for ta, sv in zip(arr, service):
            fin = max(fin, ta) + sv
            tts.append(fin - ta)
        out[tag]["sequential_fp64_p50_s"] = round(float(np.percentile(tts, 50)), 4)
        out[tag]["sequential_fp64_p99_s"] = round(float(np.percentile(tts, 99)), 4)
    out["sequential_fp64_mlups"] = round(work / sum(service) / 1e6, 1)
    return out


def copy_reference(torch, mib=1024, reps=10):
    """A plain device-to-device copy of mib MiB (torch copy_, its own kernel):
    the practical streaming ceiling beside the 8 TB/s peak, read plus write
    bytes per second, timed with HIP events on torch's current stream (where
    the copies run)."""
    nb = mib << 20
    a = torch.ones(nb // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        b.copy_(a)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    gbs = 2 * nb / (ms * 1e-3) / 1e9
    del a, b
    return {"copy_bytes_each_way": nb, "ms": round(ms, 4), "gbs_read_plus_write": round(gbs, 1),
            "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4)}


def stream_reference(tlb, torch, mib=1024, nx=1024, ny=2048, rows=64, reps=20):
    """Hand-written streaming references (the library's probe kernels), read
    plus write bytes per second: a copy in 16-byte words (dwordx4) of mib MiB,
    and the step kernel's FP32 access shape without its arithmetic (31 planes
    read at the pulled offsets and written, 248 B per node) on the benchmark
    lattice with the benchmark's 64-row strips."""
    nb = mib << 20
    a = torch.ones(nb // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    ms0 = tlb.probe_bandwidth(0, a, b, reps=reps)
    del a, b
    pitch = -(-nx // 64) * 64
    n31 = 31 * pitch * ny
    a = torch.ones(n31, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    ms1 = tlb.probe_bandwidth(1, a, b, nx=nx, ny=ny, tile_rows=rows, reps=reps)
    del a, b
    g0 = 2 * nb / (ms0 * 1e-3) / 1e9
    g1 = 248.0 * nx * ny / (ms1 * 1e-3) / 1e9
    return {"copy16": {"bytes_each_way": nb, "ms": round(ms0, 4), "gbs_read_plus_write": round(g0, 1),
                       "frac_of_peak": round(g0 / HBM_PEAK_GBS, 4)},
            "step_shape_fp32": {"lattice": "%dx%d" % (nx, ny), "tile_rows": rows,
                                "ms": round(ms1, 4), "gbs_read_plus_write": round(g1, 1),
                                "frac_of_peak": round(g1 / HBM_PEAK_GBS, 4)}}


def config_table(tlb, torch, cpu=True, gpu_steps=400, oracle_budget_s=2.0):
    """Per-configuration rates: the 64x64 reduction case, binary drops
    256x128, the compound drop between moving walls 512x256 and the
    1024x2048 cylinder impact, each on the GPU in every storage precision
    (step-kernel device time from HIP events over gpu_steps launches) and,
    with cpu, the FP64 oracle on one thread and on all host cores (as many
    steps as fit oracle_budget_s after one untimed step; the rate is
    extrapolated from that sample).  The three small lattices fit in the
    memory-side cache, so only the cylinder row's %HBM is a roofline figure."""
    from paper_1710_09534_amd import workloads as W
    rows = [("C1 reduction 64x64", W.reduction_case()),
            ("C2 binary drops 256x128", W.binary_drops(seed=0)),
            ("C3 compound drop under shear 512x256", W.compound_shear(seed=0)),
            ("C4 cylinder impact 1024x2048", W.cylinder_impact(We=10.0, theta=90.0))]
    out = []
    cores = None
    if cpu:
        import oracle
        cores = oracle.Oracle.num_threads()
    for name, prob in rows:
        n = prob["nx"] * prob["ny"]
        row = {"config": name, "nodes": n}
        for prec in ("fp64", "fp32", "fp16dev"):
            s = tlb.from_problem(prob, prec)
            s.set_check_interval(0)
            s.time_steps(20)
            kms = s.time_steps(gpu_steps)
            del s
            torch.cuda.synchronize()
            row["gpu_%s_mlups" % prec] = round(n / kms / 1e3, 1)
            if name.startswith("C4"):
                gbs = algorithmic_bytes(prob, prec) / (kms * 1e-3) / 1e9
                row["hbm_frac_%s" % prec] = round(gbs / HBM_PEAK_GBS, 4)
        if cpu:
            import oracle
            r_all, k_all = oracle_rate(prob, oracle_budget_s, 2000)
            oracle.Oracle.set_num_threads(1)
            try:
                r_one, k_one = oracle_rate(prob, oracle_budget_s, 2000)
            finally:
                oracle.Oracle.set_num_threads(cores)
            row["oracle_1thread_mlups"] = round(r_one, 3)
            row["oracle_all_cores_mlups"] = round(r_all, 3)
            row["oracle_steps_timed"] = [k_one, k_all]
        out.append(row)
        print("# config %s: %s" % (name, row), file=sys.stderr, flush=True)
    return {"oracle_cores": cores, "cpu_model": cpu_model() if cpu else None, "rows": out}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_rate(problem, budget_s, max_steps):
    """MLUPS of the FP64 oracle on `problem`: one untimed step, then as many
    steps as fit the budget (at most max_steps)."""
    import oracle
    o = oracle.Oracle(problem)
    o.init(problem["c1"], problem["c2"], problem["ux"], problem["uy"])
    t0 = time.perf_counter()
    o.step(1)
    one = time.perf_counter() - t0
    k = max(1, min(max_steps, int(budget_s / max(one, 1e-3))))
    t0 = time.perf_counter()
    o.step(k)
    dt = time.perf_counter() - t0
    del o
    return problem["nx"] * problem["ny"] * k / dt / 1e6, k


def cpu_baseline(problem, budget_s=12.0, single_budget_s=6.0):
    import oracle
    cores = oracle.Oracle.num_threads()
    rate, k = oracle_rate(problem, budget_s, 50)
    oracle.Oracle.set_num_threads(1)
    try:
        rate1, k1 = oracle_rate(problem, single_budget_s, 20)
    finally:
        oracle.Oracle.set_num_threads(cores)
    return {"value": round(rate, 3), "unit": "MLUPS", "cores": cores,
            "kind": "oracle",
            "sample": "%d steps of the %dx%d workload (after 1 untimed step), FP64 oracle"
                      % (k, problem["nx"], problem["ny"]),
            "single_thread": {"value": round(rate1, 3), "unit": "MLUPS",
                              "sample": "%d steps, 1 thread" % k1},
            "cpu_model": cpu_model()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "fp16dev"])
    ap.add_argument("--workload", default="cylinder_impact")
    ap.add_argument("--nx", type=int, default=None)
    ap.add_argument("--ny", type=int, default=None)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only", action="store_true", help="time the headline precision only")
    ap.add_argument("--no-serving", action="store_true", help="skip the batching and serving legs")
    ap.add_argument("--no-sweep", action="store_true", help="skip the bandwidth sweep leg")
    ap.add_argument("--no-3d", action="store_true", help="skip the three-dimensional leg")
    ap.add_argument("--only-3d", action="store_true",
                    help="run only the three-dimensional leg (--steps steps per precision)")
    ap.add_argument("--serving-slice", action="store_true",
                    help="serve a 120-request, 1000-4000-step slice of the stream instead of the "
                         "whole 1000-request stream (seconds instead of about three minutes)")
    ap.add_argument("--serving-fp16dev", action="store_true",
                    help="also serve the stream with FP16-deviation storage (capacity, 0.7x load)")
    ap.add_argument("--serving-full", action="store_true",
                    help="serve only the whole stream (with --only: nothing else is timed)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB, 10 times (counter scale)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        print(json.dumps(copy_reference(torch, args.copy_calibration)), flush=True)
        return
    from paper_1710_09534_amd import tlb

    if args.only_3d:
        # diagnostic mode (profiling): the three-dimensional leg alone
        print(json.dumps({"d3q19": leg_3d(tlb, torch, steps=args.steps)}), flush=True)
        return
    problem = make_problem(args.workload, args.nx, args.ny)
    n = problem["nx"] * problem["ny"]
    fluid = int((problem["material"] == 0).sum())
    precs = [args.precision] if args.only else ["fp64", "fp32", "fp16dev"]
    table = {}
    for prec in precs:
        dt, kms, m = time_precision(tlb, torch, problem, prec, args.steps, args.warmup)
        alg = algorithmic_bytes(problem, prec)
        table[prec] = {
            "mlups": round(n * args.steps / dt / 1e6, 1),
            "fluid_mlups": round(fluid * args.steps / dt / 1e6, 1),
            "ms_per_step": round(dt * 1e3 / args.steps, 5),
            "kernel_ms": round(kms, 5),
            "bytes_per_node_step": pop_bytes(prec),
            "hbm_frac_algorithmic": round(alg / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "mass_final": [float(x) for x in m],
        }
        print("# %s: %.1f MLUPS, kernel %.4f ms, %.1f%% of HBM peak (algorithmic)"
              % (prec, table[prec]["mlups"], kms, 100 * table[prec]["hbm_frac_algorithmic"]),
              file=sys.stderr, flush=True)
    head = table[args.precision]
    spl = steps_per_launch(problem, args.precision)
    alg = algorithmic_bytes(problem, args.precision)
    # per launch: spl steps' algorithmic bytes over spl steps' kernel time
    achieved = alg / (head["kernel_ms"] * 1e-3) / 1e9
    traffic = measured_traffic(args.precision)
    kname = ("step2_kernel<1, 0u> (two steps per launch, fp32 populations)" if spl == 2 else
             "step_kernel<%d> (%s populations)" % ({"fp64": 0, "fp32": 1, "fp16dev": 2}[args.precision],
                                                   args.precision))
    out = {
        "metric": "MLUPS & %HBM peak per ternary step (FP64 vs FP32/FP16-store); p50/p99 solve latency",
        "value": head["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp16dev": "f16-store/f32"}[args.precision],
        "data": "synthetic",
        "config": {"workload": "%s %dx%d (compound drop on a staircase cylinder R=128, We=10, "
                               "theta=90), %s populations"
                               % (args.workload, problem["nx"], problem["ny"], args.precision),
                   "nx": problem["nx"], "ny": problem["ny"], "fluid_nodes": fluid,
                   "precision": args.precision, "check_interval": 100},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     # measured HBM bytes per launch over the launch time: the
                     # real traffic rate (about half the algorithmic one when a
                     # launch covers two steps)
                     "traffic_gbs": (round(traffic / (spl * head["kernel_ms"] * 1e-3) / 1e9, 1)
                                     if traffic else None),
                     "kernel": kname, "steps_per_launch": spl,
                     "algorithmic_bytes_per_launch": spl * alg},
        "precisions": table,
    }
    if not (args.only or args.no_sweep):
        out["bw_sweep"] = bw_sweep_leg(tlb, torch)
    if not (args.only or args.no_3d):
        out["d3q19"] = leg_3d(tlb, torch)
    out["host_inclusive"] = host_inclusive(tlb, torch, problem, args.precision, args.steps)
    out["copy_reference"] = copy_reference(torch)
    out["stream_reference"] = stream_reference(tlb, torch)
    if not args.only:
        out["configs"] = config_table(tlb, torch, cpu=not args.no_cpu)
    # the whole seeded stream of the serving workload: 1000 requests of
    # 1000-20000 steps under a 200 GB arena, 128 slots, at 0.7x and 1.2x the
    # measured capacity, against the same stream served one request at a
    # time by the plain FP64 path (service times from per-size-class
    # measurements of that path)
    full = dict(n_requests=1000, steps=(1000, 20000), arena_gb=200.0, slots=128, quantum=500,
                calibrate_sequential=True)
    if not (args.only or args.no_serving):
        out["batching"] = batching_leg(tlb, torch)
        print("# batching: %s" % out["batching"], file=sys.stderr, flush=True)
    if args.serving_full or not (args.only or args.no_serving):
        if args.serving_slice and not args.serving_full:
            out["serving"] = serving_leg(tlb, torch)
        else:
            out["serving"] = serving_leg(tlb, torch, **full)
            out["serving"]["stream"] = "full: 1000 requests, 1000-20000 steps, 200 GB arena"
        print("# serving: %s" % out["serving"], file=sys.stderr, flush=True)
        if args.serving_fp16dev:
            kw = dict(full, calibrate_sequential=False)
            if args.serving_slice and not args.serving_full:
                kw = {}
            out["serving_fp16dev"] = serving_leg(tlb, torch, precision="fp16dev", loads=(0.7,),
                                                 sequential=False, **kw)
            print("# serving fp16dev: %s" % out["serving_fp16dev"], file=sys.stderr, flush=True)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(problem)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
