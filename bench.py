"""Benchmark: reachability solves to 1e-10 error on one MI355X.

Default workload (--workload batched_mixed_leaky): 256 independent random
chains packed block-diagonally, n log-uniform in [1,000, 200,000] (7.68 M
states, 34.3 M transitions), out-degree uniform in [1, 8], weights uniform on
(0,1] normalised, 1% goal states and 1% absorbing non-goal states per chain
(the literal recipe has no sinks, so most chains would have S_? empty; the
sinks make every chain a real solve).  One step runs the whole hot path on
the batch:
  precompute (validation, the two backward searches, reduced system),
  Jacobi FP64, BiCGStab FP64, Jacobi FP32-in-FP64-refinement,
  BiCGStab FP32-in-FP64-refinement (all certified to max|x - x*| <= 1e-10),
  and the adjoint solve (FP32 inside FP64 refinement) + gradient of x at the
  first undecided state of every chain.
value = solves per second (5 solves per chain per step).

Prints one JSON line.  --gpus above 1 is refused (single-GPU build).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "solves/s & HBM GB/s to 1e-10 error: FP64 vs FP32-refined vs batched"
HBM_PEAK_GBS = 8000.0
PMC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1210_6412_amd", "csrc", f)
                  for f in ("rp_kernels.hip", "rp_internal.h", "rp_api.hip")]


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def pmc_traffic(kernel_id, kernel_name=None, workload=None):
    """HBM bytes per launch of a kernel from the committed rocprofv3 FETCH_SIZE
    and WRITE_SIZE runs (scaled by a plain copy of known size), or None when
    the kernel sources changed since the counters were taken, the counters
    were taken on another workload, or they are of another kernel than
    kernel_name (a name or name prefix: another row layout)."""
    try:
        with open(PMC_FILE) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("sources_sha256") != kernel_sources_sha256():
        return None
    if workload is not None and d.get("workload") != workload:
        return None
    entries = d.get("kernels", {}).get(kernel_id)
    if entries is None:
        return None
    for e in entries if isinstance(entries, list) else [entries]:
        if kernel_name is None or str(e.get("kernel", "")).startswith(kernel_name):
            return e.get("traffic_bytes_per_launch")
    return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_batch(batch):
    import chaingen as cg
    chains = [cg.random_sparse(20_000, 1, 16, 0.01, 0.01, cg.SEED_BASE + 2 + 1000 * i) for i in range(batch)]
    return cg.concat(chains, name=f"{batch} x random_sparse(n=20000,deg=1..16)")


WORKLOADS = {
    "batch": "B chains of 20,000 states (out-degree 1..16, 1% goals, 1% sinks; 64 chains: ~150 MB per FP64 "
             "sweep, which the 256 MB last-level cache holds)",
    "gamblers_ruin": "gambler's ruin, 1,000 states, p = 0.45",
    "random_sparse": "one random sparse chain, 20,000 states, out-degree 1..16",
    "dense_random": "dense random chain, 8,192 states, 10% density (every state reaches the goals: S? empty)",
    "program_graph": "model-checker-shaped chain, 2,000,000 states, successors within +-64 or a 2% jump",
    "batched_mixed": "256 random sparse chains, 1,000..200,000 states (log-uniform), out-degree 1..8",
    "program_graph_2p25": "the model-checker-shaped chain at 2^25 = 33,554,432 states (~1.2 GB FP64 sweep: "
                          "far larger than the last-level cache)",
    "batch_1024": "1,024 chains of 20,000 states (20.5 M states, ~2 GB FP64 sweep)",
    "dense_random_leaky": "dense random chain, 8,192 states, 10% density, plus 0.5% absorbing non-goal states",
    "batched_mixed_leaky": "the default: the 256 chains of batched_mixed with 1% absorbing non-goal states each",
}


def make_workload(name, batch):
    import chaingen as cg
    if name == "batch":
        return make_batch(batch)
    if name == "dense_random_leaky":
        return cg.dense_random(8192, 0.10, 0.005, 0.005, cg.SEED_BASE + 3)
    if name == "program_graph_2p25":
        return cg.program_graph(1 << 25, 0.01, 0.001, 64, 0.02, cg.SEED_BASE + 4)
    if name == "batch_1024":
        return make_batch(1024)
    if name == "batched_mixed_leaky":
        return cg.batched(256, 1_000, 200_000, 1, 8, 0.01, 0.01, cg.SEED_BASE + 5)
    return {"gamblers_ruin": cg.CONFIGS[1], "random_sparse": cg.CONFIGS[2], "dense_random": cg.CONFIGS[3],
            "program_graph": cg.CONFIGS[4], "batched_mixed": cg.CONFIGS[5]}[name]()


def _oracle_chains(chains, budget_s, keep=None):
    """The oracle as it stands, single-threaded, on whole chains in turn until
    about budget_s: partition, reduced system, certificate, certified Jacobi
    and BiCGStab, adjoint solve and gradient (3 solves per chain).  Returns
    (solves, chains done, states done, seconds); keep (a list), when given,
    receives the oracle's certified solution of each chain done."""
    import oracle
    solves = done = states = 0
    t0 = time.perf_counter()
    for c in chains:
        j = oracle.solve(c.n, c.rp, c.col, c.val, c.goal, "jacobi", tol=1e-10, stop_mode=1)
        if keep is not None:
            keep.append(j.x)
        oracle.solve(c.n, c.rp, c.col, c.val, c.goal, "bicgstab", tol=1e-10, stop_mode=1)
        sq = np.nonzero(j.cls == oracle.SQ)[0]
        if sq.size:
            seed = np.zeros(c.n)
            seed[sq[0]] = 1.0
            lam, _, _, _ = oracle.adjoint(j, seed, tol=1e-10)
            oracle.gradient(c.n, c.rp, c.col, j.cls, j.red, lam, j.x)
        solves += 3
        done += 1
        states += c.n
        if time.perf_counter() - t0 >= budget_s:
            break
    return solves, done, states, time.perf_counter() - t0


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(chain, budget_s=12.0, max_workers=16, gpu_x=None):
    """The oracle timed on the host: one thread on the workload's chains in
    batch order for about budget_s, then every available core (at most
    max_workers single-threaded oracle processes, each on its own chains, the
    oracle itself unchanged) for about budget_s.  value is the all-cores rate.
    gpu_x (solver name -> full solution of the workload): the largest
    difference of each GPU solution from the oracle's certified solution over
    the chains the single-thread leg solved."""
    import multiprocessing as mp
    order = list(range(chain.num_instances))
    ref = []
    single = _oracle_chains((chain.instance(k) for k in order), budget_s, keep=ref)
    errs = {}
    for name, xg in (gpu_x or {}).items():
        errs[name] = max(float(np.abs(xg[chain.inst_off[k]:chain.inst_off[k + 1]] - ref[k]).max())
                         for k in range(len(ref)))
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    workers = max(1, min(max_workers, avail))
    # chains dealt round-robin from a seeded shuffle, so that every worker
    # gets a similar mix of sizes; each worker stops after about budget_s
    rng = np.random.Generator(np.random.PCG64(1))
    perm = rng.permutation(chain.num_instances)
    lists = [[chain.instance(int(k)) for k in perm[w::workers][:8]] for w in range(workers)]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(workers) as pool:
        res = pool.starmap(_oracle_chains, [(lst, budget_s) for lst in lists])
    wall = time.perf_counter() - t0
    solves = sum(r[0] for r in res)
    span = max(r[3] for r in res)
    return {"value": solves / span, "unit": "solves/s", "cores": workers, "kind": "oracle",
            "max_abs_err_gpu_vs_oracle": errs, "chains_compared": len(ref),
            "single_thread_value": single[0] / single[3],
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(), "cores_available": avail,
            "sample": f"oracle (plain single-threaded FP64 C, -O2) on whole chains of the workload, per chain: "
                      f"partition + reduced system + certificate + certified Jacobi + certified BiCGStab + "
                      f"adjoint solve and gradient (3 solves). One thread: {single[1]} chain(s) in batch order "
                      f"({single[2]} states) in {single[3]:.1f} s. All cores: {workers} processes, "
                      f"{sum(r[1] for r in res)} chains ({sum(r[2] for r in res)} states) in {span:.1f} s "
                      f"(pool wall {wall:.1f} s)"}


def section6_cpu_baseline(ms):
    """CPU-baseline leg of the Section 6 experiment: the oracle (plain
    single-threaded FP64 C) timed on the host on the same systems, certified
    to 1e-10 by Varah's bound, per method (ms for all of them)."""
    import oracle
    out = {}
    for name in ("jacobi", "bicgstab"):
        t0 = time.perf_counter()
        for mk in ms:
            oracle.solve_matrix(mk.n, mk.rp, mk.col, mk.val, mk.rhs, name, tol=1e-10)
        out[name] = round(1000 * (time.perf_counter() - t0), 3)
    return out


def section6_sweep(steps=3):
    """The paper's own experiments (Section 6, Figs. 1-3; Section 7.1 shapes
    of Table 1) on this build: random strictly diagonally dominant
    positive-integer systems A x = b solved by the GPU Jacobi and BiCGStab
    kernels (FP64, certified to 1e-10 by Varah's bound), with the oracle's
    single-threaded CPU times beside the small ones.  Returns a list of
    points."""
    import torch
    import chaingen as cg
    import paper_1210_6412_amd as rp
    from paper_1210_6412_amd import binding as B
    dev = torch.device("cuda", 0)
    ctx = rp.rp_context_create(0)
    points = []
    specs = [("density", n, d, 1) for n in (1000, 4000, 16000) for d in (0.001, 0.01, 0.05, 0.10)]
    specs += [("size_at_10pct", n, 0.10, 1) for n in (500, 2000, 8000)]
    specs += [("table1_shape", n, m, 40) for n, m in ((92, 211), (313, 669), (667, 1333), (7647, 15293))]
    for kind, n, arg, K in specs:
        if kind == "table1_shape":
            ms = [cg.diag_dominant(n, offdiag=arg - n, seed=cg.SEED_BASE + 60 + i) for i in range(K)]
        else:
            ms = [cg.diag_dominant(n, density=arg, seed=cg.SEED_BASE + 60)]
        m = cg.concat_matrices(ms) if K > 1 else ms[0]
        t = [torch.from_numpy(a).to(dev) for a in (m.rp, m.col, m.val, m.rhs)]
        sys_ = rp.rp_matrix_system(ctx, *t, list(m.inst_off))
        pt = {"kind": kind, "n": n, ("nnz" if kind == "table1_shape" else "density"): arg, "systems": K,
              "nnz_total": m.nnz}
        x = torch.empty(m.n, dtype=torch.float64, device=dev)
        for name, fn in (("jacobi", rp.rp_jacobi), ("bicgstab", rp.rp_bicgstab)):
            fn(ctx, sys_, x, tol=1e-10, stop=B.RP_STOP_CERTIFIED)  # warm (layout tuning)
            ts = []
            for _ in range(steps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, info, code = fn(ctx, sys_, x, tol=1e-10, stop=B.RP_STOP_CERTIFIED)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            pt[name] = {"gpu_ms": round(1000 * sorted(ts)[len(ts) // 2], 3), "status": B.STATUS_NAMES[code],
                        "iterations": max(i["iterations"] for i in info),
                        "error_bound": max(i["error_bound"] for i in info)}
        if m.nnz <= 2_000_000:
            for name, ms_cpu in section6_cpu_baseline(ms).items():
                pt[name]["cpu_oracle_ms"] = ms_cpu
        sys_.close()
        points.append(pt)
        log(f"section 6 point {kind} n={n} {arg}: jacobi {pt['jacobi']['gpu_ms']} ms, "
            f"bicgstab {pt['bicgstab']['gpu_ms']} ms")
    return points


def jacobi_variants(chain, sweeps=50):
    """Jacobi update rules and row-sum layouts on one workload: time per
    sweep (kernel time over a fixed number of sweeps, HIP events) and the
    sweeps and wall time of a certified 1e-10 solve, FP64.  Layouts: the
    tuned tiles (the default), two-buffer sweeps on row chunks read from
    device memory, the in-place update (Section 5.1) and segmented-scan row
    sums (Section 8) on the same row chunks."""
    import torch
    import paper_1210_6412_amd as rp
    from paper_1210_6412_amd import binding as B
    dev = torch.device("cuda", 0)
    ctx = rp.rp_context_create(0)
    t = [torch.from_numpy(a).to(dev) for a in (chain.rp, chain.col, chain.val, chain.goal)]
    sys_ = rp.rp_precompute(ctx, t[0], t[1], t[2], t[3], list(chain.inst_off), 0, 0.0)
    x = torch.empty(chain.n, dtype=torch.float64, device=dev)
    kinds = {"tiled_tuned": {}, "chunks_two_buffer": dict(tiling=B.RP_TILING_OFF, schedule=1),
             "chunks_in_place": dict(update=B.RP_UPDATE_IN_PLACE),
             "chunks_segscan": dict(schedule=B.RP_SCHEDULE_SEGSCAN)}
    out = {}
    for name, kw in kinds.items():
        rp.rp_jacobi(ctx, sys_, x, tol=1e-10, stop=B.RP_STOP_CERTIFIED, **kw)  # warm (layout tuning)
        B.rp_profile_enable(ctx, True)
        rp.rp_jacobi(ctx, sys_, x, tol=0.0, max_iter=sweeps, stop=B.RP_STOP_DELTA, **kw)
        pr = B.rp_profile_read(ctx)
        B.rp_profile_enable(ctx, False)
        n, ms, b = pr["jacobi_fp64"]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info, code = rp.rp_jacobi(ctx, sys_, x, tol=1e-10, stop=B.RP_STOP_CERTIFIED, **kw)
        torch.cuda.synchronize()
        out[name] = {"us_per_sweep": round(1000 * ms / max(n, 1), 2),
                     "alg_GBps": round(b / (ms * 1e6), 1) if ms else None,
                     "certified_ms": round(1000 * (time.perf_counter() - t0), 2),
                     "certified_sweeps_max": max(i["iterations"] for i in info), "status": B.STATUS_NAMES[code]}
        log(f"jacobi variant {name}: {out[name]}")
    sys_.close()
    return out


def scc_compare(steps=3):
    """Solve by strongly connected components (Section 8's proposal) against
    the ordinary certified solve, FP64 to 1e-10, on chains whose S_? has
    different component structure: the default batch (one large component
    per chain), blocks in sequence, an acyclic path, the model-checker-shaped
    chain.  Reports decomposition time, counts, and the median wall time of
    each solve."""
    import torch
    import chaingen as cg
    import paper_1210_6412_amd as rp
    from paper_1210_6412_amd import binding as B
    dev = torch.device("cuda", 0)
    ctx = rp.rp_context_create(0)
    out = []
    chains = [make_workload("batched_mixed_leaky", 0), cg.layered(64, 4000, transient=20000),
              cg.ladder(20_000), cg.CONFIGS[4]()]
    for c in chains:
        t = [torch.from_numpy(a).to(dev) for a in (c.rp, c.col, c.val, c.goal)]
        sys_ = rp.rp_precompute(ctx, t[0], t[1], t[2], t[3], list(c.inst_off), 0, 0.0)
        x = torch.empty(c.n, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, info = rp.rp_scc(ctx, sys_)
        torch.cuda.synchronize()
        pt = {"workload": c.name, "states": c.n, "nnz": c.nnz, "decompose_ms": round(1000 * (time.perf_counter() - t0), 2),
              "scc": info}
        for name, fn in (("jacobi", lambda: rp.rp_jacobi(ctx, sys_, x, tol=1e-10, stop=B.RP_STOP_CERTIFIED)),
                         ("bicgstab", lambda: rp.rp_bicgstab(ctx, sys_, x, tol=1e-10, stop=B.RP_STOP_CERTIFIED)),
                         ("scc_solve", lambda: rp.rp_scc_solve(ctx, sys_, x, tol=1e-10, stop=B.RP_STOP_CERTIFIED))):
            fn()  # warm (layout tuning)
            ts, res = [], None
            for _ in range(steps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                res = fn()
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            info = res[1]
            pt[name] = {"ms": round(1000 * sorted(ts)[len(ts) // 2], 2), "status": B.STATUS_NAMES[res[2]],
                        "iterations_max": max(i["iterations"] for i in info)}
            if name == "scc_solve":
                pt[name]["levels"] = {k: res[3][k] for k in ("substitution_levels", "jacobi_levels",
                                                             "substitution_rows", "jacobi_rows", "jacobi_sweeps")}
        sys_.close()
        out.append(pt)
        log(f"scc {c.name}: decompose {pt['decompose_ms']} ms, jacobi {pt['jacobi']['ms']} ms, "
            f"bicgstab {pt['bicgstab']['ms']} ms, scc_solve {pt['scc_solve']['ms']} ms")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--workload", choices=list(WORKLOADS), default="batched_mixed_leaky",
                    help="; ".join(f"{k}: {v}" for k, v in WORKLOADS.items()).replace("%", "%%"))
    ap.add_argument("--tiling", choices=["auto", "off"], default="auto",
                    help="off: row-chunk kernels reading every operand from device memory (A/B runs)")
    ap.add_argument("--schedule", type=int, default=-1,
                    help="opts.schedule of every solve: -1 tuned (default), 0 sliced rows, 1..64 lanes per row "
                         "(the byte-counter runs fix the layout, since counter collection skews the tuner's timing)")
    ap.add_argument("--graph", type=int, default=0, choices=[0, 1],
                    help="opts.graph of every solve: 1 replays the tiled Jacobi batches as one captured HIP graph")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip the per-kernel event timing")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip what runs after the timed steps (unprofiled re-run, single-chain comparison, "
                         "accuracy check), e.g. to profile only the timed work")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB five times (scale reference for "
                         "the HBM byte counters) and exit")
    ap.add_argument("--section6", action="store_true",
                    help="only run the paper's own experiments (random diagonally dominant integer systems, "
                         "Jacobi against BiCGStab over density and size) and print them as one JSON line")
    ap.add_argument("--jacobi-variants", action="store_true",
                    help="only compare the Jacobi update rules and row-sum layouts (tiled, two-buffer chunks, "
                         "in place, segmented scan) on --workload and print them as one JSON line")
    ap.add_argument("--scc", action="store_true",
                    help="only compare the solve by strongly connected components with the ordinary solves on "
                         "chains of different component structure and print one JSON line")
    args = ap.parse_args()
    if args.scc:
        if args.gpus != 1:
            print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
            sys.exit(2)
        print(json.dumps({"experiment": "solve by strongly connected components vs whole-system solves, FP64 "
                                        "certified to 1e-10", "points": scc_compare()}), flush=True)
        return
    if args.jacobi_variants:
        if args.gpus != 1:
            print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
            sys.exit(2)
        chain = make_workload(args.workload, args.batch)
        print(json.dumps({"experiment": "Jacobi variants, FP64", "workload": chain.name, "states": chain.n,
                          "nnz": chain.nnz, "variants": jacobi_variants(chain)}), flush=True)
        return
    if args.section6:
        if args.gpus != 1:
            print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
            sys.exit(2)
        print(json.dumps({"experiment": "section 6: diagonally dominant integer A x = b, Jacobi vs BiCGStab, "
                                        "FP64 certified to 1e-10", "points": section6_sweep()}), flush=True)
        return
    if args.copy_calibration:
        import torch
        n = args.copy_calibration << 20
        a = torch.ones(n // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "copies": 5}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1210_6412_amd as rp
    from paper_1210_6412_amd import binding as B

    dev = torch.device("cuda", 0)
    chain = make_workload(args.workload, args.batch)
    tiling = B.RP_TILING_AUTO if args.tiling == "auto" else B.RP_TILING_OFF
    log(f"workload {chain.name}: n={chain.n} nnz={chain.nnz}")
    rowp = torch.from_numpy(chain.rp).to(dev)
    col = torch.from_numpy(chain.col).to(dev)
    val = torch.from_numpy(chain.val).to(dev)
    goal = torch.from_numpy(chain.goal).to(dev)
    off = [int(v) for v in chain.inst_off]
    cls = torch.empty(chain.n, dtype=torch.uint8, device=dev)
    ctx = rp.rp_context_create(0)
    x = torch.empty(chain.n, dtype=torch.float64, device=dev)
    # each solver's last solution, for the comparison with the oracle made in
    # the CPU-baseline leg
    xs = {r: torch.empty(chain.n, dtype=torch.float64, device=dev)
          for r in ("jacobi_fp64", "bicgstab_fp64", "jacobi_fp32r", "bicgstab_fp32r")}
    seed_v = torch.zeros(chain.n, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()

    rows = ["precompute", "jacobi_fp64", "bicgstab_fp64", "jacobi_fp32r", "bicgstab_fp32r", "adjoint"]

    def step(times):
        t = time.perf_counter()
        sys_ = rp.rp_precompute(ctx, rowp, col, val, goal, off, 0, 0.0, cls)
        times["precompute"] += time.perf_counter() - t
        results = {}
        for name, fn, prec in [("jacobi_fp64", rp.rp_jacobi, B.RP_FP64), ("bicgstab_fp64", rp.rp_bicgstab, B.RP_FP64),
                               ("jacobi_fp32r", rp.rp_jacobi, B.RP_FP32_REFINED),
                               ("bicgstab_fp32r", rp.rp_bicgstab, B.RP_FP32_REFINED)]:
            t = time.perf_counter()
            _, info, code = fn(ctx, sys_, xs[name], tol=1e-10, stop=B.RP_STOP_CERTIFIED, precision=prec,
                               tiling=tiling, schedule=args.schedule, graph=args.graph)
            times[name] += time.perf_counter() - t
            if code != B.RP_OK:
                raise RuntimeError(f"{name}: {B.STATUS_NAMES[code]} {rp.rp_last_error(ctx)}")
            results[name] = info
        t = time.perf_counter()
        _, _, info, code = rp.rp_adjoint(ctx, sys_, xs["bicgstab_fp32r"], seed_v, 1, tol=1e-10,
                                         stop=B.RP_STOP_CERTIFIED,
                                         precision=B.RP_FP32_REFINED, tiling=tiling, schedule=args.schedule,
                                         graph=args.graph)
        times["adjoint"] += time.perf_counter() - t
        if code != B.RP_OK:
            raise RuntimeError(f"adjoint: {B.STATUS_NAMES[code]} {rp.rp_last_error(ctx)}")
        results["adjoint"] = info
        sys_.close()
        return results

    # seed of the adjoint: first undecided state of every instance
    sys0 = rp.rp_precompute(ctx, rowp, col, val, goal, off, 0, 0.0, cls)
    c_h = cls.cpu().numpy()
    sv = np.zeros(chain.n)
    for k in range(chain.num_instances):
        lo, hi = chain.inst_off[k], chain.inst_off[k + 1]
        sq = np.nonzero(c_h[lo:hi] == 2)[0]
        if sq.size:
            sv[lo + sq[0]] = 1.0
    seed_v.copy_(torch.from_numpy(sv))
    sys0.close()

    for i in range(args.warmup):
        w = {r: 0.0 for r in rows}
        step(w)
        log(f"warmup {i} done ({sum(w.values()):.3f} s)")
    if not args.no_profile:
        rp.binding.rp_profile_enable(ctx, True)
    times = {r: 0.0 for r in rows}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = None
    for i in range(args.steps):
        last = step(times)
        log(f"step {i} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = rp.binding.rp_profile_read(ctx) if not args.no_profile else {}
    rp.binding.rp_profile_enable(ctx, False)

    solves_per_step = 5 * chain.num_instances
    value = solves_per_step * args.steps / elapsed

    out_extra = {}
    if not args.no_extras:
        out_extra = extras(args, chain, ctx, rows, step, times, seed_v, dev, rp, B, x, rowp, col, val, goal, off, cls)
    roof, kernels = roofline(prof, {k: v[0]["lanes"] for k, v in last.items()}, chain.name)

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1000 * elapsed / args.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": chain.name, "tiling": args.tiling, "graph": args.graph, "batch": chain.num_instances, "states": chain.n, "nnz": chain.nnz,
                   "tol": 1e-10, "stop": "certified max|x-x*|", "solves_per_step": solves_per_step},
        "rows_ms_per_step": {r: round(1000 * times[r] / args.steps, 3) for r in rows},
        "variant_solves_per_s": {r: round(chain.num_instances * args.steps / times[r], 2) for r in rows[1:]},
        "fp32r_over_fp64": {"jacobi": round(times["jacobi_fp64"] / times["jacobi_fp32r"], 3),
                            "bicgstab": round(times["bicgstab_fp64"] / times["bicgstab_fp32r"], 3)},
        "iterations_inst0": {k: v[0]["iterations"] for k, v in last.items()},
        "lanes_per_row": {k: v[0]["lanes"] for k, v in last.items()},
        "kernels": kernels,
        "iterations_per_s": {k: round(1000.0 * v["launches"] / v["ms"], 1) for k, v in kernels.items()
                             if k.startswith(("jacobi", "bicgstab")) and v["ms"] > 0},
        "roofline": roof,
    }
    out.update(out_extra)
    out["certified_error_bound_max"] = {k: max(i["error_bound"] for i in v) for k, v in last.items()}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(chain, gpu_x={k: v.cpu().numpy() for k, v in xs.items()})
    print(json.dumps(out), flush=True)


def sweep_kernel(kernel_id, lanes):
    """Name (prefix) of the Jacobi sweep kernel a solve ran, from its reported
    layout (0: sliced rows, L > 0: L lanes per row), as the profilers print it."""
    t = {"jacobi_fp64": "double", "jacobi_fp32": "float"}.get(kernel_id)
    if t is None or lanes is None:
        return None
    return f"rpk::k_jacobi_sliced<{t}," if lanes == 0 else f"rpk::k_jacobi_tile<{t}, {lanes}>"


def roofline(prof, layouts=None, workload=None):
    """Roofline entry for the kernel with the most time, from the library's
    event timing: algorithmic bytes / summed time over the timed steps.
    layouts: lanes reported per solve row (selects the kernel whose byte
    counters apply)."""
    if not prof:
        return None, {}
    kernels = {}
    for name, (n, ms, b) in prof.items():
        if n:
            kernels[name] = {"launches": n, "ms": round(ms, 3), "avg_us": round(1000 * ms / n, 3),
                             "alg_GBps": round(b / (ms * 1e6), 1) if ms > 0 else None}
    dom = max((k for k in prof if prof[k][0] and prof[k][2] > 0), key=lambda k: prof[k][1])
    n, ms, b = prof[dom]
    ach = b / (ms * 1e6)
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4),
            "traffic": pmc_traffic(dom, sweep_kernel(dom, (layouts or {}).get(
                {"jacobi_fp64": "jacobi_fp64", "jacobi_fp32": "jacobi_fp32r"}.get(dom, dom))), workload),
            "launches": n, "avg_launch_us": round(1000 * ms / n, 3), "alg_bytes_per_launch": b / n}
    return roof, kernels


def extras(args, chain, ctx, rows, step, times, seed_v, dev, rp, B, x, rowp, col, val, goal, off, cls):
    import torch
    # the same steps without the per-kernel event timing (its overhead)
    t1 = time.perf_counter()
    for i in range(args.steps):
        step({r: 0.0 for r in rows})
    torch.cuda.synchronize()
    unprof_ms = 1000 * (time.perf_counter() - t1) / args.steps
    log("unprofiled steps done")

    # one chain of the batch on its own: the batched-vs-single comparison
    c0 = chain.instance(0)
    s_rowp = torch.from_numpy(c0.rp).to(dev); s_col = torch.from_numpy(c0.col).to(dev)
    s_val = torch.from_numpy(c0.val).to(dev); s_goal = torch.from_numpy(c0.goal).to(dev)
    s_cls = torch.empty(c0.n, dtype=torch.uint8, device=dev)
    s_x = torch.empty(c0.n, dtype=torch.float64, device=dev)
    single = {r: 0.0 for r in rows}
    reps = 3
    for _ in range(reps):
        t = time.perf_counter()
        sy = rp.rp_precompute(ctx, s_rowp, s_col, s_val, s_goal, None, 0, 0.0, s_cls)
        single["precompute"] += time.perf_counter() - t
        for name, fn, prec in [("jacobi_fp64", rp.rp_jacobi, B.RP_FP64), ("bicgstab_fp64", rp.rp_bicgstab, B.RP_FP64),
                               ("jacobi_fp32r", rp.rp_jacobi, B.RP_FP32_REFINED),
                               ("bicgstab_fp32r", rp.rp_bicgstab, B.RP_FP32_REFINED)]:
            t = time.perf_counter()
            fn(ctx, sy, s_x, tol=1e-10, stop=B.RP_STOP_CERTIFIED, precision=prec)
            single[name] += time.perf_counter() - t
        t = time.perf_counter()
        rp.rp_adjoint(ctx, sy, s_x, seed_v[:c0.n].contiguous(), 1, tol=1e-10, stop=B.RP_STOP_CERTIFIED,
                      precision=B.RP_FP32_REFINED)
        single["adjoint"] += time.perf_counter() - t
        sy.close()
    single_sps = {r: round(reps / single[r], 2) for r in rows[1:]}
    log("single-chain comparison done")

    return {
        "ms_per_step_without_event_timing": round(unprof_ms, 3),
        "single_chain_solves_per_s": single_sps,
        "batched_over_single": {r: round(chain.num_instances * args.steps / times[r] / single_sps[r], 2)
                                for r in rows[1:]},
    }


if __name__ == "__main__":
    main()
