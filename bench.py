"""Benchmark: WoS toolbox build throughput on one MI355X.

A step is one complete pass of the hot path over one batch of synthetic
input: a toolbox build (cell weights lambda, the walks of every (site, walk)
pair binned into A, B, H, K, normalisation) followed by its direct
application to the boundary data g = x^2 - y^2 (u = A 0 + H g,
grad u = B 0 + K g).  Each step uses a new seed.  `value` is walk-steps per
second over the whole step, inputs resident in HBM.

Workload (default): the largest single-GPU configuration, the 3-D unit cube
minus the ball of radius 0.3 about its centre: 32768 uniform interior sites,
8192 boundary nodes (6936 face-cell midpoints on the cube, 1256 Fibonacci
points on the sphere), 1e5 walks per site, eps = 1e-5, FP32 walker (its rows
exceed LDS: the windowed tally mode).

The line also carries "serving": solves/s and p50/p99 latency of served
streams of Dirichlet problems on resident L-shape toolboxes (256/1024/4096
sites), every request with its own seeded coefficients, mixed precision
against FP64, with the L2 errors of both against the manufactured
solutions, and "newton_ball4096": the 3-D unit-ball toolbox build and a
regularised Newton solve of -Lap u + u^3 = f, mixed precision against FP64,
and "el_plaplace": Adam on the discrete p-Laplace functional (the paper's
disk p-torsion example), and "el_energies": the paper's semilinear example
(Adam and p-HiSD saddle points) and its example "elliptic div min".

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline] [--no-serving]

Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import re
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "WoS walk-steps/s (toolbox build)"  # the served-solve rates are reported under "serving"
MI355X_CUS = 256
MI355X_CLOCK = 2.4e9
# FP32 vector peak 157.3 TFLOP/s = 256 CU x 128 FMA lanes x 2.4 GHz: 7.86e13
# full-rate lane-ops/s (one FMA = one lane-op).  Measured on gfx950: plain
# (non-packed) FP32 and INT32 VALU ops issue at 128 lanes/clk/CU, FP64 FMA,
# v_mul_hi at 64, transcendentals and 32x32->64 multiplies at 32.
LANE_OPS_PEAK = MI355X_CUS * 128 * MI355X_CLOCK
BF16_PEAK_TFLOPS = 2500.0  # dense BF16 matrix-core peak
# Algorithmic lane-op budget of the walker (slots: full-rate op = 1,
# transcendental / 32-bit integer multiply = 4), per walk-step and per walk
# (the per-step and per-walk counts of the method: distance, tally point,
# nearest-centre scan, tally weights, direction, move, Philox words).
WALKER_BUDGET = {  # (C_step, C_walk) by workload geometry
    "disk": (113, 450), "square": (113, 450), "lshape": (187, 450), "ball": (216, 700), "cubeball": (228, 700),
}


def walker_source_hash():
    h = hashlib.sha256()
    for f in ("walker.hip", "walker_impl.hpp", "walker_f32_2d.hip", "walker_f32_3d.hip", "wos_device.hpp",
              "wos_types.hpp", "grid.cpp"):
        with open(os.path.join(ROOT, "paper_2608_07017_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, walk_steps):
    """HBM bytes of one walker launch of `walk_steps` walk-steps, from the
    committed FETCH_SIZE / WRITE_SIZE summary of this workload (bytes per
    walk-step), or None when the walker source has changed since the
    counters were taken (or no summary exists)."""
    path = os.path.join(ROOT, "profiles", "walker_%s.md" % workload)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    h = re.search(r"sha256/16\): `([0-9a-f]+)`", text)
    t = re.search(r"walker_traffic_bytes_per_walk_step = ([0-9.eE+]+)", text)
    if not h or not t or h.group(1) != walker_source_hash():
        return None
    return float(t.group(1)) * walk_steps


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cubeball32768")
    ap.add_argument("--walks", type=int, default=0, help="override the workload's walks per site (profiling runs)")
    ap.add_argument("--no-autotune", action="store_true", help="workgroup size by occupancy, no timing pass")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-walks", type=int, default=0,
                    help="walks of the oracle's sample per site (0: sized for about 5 s per site)")
    ap.add_argument("--cpu-procs", type=int, default=0, help="processes of the all-core oracle run (0: the CPU share)")
    ap.add_argument("--no-cpu-solves", action="store_true", help="skip the numpy FP64 solve baseline")
    ap.add_argument("--probe", action="store_true", help="also report the VALU issue-rate probe")
    ap.add_argument("--minimal-surface", action="store_true", help="also run the minimal surface energies")
    ap.add_argument("--no-serving", action="store_true", help="skip the served-solve stream")
    ap.add_argument("--no-bf16", action="store_true", help="skip the BF16 shadows, applies and products")
    ap.add_argument("--no-newton", action="store_true", help="skip the 3-D Newton run")
    ap.add_argument("--newton-iters", type=int, default=10)
    ap.add_argument("--no-el", action="store_true", help="skip the Euler-Lagrange (Adam) runs")
    ap.add_argument("--el-walks", type=int, default=100000)
    ap.add_argument("--el-max-iter", type=int, default=20000)
    ap.add_argument("--el-rate-iters", type=int, default=100)
    ap.add_argument("--el-conv-iters", type=int, default=20000)
    ap.add_argument("--hisd-max-iter", type=int, default=40000)
    ap.add_argument("--newton-rcond", type=float, default=1e-2)
    ap.add_argument("--serve-requests", type=int, default=10000, help="requests of each open-loop mixed run")
    ap.add_argument("--serve-saturation", type=int, default=2000, help="requests of the saturation run")
    ap.add_argument("--serve-f64-requests", type=int, default=2000, help="requests of the FP64 open-loop run")
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-problems", type=int, default=400, help="distinct seeded problems per toolbox")
    ap.add_argument("--serve-rho", default="0.5,0.8,0.95")
    ap.add_argument("--serve-rcond", type=float, default=0.1)
    ap.add_argument("--serve-seed", type=int, default=7)
    ap.add_argument("--serve-op-requests", type=int, default=20000,
                    help="requests of each prepared-operator run")
    ap.add_argument("--cubeball", action="store_true",
                    help="also build the 3-D cube-minus-ball toolbox (32768 sites, 1e5 walks/site; about "
                         "a minute) and solve the quasilinear problem on it by Picard")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after the timed steps, copy a MIB-sized device buffer 3 times (a known-size "
                         "kernel for scaling the FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


def geometry_key(name):
    for k in ("disk", "square", "lshape", "ball", "cubeball"):
        if name.startswith(k):
            return k
    return "square"


def _oracle_site_sample(job):
    """One bounded sample of the oracle (run in a child process): `walks`
    walks of site i of the named workload, binned.  Returns (walk-steps, s)."""
    name, i, walks = job
    import workloads as W
    from oracle.walker import site_events, bin_site
    c = W.config(name)
    t0 = time.perf_counter()
    ev = site_events(c["domain"], c["sites"][i], i, np.arange(walks), c["eps"], c["seed"])
    bin_site(ev, c["sites"], c["bnodes"])
    return int(ev.nsteps.sum()), time.perf_counter() - t0


def _host_cpu():
    model = ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in out.splitlines():
            if ln.startswith("Model name:"):
                model = ln.split(":", 1)[1].strip()
    except Exception:
        pass
    try:
        share = len(os.sched_getaffinity(0))
    except AttributeError:
        share = os.cpu_count() or 1
    return model, os.cpu_count(), share


def cpu_baseline(name, walks, procs):
    """The oracle, as it stands, on a bounded sample of the same workload:
    `walks` walks of whole sites (the oracle's rate per walk-step does not
    depend on the sample size), once in one process (one thread: NumPy's
    element-wise kernels), then `procs` sites at once in as many processes.
    Rates in walk-steps/s."""
    import multiprocessing as mp
    model, ncpu, share = _host_cpu()
    steps1, dt1 = _oracle_site_sample((name, 0, walks))
    ctx = mp.get_context("spawn")
    jobs = [(name, 1 + k, walks) for k in range(procs)]
    t0 = time.perf_counter()
    with ctx.Pool(procs) as pool:
        res = pool.map(_oracle_site_sample, jobs)
    dtn = time.perf_counter() - t0
    stepsn = sum(r[0] for r in res)
    return {"value": stepsn / dtn, "unit": "walk-steps/s", "cores": procs, "kind": "oracle",
            "sample": "%d sites x %d walks of the same workload in %d processes (%d walk-steps, %.1f s wall); FP64 "
                      "NumPy oracle, brute-force nearest centre" % (procs, walks, procs, stepsn, dtn),
            "single_thread": {"value": steps1 / dt1, "sample": "1 site x %d walks (%d walk-steps, %.1f s)"
                                                               % (walks, steps1, dt1)},
            "host": {"lscpu_model": model, "os_cpu_count": ncpu, "affinity": share}}


def cpu_solve_baseline():
    """numpy/LAPACK FP64 solves of eq. linear_q by the oracle (Tikhonov,
    the generalised inverse the served route uses) on toolboxes of the
    served sizes (d = 2, p = n / 4; random matrices: the time does not depend
    on their values), BLAS threads as the environment sets them."""
    from oracle import linalg as OL
    rng = np.random.default_rng(3)
    out = {"threads": os.environ.get("OMP_NUM_THREADS", "default")}
    for n, reps in ((256, 10), (1024, 3), (4096, 1)):
        p, d = n // 4, 2
        tb = {"A": rng.random((n, n)), "B": rng.normal(size=(d, n, n)), "H": rng.random((n, p)),
              "K": rng.normal(size=(d, n, p))}
        lam = rng.random(n) / n
        M = rng.normal(size=(n, d, d))
        Ac = M @ M.transpose(0, 2, 1) + np.eye(d)
        bc = rng.normal(size=(n, d))
        f, g = rng.normal(size=n), rng.normal(size=p)
        t0 = time.perf_counter()
        for _ in range(reps):
            OL.solve_linear(tb, lam, f, g, Acoef=Ac, bcoef=bc, rcond=0.1, solver="tikhonov")
        dt = (time.perf_counter() - t0) / reps
        out[str(n)] = {"solves_per_s": 1.0 / dt, "ms_per_solve": 1e3 * dt}
    return out


SERVE_SIZES = (256, 1024, 4096)


def serving(a, torch, W, P):
    """Served streams on resident L-shape toolboxes: -div(A grad u) + b . grad u = f
    with A anisotropic (up to 1:100) and b smooth, solved by the Tikhonov route
    in mixed precision and in FP64.  Every request carries its own seeded
    coefficient fields and data (serve_problems distinct problems per
    toolbox; nothing is cached between requests).  Saturation rate (all
    requests queued at once), then Poisson arrivals at rho times that rate
    for each rho; latency = finish - arrival.  Every mixed result is checked
    against its problem's FP64 plain solve: L2 error against u_ex within
    1.01 times the FP64 one plus 1e-6.  The prepared-operator route is
    reported for a stream that shares coefficients (one set per toolbox, a
    new right-hand side per request)."""
    rng = np.random.default_rng(a.serve_seed)
    rhos = [float(r) for r in str(a.serve_rho).split(",")]
    boxes = []
    print("serving: toolboxes and %d problems per toolbox" % a.serve_problems, file=sys.stderr, flush=True)
    for n in SERVE_SIZES:
        cfg = W.config("lshape%d" % n)
        tb = P.Toolbox(cfg["domain"], cfg["sites"], cfg["bnodes"], cfg["walks"], cfg["eps"], seed=cfg["seed"],
                       precision="f32")
        tb.build()
        lam = torch.as_tensor(tb.export("lambda"), dtype=torch.float64)
        probs = []
        for k in range(a.serve_problems):
            pr = W.anisotropic_problem(a.serve_seed * 100000 + 1000 * (n // 256) + k, cfg["sites"], cfg["bnodes"])
            dev = {key: torch.as_tensor(v, dtype=torch.float64, device="cuda").contiguous()
                   for key, v in (("f", -pr["f"]), ("g", pr["g"]), ("A", pr["A"]), ("b", -pr["b"]), ("u", pr["u"]))}
            probs.append(dev)
        boxes.append((tb, lam, probs))
    torch.cuda.synchronize()

    def kw(dev, prec):
        return dict(kind="linear", A=dev["A"], b=dev["b"], rcond=a.serve_rcond, solver="tikhonov", precision=prec,
                    refine_tol=1e-8)

    def l2(lam, u, dev):
        return float(torch.sqrt(torch.sum(lam * (u - dev["u"]) ** 2)))

    # the FP64 plain solve of every problem: its L2 error is the bar each
    # served mixed result must reach
    print("serving: FP64 reference solves", file=sys.stderr, flush=True)
    sv = P.Server(slots=a.serve_slots)
    pend = [[sv.submit(tb, dev["f"], dev["g"], **kw(dev, "f64")) for dev in probs] for tb, _, probs in boxes]
    ref_err = []
    for (tb, lam, probs), row in zip(boxes, pend):
        ref_err.append([])
        for dev, (tk, u, _) in zip(probs, row):
            sv.poll(tk)
            ref_err[-1].append(l2(lam, u, dev))
    sv.close()

    def run(prec, nreq, rate, check=False):
        sv = P.Server(slots=a.serve_slots)
        for tb, lam, probs in boxes:  # warm every workspace
            sv.poll(sv.submit(tb, probs[0]["f"], probs[0]["g"], **kw(probs[0], prec))[0])
        picks = [(int(rng.integers(len(boxes))), int(rng.integers(a.serve_problems))) for _ in range(nreq)]
        gaps = rng.exponential(1.0 / rate, nreq) if rate else np.zeros(nreq)
        arrivals = np.cumsum(gaps)
        tickets = []
        t0 = time.perf_counter()
        for (bi, pi), ta in zip(picks, arrivals):
            while time.perf_counter() - t0 < ta:
                pass
            tb, lam, probs = boxes[bi]
            dev = probs[pi]
            tk, u, _ = sv.submit(tb, dev["f"], dev["g"], **kw(dev, prec))
            tickets.append((tk, u))
        res = [sv.poll(tk) for tk, _ in tickets]
        sv.close()
        times = [r[1] for r in res]
        first = min(t[0] for t in times)
        last = max(t[2] for t in times)
        lat = np.array([t[2] - t[0] for t in times]) * 1e3
        out = {"requests": nreq, "solves_per_s": nreq / (last - first), "p50_ms": float(np.percentile(lat, 50)),
               "p99_ms": float(np.percentile(lat, 99))}
        if check:
            ok = 0
            for (bi, pi), (_, u) in zip(picks, tickets):
                tb, lam, probs = boxes[bi]
                ok += l2(lam, u, probs[pi]) <= 1.01 * ref_err[bi][pi] + 1e-6
            out["at_fp64_l2_error"] = ok / nreq
        return out

    out = {"workload": "L-shape toolboxes of %s sites (n/4 boundary nodes, 1e4 walks/site, eps 1e-4, FP32), "
                       "requests uniform over them and over %d seeded problems per toolbox: -div(A grad u) + "
                       "b.grad u = f, A smooth SPD with anisotropy up to 1:100, |b| <= 0.8, manufactured u; "
                       "Tikhonov rcond %g" % ("/".join(map(str, SERVE_SIZES)), a.serve_problems, a.serve_rcond),
           "slots": a.serve_slots,
           "l2_error_f64": {str(tb.n): float(np.mean(e)) for (tb, _, _), e in zip(boxes, ref_err)}}
    print("serving: mixed saturation", file=sys.stderr, flush=True)
    sat = run("mixed", a.serve_saturation, 0.0, check=True)
    out["mixed"] = {"saturation": sat, "open_loop": []}
    for rho in rhos:
        print("serving: mixed open loop rho %g" % rho, file=sys.stderr, flush=True)
        rate = rho * sat["solves_per_s"]
        out["mixed"]["open_loop"].append(dict(run("mixed", a.serve_requests, rate, check=True), rho=rho,
                                              arrival_rate=rate))
    print("serving: BF16 saturation and open loop", file=sys.stderr, flush=True)
    for tb, _, _ in boxes:
        tb.make_bf16()
    torch.cuda.synchronize()
    satb = run("bf16", a.serve_saturation, 0.0, check=True)
    out["bf16"] = {"saturation": satb,
                   "open_loop": [dict(run("bf16", a.serve_requests, 0.8 * satb["solves_per_s"], check=True), rho=0.8,
                                      arrival_rate=0.8 * satb["solves_per_s"])]}
    print("serving: FP64 saturation and open loop", file=sys.stderr, flush=True)
    sat64 = run("f64", max(200, a.serve_saturation // 4), 0.0)
    rho = 0.8
    out["f64"] = {"saturation": sat64,
                  "open_loop": [dict(run("f64", a.serve_f64_requests, rho * sat64["solves_per_s"]), rho=rho,
                                     arrival_rate=rho * sat64["solves_per_s"])]}
    out["mixed_vs_f64_saturation"] = sat["solves_per_s"] / sat64["solves_per_s"]
    out["bf16_vs_f64_saturation"] = satb["solves_per_s"] / sat64["solves_per_s"]
    out["bf16_at_fp64_l2_error"] = min([satb["at_fp64_l2_error"]] +
                                       [r["at_fp64_l2_error"] for r in out["bf16"]["open_loop"]])
    out["mixed_at_fp64_l2_error"] = min([sat["at_fp64_l2_error"]] +
                                        [r["at_fp64_l2_error"] for r in out["mixed"]["open_loop"]])

    # a stream that shares coefficients: one prepared solution operator per
    # toolbox (FP32 storage), a new right-hand side per request; queued
    # requests on one operator are batched
    print("serving: preparing operators", file=sys.stderr, flush=True)
    ops, prep_ms, op_l2 = [], {}, {}
    for tb, lam, probs in boxes:
        dev = probs[0]
        op = tb.operator(A=dev["A"], b=dev["b"], rcond=a.serve_rcond, storage="f32")
        ops.append(op)
        prep_ms[str(tb.n)] = op.info()["prep_ms"]
        u, _ = op.apply(dev["f"], dev["g"])
        op_l2[str(tb.n)] = l2(lam, u, dev)
    rhs = []
    for (tb, lam, probs) in boxes:
        rhs.append([(torch.randn(tb.n, dtype=torch.float64, device="cuda"),
                     torch.randn(tb.p, dtype=torch.float64, device="cuda")) for _ in range(64)])

    def run_op(nreq, rate):
        sv = P.Server(slots=a.serve_slots, max_batch=64)
        picks = [(int(rng.integers(len(boxes))), int(rng.integers(64))) for _ in range(nreq)]
        gaps = rng.exponential(1.0 / rate, nreq) if rate else np.zeros(nreq)
        arrivals = np.cumsum(gaps)
        tickets = []
        t0 = time.perf_counter()
        for (bi, pi), ta in zip(picks, arrivals):
            while time.perf_counter() - t0 < ta:
                pass
            f, g = rhs[bi][pi]
            tickets.append(sv.submit_op(ops[bi], f, g)[0])
        times = [sv.poll(t)[1] for t in tickets]
        sv.close()
        first = min(t[0] for t in times)
        last = max(t[2] for t in times)
        lat = np.array([t[2] - t[0] for t in times]) * 1e3
        return {"requests": nreq, "solves_per_s": nreq / (last - first), "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99))}

    print("serving: operator saturation", file=sys.stderr, flush=True)
    sat = run_op(a.serve_op_requests, 0.0)
    rate = 0.8 * sat["solves_per_s"]
    out["operator_f32_shared_coefficients"] = {
        "prep_ms": prep_ms, "l2_error": op_l2, "saturation_solves_per_s": sat["solves_per_s"],
        "open_loop": dict(run_op(a.serve_op_requests, rate), rho=0.8, arrival_rate=rate)}
    for op in ops:
        op.free()
    for tb, _, _ in boxes:
        tb.free()
    return out


def bf16_products(torch, P):
    """The BF16 matrix-core product of the BF16 route (C = X Y^T, FP32
    accumulation) at the assembly shapes of the 4096-site 3-D ball (4096 x
    4096 from K = 4 x 4096) and of a 8192-site problem, in TFLOP/s against
    the dense BF16 peak, timed with HIP events on the launch stream."""
    out = []
    for M, K in ((4096, 4 * 4096), (8192, 4 * 8192)):
        X = torch.randn(M, K, device="cuda").bfloat16()
        Y = torch.randn(M, K, device="cuda").bfloat16()
        C = torch.empty(M, M, device="cuda")
        P.gemm_bf16_nt(X, Y, C)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 10
        e0.record()
        for _ in range(reps):
            P.gemm_bf16_nt(X, Y, C)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        tf = 2.0 * M * M * K / (ms * 1e-3) / 1e12
        out.append({"M": M, "N": M, "K": K, "ms": ms, "tflops": tf, "frac_of_bf16_peak": tf / BF16_PEAK_TFLOPS})
        del X, Y, C
    torch.cuda.empty_cache()
    return out


def bf16_applies(torch, tb, g):
    """BF16 shadows of the headline toolbox: their size and making time, and
    the direct application u = A fbar + H g, grad u = B fbar + K g from the
    FP32 toolbox and from the shadows (HBM-bound: the shadows are half the
    bytes), with the relative difference of the two."""
    fbar = torch.randn(tb.m, dtype=torch.float64, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    tb.make_bf16()
    e1.record()
    torch.cuda.synchronize()
    make_ms = e0.elapsed_time(e1)
    res = {}
    for name, fn in (("f32", lambda: tb.apply(fbar, g)), ("bf16", lambda: tb.apply_bf16(fbar, g))):
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(5):
            u, gu = fn()
        e1.record()
        torch.cuda.synchronize()
        res[name] = (e0.elapsed_time(e1) / 5, u, gu)
    d, n, m, p = tb.dim, tb.n, tb.m, tb.p
    rel = lambda a, b: float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
    return {"shadow_gib": 2.0 * (d + 1) * n * (m + p) / 2 ** 30, "make_bf16_ms": make_ms,
            "apply_f32_ms": res["f32"][0], "apply_bf16_ms": res["bf16"][0],
            "apply_bytes_f32": 4.0 * (d + 1) * n * (m + p), "apply_bytes_bf16": 2.0 * (d + 1) * n * (m + p),
            "bf16_vs_f32_rel_diff_u": rel(res["bf16"][1], res["f32"][1]),
            "bf16_vs_f32_rel_diff_grad_u": rel(res["bf16"][2], res["f32"][2])}


def picard_cubeball(a, torch, W, P):
    """The 3-D unit cube minus the ball of radius 0.3 (32768 sites, 8192
    boundary nodes, 1e5 walks/site, eps 1e-5, FP32 tallies written straight to
    HBM) and Picard for -div((1 + u^2) grad u) = f with a seeded manufactured
    solution, Tikhonov steps in mixed precision and in FP64."""
    cfg = W.config("cubeball32768")
    x, z = cfg["sites"], cfg["bnodes"]
    tb = P.Toolbox(cfg["domain"], x, z, cfg["walks"], cfg["eps"], seed=cfg["seed"], precision="f32", autotune=False)
    tb.set_timing(True)
    print("cubeball: build", file=sys.stderr, flush=True)
    tb.build()
    t = tb.timings()
    inf = tb.info()
    lam = tb.export("lambda").cpu().numpy()
    ue, ge, le = W.smooth_field(2026, 3, terms=8, max_freq=2.0, scale=0.5)
    u0, g0 = ue(x), ge(x)
    f = -(1 + u0 ** 2) * le(x) - 2 * u0 * np.sum(g0 * g0, axis=1)
    g = ue(z)
    nrm = float(np.sqrt(np.sum(lam * u0 ** 2)))
    out = {"workload": cfg["label"] + "; -div((1 + u^2) grad u) = f, Picard (3 steps), Tikhonov rcond 1e-2",
           "walker_ms": t["walker_ms"], "walk_steps": inf["walk_steps"],
           "walk_steps_per_s": inf["walk_steps"] / (t["walker_ms"] * 1e-3), "device_gib": inf["device_bytes"] / 2**30}
    tb.make_bf16()
    for prec in ("bf16", "mixed", "f64"):
        print("cubeball: picard", prec, file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u, _, _, info = tb.solve(f, g, kind="quasilinear", rcond=1e-2, tol=1e-300, max_iter=3, solver="tikhonov",
                                 precision=prec, refine_tol=1e-8)
        torch.cuda.synchronize()
        out[prec] = {"seconds": time.perf_counter() - t0, "refine_converged": info["refine_converged"],
                     "rel_l2_error": float(np.sqrt(np.sum(lam * (u.cpu().numpy() - u0) ** 2))) / nrm}
        us = out.setdefault("_u", {})
        us[prec] = u.cpu().numpy()
    us = out.pop("_u")
    for prec in ("bf16", "mixed"):
        out[prec + "_vs_f64_rel_diff_u"] = float(np.sqrt(np.sum(lam * (us[prec] - us["f64"]) ** 2)
                                                         / np.sum(lam * us["f64"] ** 2)))
    out["mixed_vs_f64"] = out["f64"]["seconds"] / out["mixed"]["seconds"]
    out["bf16_vs_f64"] = out["f64"]["seconds"] / out["bf16"]["seconds"]
    tb.free()
    return out


def newton_ball(a, torch, W, P):
    """The 3-D unit ball toolbox (4096 sites, 1024 Fibonacci nodes, 1e4
    walks/site, eps 1e-4, FP32) and Newton for -Lap u + u^3 = f with a seeded
    manufactured solution, regularised steps in mixed precision and in FP64."""
    cfg = W.config("ball4096")
    x, z = cfg["sites"], cfg["bnodes"]
    tb = P.Toolbox(cfg["domain"], x, z, cfg["walks"], cfg["eps"], seed=cfg["seed"], precision="f32")
    tb.set_timing(True)
    tb.build()
    tb.build(seed=cfg["seed"] + 1)
    t = tb.timings()
    inf = tb.info()
    lam = tb.export("lambda").cpu().numpy()
    ue, _, le = W.smooth_field(2026, 3, terms=8, max_freq=3.0, scale=0.5)
    f, g = -le(x) + ue(x) ** 3, ue(z)
    nrm = float(np.sqrt(np.sum(lam * ue(x) ** 2)))
    out = {"workload": "3D unit ball, 4096 sites, 1024 Fibonacci boundary nodes, 1e4 walks/site, eps 1e-4, FP32; "
                       "-Lap u + u^3 = f, Newton (%d steps), Tikhonov rcond %g" % (a.newton_iters, a.newton_rcond),
           "walker_ms": t["walker_ms"], "walk_steps_per_s": inf["walk_steps"] / (t["walker_ms"] * 1e-3)}
    us = {}
    for prec in ("f64", "mixed"):
        tb.solve(f, g, kind="semilinear_cubic", rcond=a.newton_rcond, tol=1e-300, max_iter=1, solver="tikhonov",
                 precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u, _, _, info = tb.solve(f, g, kind="semilinear_cubic", rcond=a.newton_rcond, tol=1e-300,
                                 max_iter=a.newton_iters, solver="tikhonov", precision=prec, refine_tol=1e-10,
                                 max_refine=30)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        us[prec] = u.cpu().numpy()
        out[prec] = {"seconds": dt, "grad_norm_rel": info["grad_norm"] / info["grad_norm0"],
                     "refine_converged": info["refine_converged"],
                     "rel_l2_error": float(np.sqrt(np.sum(lam * (us[prec] - ue(x)) ** 2))) / nrm}
    # the mixed route's result against the FP64 route's (same regularised
    # system, refined to 1e-8 or better)
    out["mixed_vs_f64_rel_diff_u"] = float(np.sqrt(np.sum(lam * (us["mixed"] - us["f64"]) ** 2)
                                               / np.sum(lam * us["f64"] ** 2)))
    out["mixed_vs_f64"] = out["f64"]["seconds"] / out["mixed"]["seconds"]
    return out


def el_plaplace(a, torch, W, P):
    """Euler-Lagrange route: Adam on the discrete p-Laplace functional.

    (1) The paper's p-torsion example on the unit disk (its ring layout: 300
    sites, 60 boundary nodes; 1e5 walks/site, eps 1e-4, FP32 toolbox),
    f = 1, g = 0, Adam with the paper's fbar_0 = 1 and step sizes, run until
    the gradient norm reaches the paper's final values (1e-5 for P <= 2,
    5e-6 otherwise, in absolute cell measures; divided here by sqrt(|D|) for
    the normalised weights), checked every 50 iterations; relative L2 error
    against the closed form.  (2) The iteration rate on the 4096-site
    L-shape toolbox (FP32), where each iteration streams B twice (grad u
    forward, grad J back; the A and K terms are constants of the
    iteration): achieved bytes / s against HBM."""
    sites, bn = W.paper_disk_layout()
    tb = P.Toolbox(W.unit_disk(), sites, bn, a.el_walks, 1e-4, seed=11, precision="f32", volume_samples=1 << 20)
    tb.build()
    torch.cuda.synchronize()
    lam = tb.export("lambda").cpu().numpy()
    rows = {}
    for Pexp, alpha, paper_norm in ((1.5, 1e-3, 1e-5), (2.0, 1e-3, 1e-5), (5.0, 1e-2, 5e-6), (10.0, 1e-2, 5e-6),
                                    (50.0, 1e-1, 5e-6)):
        tol = paper_norm / np.sqrt(np.pi)
        u, _, _, info = tb.minimize(np.ones(tb.n), np.zeros(tb.p), Pexp, alpha, a.el_max_iter, fbar0=1.0, tol=tol,
                                    check_every=50)
        ex = W.plaplace_torsion_disk_exact(sites, Pexp)
        err = float(np.sqrt(np.sum(lam * (u.cpu().numpy() - ex) ** 2)) / np.sqrt(np.sum(lam * ex ** 2)))
        rows["P=%g" % Pexp] = {"alpha": alpha, "iters": info["iters"], "seconds": info["seconds"],
                               "iters_per_s": info["iters"] / info["seconds"], "grad_norm": info["grad_norm"],
                               "tol": tol, "J": info["J"], "rel_l2_error": err}
    # the same small problem is launch-bound: the iterations launch by
    # launch against blocks of 64 replayed from one captured HIP graph
    rate = {}
    for graph in (False, True):
        tb.minimize(np.ones(tb.n), np.zeros(tb.p), 2.0, 1e-3, 128, graph=graph)
        _, _, fb, info = tb.minimize(np.ones(tb.n), np.zeros(tb.p), 2.0, 1e-3, 20000, graph=graph)
        rate["graph" if graph else "eager"] = {"iters": info["iters"], "iters_per_s": info["iters"] / info["seconds"],
                                               "J": info["J"]}
    rate["graph_speedup"] = rate["graph"]["iters_per_s"] / rate["eager"]["iters_per_s"]
    rate["same_result"] = rate["graph"]["J"] == rate["eager"]["J"]
    tb.free()
    out = {"workload": "paper disk p-torsion: 300 ring sites, 60 nodes, %g walks/site, eps 1e-4, FP32; Adam "
                       "(beta 0.9/0.999, eps 1e-10, fbar_0 = 1) to the paper's gradient norms" % a.el_walks,
           "disk": rows, "disk_P2_iteration_rate": rate}
    # run on to 20000 iterations (near the minimiser of J): with W = V the
    # minimiser is far from the closed form; with a finer W partition (1200
    # ring sites) for the same 300 V cells it is not
    wfine = []
    for k in range(1, 21):
        th = 2 * np.pi * np.arange(6 * k - 3) / (6 * k - 3)
        wfine.append(np.stack([(k - 0.5) / 20 * np.cos(th), (k - 0.5) / 20 * np.sin(th)], 1))
    wfine = np.concatenate(wfine)
    conv = {}
    for label, wsites, vc in (("W=V=300", sites, None), ("W=1200,V=300", wfine, sites)):
        tb = P.Toolbox(W.unit_disk(), wsites, bn, a.el_walks, 1e-4, seed=11, precision="f32",
                       volume_samples=1 << 20, vcentres=vc)
        tb.build()
        lam = tb.export("lambda").cpu().numpy()
        conv[label] = {}
        for Pexp, alpha in ((1.5, 1e-3), (2.0, 1e-3), (5.0, 1e-2)):
            u, _, _, info = tb.minimize(np.ones(tb.n), np.zeros(tb.p), Pexp, alpha, a.el_conv_iters, fbar0=1.0)
            ex = W.plaplace_torsion_disk_exact(wsites, Pexp)
            conv[label]["P=%g" % Pexp] = float(np.sqrt(np.sum(lam * (u.cpu().numpy() - ex) ** 2))
                                               / np.sqrt(np.sum(lam * ex ** 2)))
        tb.free()
    out["disk_%d_iters_rel_l2_error" % a.el_conv_iters] = conv
    cfg = W.config("lshape4096")
    tb = P.Toolbox(cfg["domain"], cfg["sites"], cfg["bnodes"], 1000, cfg["eps"], seed=cfg["seed"], precision="f32")
    tb.build()
    torch.cuda.synchronize()
    n, p, d = tb.n, tb.p, tb.dim
    f, g = np.ones(n), np.zeros(p)
    tb.minimize(f, g, 2.0, 1e-3, 5)
    _, _, _, info = tb.minimize(f, g, 2.0, 1e-3, a.el_rate_iters)
    per_iter = info["seconds"] / info["iters"]
    # an iteration streams B (d n x m, FP32) twice: B fbar, then B^T yB; the
    # A and K terms of the gradient are constants of the iteration
    bytes_iter = 2.0 * d * n * n * 4
    out["lshape4096"] = {"iters": info["iters"], "us_per_iter": per_iter * 1e6,
                         "B_bytes_per_iter": bytes_iter, "achieved_GBps": bytes_iter / per_iter / 1e9,
                         "hbm_frac": bytes_iter / per_iter / 8e12}
    tb.free()
    return out


def el_energies(a, torch, W, P):
    """The other energies of the Euler-Lagrange route.  (1) Minimal surface
    on the unit square with Scherk's boundary values, u = ln(cos k(y - 1/2)
    / cos k(x - 1/2)) / k at k = 2.5, against that closed form (the harmonic
    function with the same boundary values is reported beside it); (2) the
    semilinear Lap u + u^2 = f with u* = sin(pi x) sin(pi y) against u*.
    Both on W = 48 x 48, V = 24 x 24 cell centres, 160 boundary nodes,
    el_walks walks/site, FP32, Adam run to a gradient norm of 1e-9 (checked
    every 100 iterations).  (3) The paper's minimal surface example on the
    disk (g = 0.3 sin 5 phi; no closed form: J is the graph's area over
    |D|) and its semilinear example with s = 800 on its 20 x 20 square
    layout, with its Adam parameters (fbar_0 = 1, alpha 0.01 and 1) to its
    final gradient norm 1e-6, and that example's index-1 and index-2 saddle
    points by p-HiSD with its parameters (k = 1, 2, 3), also at s = 8000; and its example "elliptic div
    min" on the disk layout against the closed form.  (4) The semilinear iteration rate on the 4096-site L-shape
    toolbox, which streams A and B twice each."""
    def grid(k):
        t = (np.arange(k) + 0.5) / k
        return np.stack(np.meshgrid(t, t, indexing="ij"), -1).reshape(-1, 2)
    out = {"workload": "the paper's examples: semilinear (s = 800, 8000) on its 20 x 20 square layout, Adam and "
                       "p-HiSD; elliptic div min on its disk layout; %g walks/site, eps 1e-4, FP32" % a.el_walks}
    if a.minimal_surface:
        sw, sv, bn = grid(48), grid(24), W.square_nodes(40)
        tb = P.Toolbox(W.unit_square(), sw, bn, a.el_walks, 1e-4, seed=17, precision="f32", volume_samples=1 << 20,
                       vcentres=sv)
        tb.build()
        torch.cuda.synchronize()
        lam = tb.export("lambda").cpu().numpy()
        H = tb.export("H").cpu().numpy().astype(np.float64)
        err = lambda u, ex: float(np.sqrt(np.sum(lam * (u - ex) ** 2) / np.sum(lam * ex ** 2)))
        k = 2.5
        scherk = lambda x: np.log(np.cos(k * (x[:, 1] - 0.5)) / np.cos(k * (x[:, 0] - 0.5))) / k
        u, _, _, info = tb.minimize(np.zeros(tb.n), scherk(bn), 0.0, 0.01, a.el_max_iter, fbar0=0.0,
                                    energy="minimal_surface", tol=1e-9, check_every=100)
        out["minimal_surface_scherk"] = {"k": k, "alpha": 0.01, "iters": info["iters"], "seconds": info["seconds"],
                                         "grad_norm": info["grad_norm"],
                                         "rel_l2_error": err(u.cpu().numpy(), scherk(sw)),
                                         "harmonic_rel_l2_error": err(H @ scherk(bn), scherk(sw))}
        ex = np.sin(np.pi * sw[:, 0]) * np.sin(np.pi * sw[:, 1])
        u, _, _, info = tb.minimize(-2 * np.pi ** 2 * ex + ex ** 2, np.zeros(tb.p), 0.0, 0.1, a.el_max_iter,
                                    fbar0=0.0, energy="semilinear", tol=1e-9, check_every=100)
        out["semilinear_sin"] = {"alpha": 0.1, "iters": info["iters"], "seconds": info["seconds"],
                                 "grad_norm": info["grad_norm"], "rel_l2_error": err(u.cpu().numpy(), ex)}
        tb.free()
        sites, bnd = W.paper_disk_layout()
        tb = P.Toolbox(W.unit_disk(), sites, bnd, a.el_walks, 1e-4, seed=11, precision="f32", volume_samples=1 << 20)
        tb.build()
        phi = np.arctan2(bnd[:, 1], bnd[:, 0])
        u, _, _, info = tb.minimize(np.zeros(tb.n), 0.3 * np.sin(5 * phi), 0.0, 0.01, a.el_max_iter, fbar0=1.0,
                                    energy="minimal_surface", tol=1e-6 / np.sqrt(np.pi), check_every=50)
        out["minimal_surface_disk_paper"] = {"alpha": 0.01, "fbar0": 1.0, "iters": info["iters"],
                                             "seconds": info["seconds"], "grad_norm": info["grad_norm"],
                                             "J_area_over_D": info["J"], "u_range": [float(u.min()), float(u.max())]}
        tb.free()
    # the example "elliptic div min" on the disk layout, with its Adam
    # parameters (fbar_0 = 0.1, alpha = 0.01) to its final norm 1e-4
    sites, bnd = W.paper_disk_layout()
    tb = P.Toolbox(W.unit_disk(), sites, bnd, a.el_walks, 1e-4, seed=11, precision="f32", volume_samples=1 << 20)
    tb.build()
    lam = tb.export("lambda").cpu().numpy()
    ue, _, fe = W.elliptic_divmin_disk(sites)
    cA, cc, cw = W.elliptic_divmin_coef(sites)
    u, _, _, info = tb.minimize(fe, np.zeros(tb.p), 0.0, 0.01, a.el_max_iter, fbar0=0.1, energy="elliptic",
                                coef_A=cA, coef_c=cc, coef_w=cw, tol=1e-4 / np.sqrt(np.pi), check_every=50)
    out["elliptic_divmin_disk_paper"] = {
        "alpha": 0.01, "fbar0": 0.1, "iters": info["iters"], "seconds": info["seconds"],
        "grad_norm": info["grad_norm"],
        "rel_l2_error": float(np.sqrt(np.sum(lam * (u.cpu().numpy() - ue) ** 2) / np.sum(lam * ue ** 2)))}
    tb.free()
    # the same with a finer W partition (1200 ring sites) for the paper's 300
    # V cells, run to el_conv_iters iterations (near the minimiser of J)
    wfine = np.concatenate([np.stack([(k - 0.5) / 20 * np.cos(2 * np.pi * np.arange(6 * k - 3) / (6 * k - 3)),
                                      (k - 0.5) / 20 * np.sin(2 * np.pi * np.arange(6 * k - 3) / (6 * k - 3))], 1)
                            for k in range(1, 21)])
    tb = P.Toolbox(W.unit_disk(), wfine, bnd, a.el_walks, 1e-4, seed=11, precision="f32", volume_samples=1 << 20,
                   vcentres=sites)
    tb.build()
    lam = tb.export("lambda").cpu().numpy()
    ue, _, fe = W.elliptic_divmin_disk(wfine)
    cA, cc, cw = W.elliptic_divmin_coef(wfine)
    u, _, _, info = tb.minimize(fe, np.zeros(tb.p), 0.0, 0.01, a.el_conv_iters, fbar0=0.1, energy="elliptic",
                                coef_A=cA, coef_c=cc, coef_w=cw)
    out["elliptic_divmin_disk_W1200_V300"] = {
        "iters": info["iters"], "seconds": info["seconds"], "grad_norm": info["grad_norm"],
        "rel_l2_error": float(np.sqrt(np.sum(lam * (u.cpu().numpy() - ue) ** 2) / np.sum(lam * ue ** 2)))}
    tb.free()
    sites, bnd = W.paper_square_layout()
    tb = P.Toolbox(W.unit_square(), sites, bnd, a.el_walks, 1e-4, seed=11, precision="f32", volume_samples=1 << 20)
    tb.build()
    f = 800.0 * np.sin(np.pi * sites[:, 0]) * np.sin(np.pi * sites[:, 1])
    u, _, _, info = tb.minimize(f, np.zeros(tb.p), 0.0, 1.0, a.el_max_iter, fbar0=1.0, energy="semilinear",
                                tol=1e-6, check_every=50)
    out["semilinear_s800_square_paper"] = {"alpha": 1.0, "fbar0": 1.0, "iters": info["iters"],
                                           "seconds": info["seconds"], "grad_norm": info["grad_norm"],
                                           "J": info["J"], "u_range": [float(u.min()), float(u.max())]}
    # the same example's saddle points by p-HiSD with the paper's parameters
    # (M = A, fbar_0 = 1000, eta = 20, tau = 10, directions from the Hessian)
    for k in (1, 2, 3):
        u, _, _, _, info = tb.saddle(f, np.zeros(tb.p), k, 20.0, 10.0, a.hisd_max_iter, fbar0=1000.0, precond="A",
                                     tol=1e-6, check_every=50, graph=True)
        out["semilinear_s800_phisd_k%d" % k] = {
            "iters": info["iters"], "seconds": info["seconds"], "ms_per_iter": 1e3 * info["seconds"] / info["iters"],
            "grad_norm": info["grad_norm"], "J": info["J"], "u_range": [float(u.min()), float(u.max())],
            "newton_schulz_iters": info["ns_iters"], "newton_schulz_residual": info["ns_residual"]}
    # the iteration rate launch by launch against blocks replayed from one
    # captured graph (k = 2, a fixed 4000 iterations; the same bits)
    rate = {}
    for graph in (False, True):
        _, _, fbg, _, info = tb.saddle(f, np.zeros(tb.p), 2, 20.0, 10.0, 4000, fbar0=1000.0, precond="A",
                                       graph=graph)
        rate["graph" if graph else "eager"] = {"ms_per_iter": 1e3 * info["seconds"] / info["iters"], "J": info["J"]}
    rate["graph_speedup"] = rate["eager"]["ms_per_iter"] / rate["graph"]["ms_per_iter"]
    rate["same_result"] = rate["graph"]["J"] == rate["eager"]["J"]
    out["semilinear_s800_phisd_k2_iteration_rate"] = rate
    tb.free()
    # s = 8000: the runs of the paper's parameter table (Adam, p-HiSD of
    # index 1..8 from fbar_0 = 1000 at eta 20, 5, 80, and restarts from the
    # dips of the (k, eta) = (4, 20), (5, 20), (5, 5), (6, 20) runs), on the
    # toolbox of its square layout with its walk parameters (N = 1e7, M = 30
    # steps), solutions counted modulo the square's symmetries
    from paper_2608_07017_amd import search as S
    tb = P.Toolbox(W.unit_square(), sites, bnd, 10 ** 7, 0.0, seed=11, precision="f32", fixed_M=30,
                   volume_samples=1 << 22)
    tb.build()
    f = 8000.0 * np.sin(np.pi * sites[:, 0]) * np.sin(np.pi * sites[:, 1])
    t0 = time.perf_counter()
    runs = S.semilinear_s8000_table(tb, f, np.zeros(tb.p), a.hisd_max_iter, 1e-6)
    keep = S.distinct(runs, S.square_symmetries(sites))
    out["semilinear_s8000_search"] = {
        "toolbox": "paper square layout, 1e7 walks/site, M = 30 steps, FP32",
        "seconds": time.perf_counter() - t0, "max_iter": a.hisd_max_iter, "tol": 1e-6,
        "distinct_solutions": len(keep), "paper_distinct_solutions": 22,
        "runs": [{"k": r["k"], "eta": r["eta"], "start": r["start"], "iters": r["iters"], "converged": r["converged"],
                  "grad_norm": r["grad_norm"], "J": r["J"], "distinct": i in keep, "error": r.get("error"),
                  "u_range": None if r["u"] is None else [float(np.min(r["u"])), float(np.max(r["u"]))]}
                 for i, r in enumerate(runs)]}
    tb.free()
    cfg = W.config("lshape4096")
    tb = P.Toolbox(cfg["domain"], cfg["sites"], cfg["bnodes"], 1000, cfg["eps"], seed=cfg["seed"], precision="f32")
    tb.build()
    torch.cuda.synchronize()
    n, d = tb.n, tb.dim
    f, g = np.ones(n), np.zeros(tb.p)
    tb.minimize(f, g, 0.0, 1e-3, 5, fbar0=0.0, energy="semilinear")
    _, _, _, info = tb.minimize(f, g, 0.0, 1e-3, a.el_rate_iters, fbar0=0.0, energy="semilinear")
    per_iter = info["seconds"] / info["iters"]
    bytes_iter = 2.0 * (d + 1) * n * n * 4  # A and B (FP32), forward and transposed
    out["lshape4096_semilinear"] = {"iters": info["iters"], "us_per_iter": per_iter * 1e6,
                                    "AB_bytes_per_iter": bytes_iter, "achieved_GBps": bytes_iter / per_iter / 1e9,
                                    "hbm_frac": bytes_iter / per_iter / 8e12}
    tb.free()
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only: several GPUs would each build the rows of their own "
              "share of the sites, and no multi-GPU launch is provided; use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads as W
    import paper_2608_07017_amd as P

    cfg = W.config(a.workload)
    if a.walks:
        cfg["walks"] = a.walks
        cfg["label"] = cfg["label"] + " (walks/site overridden: %d)" % a.walks
    prec = cfg["precision"]
    print("headline: creating the %s toolbox" % a.workload, file=sys.stderr, flush=True)
    tb = P.Toolbox(cfg["domain"], cfg["sites"], cfg["bnodes"], cfg["walks"], cfg["eps"], seed=cfg["seed"],
                   precision=prec, autotune=not a.no_autotune)
    plan = P.build_plan(cfg["domain"], cfg["sites"], cfg["bnodes"], cfg["walks"], cfg["eps"], precision=prec)
    bn = cfg["bnodes"]
    g = torch.tensor(bn[:, 0] ** 2 - bn[:, 1] ** 2, dtype=torch.float64, device="cuda")
    zero = torch.zeros(len(cfg["sites"]), dtype=torch.float64, device="cuda")
    # HIP events around the walker launch on its own stream (the library's
    # timing records), read after each step
    tb.set_timing(True)

    def step(k):
        tb.build(seed=cfg["seed"] + 1000 + k)
        return tb.apply(zero, g)

    for k in range(a.warmup):
        print("headline: warm-up step %d" % k, file=sys.stderr, flush=True)
        step(k)
    torch.cuda.synchronize()
    kernel_ms, finalize_ms, walk_steps, walks = [], [], [], []
    t0 = time.perf_counter()
    for k in range(a.steps):
        step(a.warmup + k)
        t = tb.timings()
        inf = tb.info()
        kernel_ms.append(t["walker_ms"])
        finalize_ms.append(t["finalize_ms"])
        walk_steps.append(inf["walk_steps"])
        walks.append(inf["walks"])
        print("headline: step %d walker %.1f ms" % (k, t["walker_ms"]), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    total_steps = float(np.sum(walk_steps))
    elapsed = t1 - t0
    value = total_steps / elapsed
    u, gu = step(a.warmup + a.steps)
    torch.cuda.synchronize()
    exact = cfg["sites"][:, 0] ** 2 - cfg["sites"][:, 1] ** 2
    herr = float(np.sqrt(np.mean((u.cpu().numpy() - exact) ** 2)))
    bf16 = None if a.no_bf16 else bf16_applies(torch, tb, g)
    tb.free()
    del tb
    torch.cuda.empty_cache()

    c_step, c_walk = WALKER_BUDGET[geometry_key(a.workload)]
    mean_steps = total_steps / a.steps
    mean_walks = float(np.mean(walks))
    walker_s = float(np.mean(kernel_ms)) * 1e-3
    alg_ops = c_step * mean_steps + c_walk * mean_walks
    achieved = alg_ops / walker_s / 1e12
    peak = LANE_OPS_PEAK / 1e12
    out = {
        "metric": METRIC, "value": value, "unit": "walk-steps/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": 1e3 * elapsed / a.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": prec, "data": "synthetic",
        "config": {"workload": cfg["label"], "sites": len(cfg["sites"]), "bnodes": len(bn),
                   "walks_per_site": cfg["walks"], "eps": cfg["eps"], "seed": cfg["seed"]},
        "walker": {"kernel_ms": float(np.mean(kernel_ms)), "walk_steps_per_s": mean_steps / walker_s,
                   "walk_steps_per_build": mean_steps, "walks_per_build": mean_walks,
                   "column_permutation_ms": float(np.mean(finalize_ms)),
                   "tally_mode": plan["tally_mode"], "window_pages": plan["window_pages"],
                   "window_bpages": plan["window_bpages"], "harmonic_extension_rms_err": herr},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tlane-op/s",
                     "frac": achieved / peak, "traffic": measured_traffic(a.workload, mean_steps),
                     "budget": {"per_walk_step": c_step, "per_walk": c_walk}},
    }
    if bf16 is not None:
        bf16["products"] = bf16_products(torch, P)
        out["bf16"] = bf16
    if a.probe:
        out["valu_probe_lane_ops_per_s"] = {op: P.probe_valu(op) for op in P.PROBE_OPS}
    if a.calibrate_copy > 0:
        src = torch.ones(a.calibrate_copy * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = src.numel() * 4
    if not a.no_serving:
        out["serving"] = serving(a, torch, W, P)
    if not a.no_newton:
        print("newton: ball4096", file=sys.stderr, flush=True)
        out["newton_ball4096"] = newton_ball(a, torch, W, P)
    if a.cubeball:
        out["picard_cubeball32768"] = picard_cubeball(a, torch, W, P)
    if not a.no_el:
        print("euler-lagrange: disk p-torsion, lshape4096", file=sys.stderr, flush=True)
        out["el_plaplace"] = el_plaplace(a, torch, W, P)
        print("euler-lagrange: semilinear and elliptic examples", file=sys.stderr, flush=True)
        out["el_energies"] = el_energies(a, torch, W, P)
    if not a.no_cpu_baseline:
        print("cpu baseline: the oracle", file=sys.stderr, flush=True)
        _, _, share = _host_cpu()
        procs = a.cpu_procs or max(1, min(16, share))
        walks = a.cpu_walks or (512 if len(cfg["sites"]) > 8192 else min(cfg["walks"], 4000))
        out["cpu_baseline"] = cpu_baseline(a.workload, walks, procs)
        if not a.no_cpu_solves:
            print("cpu baseline: numpy solves", file=sys.stderr, flush=True)
            out["cpu_baseline"]["solves"] = cpu_solve_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
