"""Throughput of the fast spectral collision hot path on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: the two-species 1-D-x Couette problem (masses 1 and 2, VHS omega
0.5/0.6/0.7, N = 32^3 velocity grid, S = 4, R = 8, icosahedron M = 12,
N_rho = 16, K = 16 DG elements of order P = 3, i.e. 64 spatial nodes,
diffuse walls at +-0.5, seeded 1% noise on unit Maxwellians).  One step is
one SSP-RK3 step (dt = 1e-3): three right-hand sides, each the DG transport
plus all 64 x 4 ordered-pair collision evaluations.  The metric is
collision evaluations per second (768 per step).  The plain FP64 path is
`value`; the FP32-mixed path with the FP64 conservation projection is
reported beside it.  Inputs are resident in HBM before timing starts.

Prints one JSON line (rank 0).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
# FP32 VALU without packed instructions (which this build does not emit):
# one FMA per lane per clock, 256 CUs x 64 lanes x 2 flops x 2.4 GHz
FP32_UNPACKED_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--workload", default="couette", choices=["couette", "vjp", "batched", "vss", "table1", "box2d"],
                    help="couette: the headline line (default); vjp: adjoint throughput, 2 species N = 32; "
                         "batched: 1024 uneven instances in one launch per stage vs per-instance launches; "
                         "vss: three-species VSS N = 48, M = 32, N_rho = 24; "
                         "table1: latency and 64-node throughput at the accuracy study's shapes; "
                         "box2d: one step of the 2-D box with the three-species VSS N = 48 collision term")
    ap.add_argument("--autotune", action="store_true",
                    help="run dgfs_autotune_rhs on each plan (the step's right-hand side) before timing; the chosen "
                         "schedule is reported")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy (reference for HBM byte counters)")
    ap.add_argument("--no-nosym", action="store_true",
                    help="skip the variant without the reuse of gain sums (its kernels carry the headline's "
                         "names, so a profile of the other variants leaves it out)")
    return ap.parse_args()


def copy_calibration():
    """A plain device-to-device copy of 256 MiB, 5 times: the per-dispatch
    FETCH_SIZE / WRITE_SIZE it shows under rocprofv3 --pmc calibrate the
    counters (expected 262144 KiB each)."""
    import torch
    n = 256 << 20
    src = torch.ones(n // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n, "dispatches": 5}))


def gain_yz_model(N, M, Nr, sigma_x, elt, gslots_pp, gslots_pq):
    """Algorithmic bytes and nominal flops of k_gain_yz per node.

    Bytes: every gain slot reads each distinct x-shifted array once (N^3
    complex each) and writes its N_rho arrays C_r.  A side has one array per
    (r, distinct sigma_x), except that a zero sigma_x gives one array for all
    r; with p == q on one input the second side reuses the first side's
    arrays of the opposite sigma_x.  gslots_pp / gslots_pq count the gain
    slots per node with p == q and p != q.
    Flops per direction term (5 n log2 n per complex length-n transform): two
    inverse 2-D transforms of every x-plane, two phase multiplies (6 flops per
    point each), product and weighted accumulation (8 flops per point); per
    (slot, r) one forward 2-D transform of the sum (added by the caller)."""
    n3 = N ** 3
    sc = 2 * elt
    vals = np.unique(np.round(np.asarray(sigma_x, dtype=float), 15))
    zero = int(np.sum(vals == 0.0))
    per_side = Nr * (len(vals) - zero) + zero
    unpaired = [v for v in vals if v != 0.0 and not np.any(vals == -v)]
    side1_shared = Nr * len(unpaired)
    arrays = gslots_pq * 2 * per_side + gslots_pp * (per_side + side1_shared)
    bytes_ = (arrays + (gslots_pp + gslots_pq) * Nr) * n3 * sc
    t2 = 5.0 * N * N * np.log2(N * N)  # per plane
    flops_term = N * (2 * t2 + (2 * 6 + 8) * N * N)
    flops_fwd = N * t2
    return bytes_, flops_term, flops_fwd


TRAFFIC_PROFILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "couette_n32_hbm_traffic.md")
KERNEL_SOURCES = ["collide_kernels.hpp", "fft.hpp", "collide.hip"]


def measured_path_bytes(prec="fp64"):
    """rocprofv3-measured HBM bytes per evaluation of the whole path (every
    kernel of a step, prec "fp64" or "fp32") from the committed summary, or
    None when the kernel sources changed since the counters were taken."""
    return measured_traffic(prec, key_prefix="path_bytes_per_eval ")


def measured_traffic(kernel, key_prefix="traffic_bytes "):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 --pmc
    summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when the
    kernel sources changed since the counters were taken."""
    import hashlib
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    h = hashlib.sha256()
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1903_04670_amd", "csrc")
    for f in KERNEL_SOURCES:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    vals = {}
    for line in text.splitlines():
        if line.startswith("source_sha256:"):
            vals["sha"] = line.split(":", 1)[1].strip()
        elif line.startswith(key_prefix):
            k, v = line.rsplit(":", 1)
            vals[k[len(key_prefix):].strip()] = float(v)
    if vals.get("sha") != h.hexdigest():
        return None
    for k, v in vals.items():
        if k == kernel or k.startswith(kernel):
            return v
    return None


def gain_schedule(cfg):
    """Gain slots per node of one mixture right-hand side, split into p == q
    and p != q, and the direction terms they sum: with an antipodal sphere set
    (octahedron, icosahedron), VHS pairs and a symmetric R, the (q, p) sums
    reuse (p, q)'s and the (p, p) sums run over half of the set; otherwise
    every ordered pair sums over all M directions."""
    ns, M = cfg["ns"], cfg["M"]
    R = np.asarray(cfg["R"])
    sym = (cfg["sphere"] in ("octahedron", "icosahedron") and np.all(np.asarray(cfg["alpha"]) == 1.0)
           and np.array_equal(R, R.T) and "DGFS_NO_SYMMETRY" not in os.environ)
    if not sym:
        return ns, ns * (ns - 1), ns * ns * M
    return ns, ns * (ns - 1) // 2, ns * (ns - 1) // 2 * M + ns * (M // 2)


def model_bytes_per_eval(N, M, Nr, elt):
    """Model bytes of one collision evaluation: one HBM round trip of an N^3
    complex intermediate per (r, m) term, plus three real N^3 arrays of I/O
    (the FP64 input pair and output)."""
    return 2 * (2 * elt) * N ** 3 * M * Nr + 3 * 8 * N ** 3


def gain_roofline(cfg, r, tname, elt, steps, evals_per_step, gpp, gpq, gterms, peak_tflops):
    """Roofline of k_gain_yz for one precision: algorithmic bytes and
    nominal flops per launch (gain_yz_model x the nodes one launch
    processes) over the event-timed average launch duration; `bound` is the
    larger of the HBM and VALU fractions."""
    name = "k_gain_yz"
    cnt, tot = r["kern"].get(name, (0, 0.0))
    if cnt == 0:
        raise RuntimeError("no gain-kernel launches were recorded")
    avg_ms = tot / cnt
    evals_per_launch = evals_per_step / (cnt / steps)
    nodes_per_launch = evals_per_launch / (cfg["ns"] * cfg["ns"])
    b, f_term, f_fwd = gain_yz_model(cfg["N"], cfg["M"], cfg["Nrho"], r["sigma_x"], elt, gpp, gpq)
    bytes_launch = b * nodes_per_launch
    flops_launch = (f_term * gterms + f_fwd * (gpp + gpq)) * cfg["Nrho"] * nodes_per_launch
    gbs = bytes_launch / (avg_ms / 1e3) / 1e9
    tf = flops_launch / (avg_ms / 1e3) / 1e12
    hbm_frac, alu_frac = gbs / HBM_PEAK_GBS, tf / peak_tflops
    if hbm_frac >= alu_frac:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(hbm_frac, 4)}
    else:
        roof = {"bound": "alu", "achieved": round(tf, 2), "peak": peak_tflops, "unit": "TFLOP/s",
                "frac": round(alu_frac, 4)}
    if cfg["N"] == 32:
        # one x-plane per wavefront, the two sides on its half-waves
        kname = "k_gain_yz_halves<%s, 32>" % tname
    else:
        groups = {("double", False): max(1, 128 // (2 * cfg["N"])), ("float", False): 1}
        kname = "%s<%s, %d, %d, %d, false>" % (name, tname, cfg["N"], groups[(tname, False)], 1 if elt == 8 else 2)
    roof.update({"traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                 "traffic": measured_traffic(kname), "kernel": kname, "avg_launch_ms": round(avg_ms, 4),
                 "evals_per_launch": evals_per_launch, "gain_slots_per_node": gpp + gpq,
                 "direction_terms_per_node": gterms, "algorithmic_bytes_per_launch": bytes_launch,
                 "nominal_flops_per_launch": flops_launch, "hbm_GBps": round(gbs, 1),
                 "hbm_frac": round(hbm_frac, 4), "fp_tflops": round(tf, 2), "alu_frac": round(alu_frac, 4)})
    return roof


def run(args):
    import torch
    from paper_1903_04670_amd import dgfs, workloads as wl

    cfg = wl.couette_two_species()
    dev = torch.device("cuda:0")
    F0 = torch.from_numpy(cfg["F"]).to(dev)
    mesh = dgfs.make_mesh(cfg["K"], u_left=cfg["u_left"], u_right=cfg["u_right"])
    n_nodes = F0.shape[0]
    evals_per_step = 3 * n_nodes * cfg["ns"] ** 2
    out = {}
    variants = [("fp64", False, False), ("fp32", False, False), ("fp64", True, False), ("fp32", True, False)]
    if not args.no_nosym:
        variants.append(("fp64", False, True))
    for prec, nyq, nosym in variants:
        # the last variant turns the reuse of gain sums off (every ordered pair
        # sums over all M directions): the rate of a workload without the
        # symmetry of this one
        if nosym:
            os.environ["DGFS_NO_SYMMETRY"] = "1"
        plan = dgfs.Plan(cfg["masses"], cfg["omega"], cfg["alpha"], cfg["N"], cfg["L"], cfg["Nrho"],
                         sphere=cfg["sphere"], M=cfg["M"], S=cfg["S"], R=cfg["R"], dg_order=cfg["P"],
                         precision=prec, nyquist_zero=nyq)
        project = prec == "fp32"
        F = F0.clone()
        sched = None
        if args.autotune:
            # tuned on the right-hand side this step runs (all pairs,
            # transport, the same projection flag)
            sched = dgfs.autotune_rhs(plan, F, mesh=mesh, project=project)
        ws = dgfs.workspace(plan, n_nodes, dgfs.OP_STEP, dev)
        stream = torch.cuda.current_stream()
        for _ in range(args.warmup):
            dgfs.step(plan, F, cfg["dt"], 1, mesh=mesh, project=project, ws=ws)
        torch.cuda.synchronize()
        # timed region: per-kernel HIP events on the library's launch stream
        dgfs.profile_enable(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(args.steps):
            dgfs.step(plan, F, cfg["dt"], 1, mesh=mesh, project=project, ws=ws)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kern = dgfs.profile_read()
        dgfs.profile_enable(False)
        gpu_ms = e0.elapsed_time(e1)
        ms = max(wall * 1e3, gpu_ms) / args.steps
        finite = bool(torch.isfinite(F).all())
        # graph-replay throughput (the production path) without kernel events
        for _ in range(args.warmup):
            dgfs.step(plan, F, cfg["dt"], 1, mesh=mesh, project=project, ws=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dgfs.step(plan, F, cfg["dt"], args.steps, mesh=mesh, project=project, ws=ws)
        torch.cuda.synchronize()
        ms_graph = (time.perf_counter() - t0) * 1e3 / args.steps
        out[prec + ("_nyq" if nyq else "") + ("_nosym" if nosym else "")] = dict(
            ms=ms, ms_graph=ms_graph, kern=kern, finite=finite, plan=plan, sigma_x=plan.sigma[:, 0].copy(),
            sched=sched)
        if nosym:
            del os.environ["DGFS_NO_SYMMETRY"]
    return cfg, evals_per_step, out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _time_oracle(plans, F, seconds, min_evals):
    """Ordered-pair evaluations of the oracle, cycling over nodes and pairs,
    until `seconds` have passed and at least `min_evals` were done."""
    from oracle.collide import collide
    pairs = list(plans)
    n = 0
    t0 = time.perf_counter()
    while True:
        node = n // len(pairs) % F.shape[0]
        p, q = pairs[n % len(pairs)]
        collide(plans[p, q], F[node, p], F[node, q])
        n += 1
        if time.perf_counter() - t0 > seconds and n >= min_evals:
            break
    return n, time.perf_counter() - t0


def cpu_baseline(seconds):
    """The oracle (as it stands) on the host's cores: ordered-pair
    evaluations of the Couette workload (N = 32, M = 12, N_rho = 16) for
    about `seconds` (the reported value), plus at least 3 evaluations of the
    space-homogeneous shape (N = 16, octahedron, N_rho = 8) and one of the
    precision workload's shape (N = 48, Fibonacci M = 32, N_rho = 24).  Plan
    tables (Algorithm 1) are built outside the timed regions; for the N = 48
    shape the table is built with alpha = 1, because the oracle's VSS
    Funk-Hecke table takes minutes at N_rho = 24 and the evaluation's
    arithmetic does not depend on the table's values."""
    from threadpoolctl import threadpool_info
    from oracle.collide import PairPlan
    from oracle.quadrature import sphere_set
    from paper_1903_04670_amd import workloads as wl

    def pair_plans(cfg, pairs, alpha=None):
        s, w = sphere_set(cfg["sphere"], cfg["M"])
        return {(p, q): PairPlan(cfg["N"], cfg["L"], cfg["masses"][p], cfg["masses"][q], cfg["omega"][p][q],
                                 cfg["alpha"][p][q] if alpha is None else alpha, cfg["Nrho"], s, w,
                                 R=cfg["R"][p][q]) for p, q in pairs}
    cfg2 = wl.couette_two_species(K=1, P=1)
    n2, t2 = _time_oracle(pair_plans(cfg2, [(p, q) for p in range(2) for q in range(2)]), cfg2["F"], seconds, 4)
    cfg1 = wl.homogeneous_single()
    n1, t1 = _time_oracle(pair_plans(cfg1, [(0, 0)]), cfg1["F"], 0.0, 3)
    cfg5 = wl.precision_vss(n_nodes=1)
    n5, t5 = _time_oracle(pair_plans(cfg5, [(0, 2)], alpha=1.0), cfg5["F"], 0.0, 1)
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    return dict(value=n2 / t2, unit="collision evals/s", cores=int(threads), kind="oracle",
                sample="%d ordered-pair evaluations (N=32, M=12, N_rho=16) of the Couette workload, %.1f s"
                       % (n2, t2),
                cpu_model=_cpu_model(), affinity_cores=len(os.sched_getaffinity(0)),
                other_shapes=[
                    {"shape": "N=16, octahedron M=6, N_rho=8 (space-homogeneous)", "evals": n1,
                     "seconds": round(t1, 3), "evals_per_s": round(n1 / t1, 3)},
                    {"shape": "N=48, Fibonacci M=32, N_rho=24, pair (1, 4) masses (precision workload)",
                     "evals": n5, "seconds": round(t5, 3), "evals_per_s": round(n5 / t5, 4)}])


def _time_cuda(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def bench_vjp(args):
    """Adjoint of Q^{pq} for the two species (masses 1, 2.5), N = 32,
    icosahedron, N_rho = 16: all four ordered pairs on 64 nodes per pass."""
    import torch
    from paper_1903_04670_amd import dgfs, workloads as wl
    cfg = wl.differentiation(n_nodes=64)
    plan = dgfs.Plan(cfg["masses"], cfg["omega"], cfg["alpha"], cfg["N"], cfg["L"], cfg["Nrho"],
                     sphere=cfg["sphere"], M=cfg["M"], R=cfg["R"])
    F = torch.from_numpy(cfg["F"]).cuda()
    W = torch.from_numpy(cfg["W"][:, 0]).cuda()
    fs = [F[:, p].contiguous() for p in range(2)]
    gf, gq = torch.empty_like(W), torch.empty_like(W)
    ws = dgfs.workspace(plan, 64, dgfs.OP_VJP)
    fws = dgfs.workspace(plan, 64, dgfs.OP_COLLIDE)
    out = torch.empty_like(W)

    def vjp_pass():
        for p in range(2):
            for q in range(2):
                dgfs.collide_vjp(plan, p, q, fs[p], fs[q], W, gf, gq, ws=ws)

    def fwd_pass():
        for p in range(2):
            for q in range(2):
                dgfs.collide(plan, p, q, fs[p], fs[q], out, ws=fws)
    tv = _time_cuda(vjp_pass, args.steps, args.warmup)
    tf = _time_cuda(fwd_pass, args.steps, args.warmup)
    dgfs.profile_enable(True)
    vjp_pass()
    torch.cuda.synchronize()
    kern = dgfs.profile_read()
    dgfs.profile_enable(False)
    ev = 4 * 64
    return {"metric": "adjoint (VJP) evaluations/s, 2 species N=32^3 M=12 N_rho=16 (FP64)",
            "value": round(ev / tv, 1), "unit": "VJP evals/s", "forward_evals_per_s": round(ev / tf, 1),
            "vjp_over_forward_time": round(tv / tf, 3),
            "kernels_ms_per_pass": {k: round(v[1], 3) for k, v in sorted(kern.items())},
            "n_gpus": 1, "steps": args.steps, "dtype": "f64",
            "data": "synthetic", "config": {"workload": cfg["name"], "nodes": 64, "pairs": 4}}


def bench_batched(args):
    """1024 space-homogeneous instances of uneven size (N in {16, 24, 32},
    1-3 species, N_rho in {8, 16}, icosahedron): every ordered pair of every
    instance through dgfs_collide_batched (one launch per stage per
    workspace chunk), with the descriptor array prepared once (dgfs.Batch)
    and built again per call, and once as one dgfs_collide call per item."""
    import torch
    from paper_1903_04670_amd import dgfs, workloads as wl
    insts = wl.batched_instances(n_inst=1024)
    plans, items = [], []
    for k, c in enumerate(insts):
        plans.append(dgfs.Plan(c["masses"], c["omega"], c["alpha"], c["N"], c["L"], c["Nrho"],
                               sphere=c["sphere"], M=c["M"], R=c["R"]))
        F = torch.from_numpy(c["F"]).cuda()
        for p in range(c["ns"]):
            for q in range(c["ns"]):
                items.append((k, p, q, F[:, p], F[:, q], torch.empty(F[:, p].shape, dtype=torch.float64, device="cuda")))
    batch = dgfs.Batch(plans, items)
    ws = batch.run()
    ws1 = torch.empty(max(pl.workspace_bytes(1) for pl in plans), dtype=torch.uint8, device="cuda")

    def batched():
        batch.run(ws=ws)

    def batched_rebuilt():
        # descriptor array built again on every call (dgfs.collide_batched)
        dgfs.collide_batched(plans, items, ws=ws)

    def single():
        for (k, p, q, fp, fq, out) in items:
            dgfs.collide(plans[k], p, q, fp, fq, out, ws=ws1)
    tb = _time_cuda(batched, args.steps, args.warmup)
    tr = _time_cuda(batched_rebuilt, args.steps, 1)
    ts = _time_cuda(single, max(1, args.steps // 2), 1)
    dgfs.profile_enable(True)
    batch.run(ws=ws)
    torch.cuda.synchronize()
    kern = {k: round(v[1], 3) for k, v in sorted(dgfs.profile_read().items())}
    dgfs.profile_enable(False)
    return {"metric": "collision evals/s, 1024 uneven space-homogeneous instances (FP64)",
            "value": round(len(items) / tb, 1), "unit": "collision evals/s",
            "descriptors_rebuilt_per_call_evals_per_s": round(len(items) / tr, 1),
            "per_instance_launches_evals_per_s": round(len(items) / ts, 1), "evals": len(items),
            "batched_ms": round(tb * 1e3, 3), "per_instance_ms": round(ts * 1e3, 3),
            "kernels_ms_per_call": kern, "n_gpus": 1,
            "dtype": "f64", "data": "synthetic", "config": {"workload": "1024 instances N in {16,24,32}"}}


def bench_vss(args):
    """Three species (masses 1, 2, 4), VSS alpha = 1.4, N = 48, Fibonacci
    M = 32, N_rho = 24; the mixture collision term of 4 nodes (36 ordered-pair
    evaluations) per pass, FP64 and FP32-mixed with the FP64 projection."""
    import torch
    from paper_1903_04670_amd import dgfs, workloads as wl
    cfg = wl.precision_vss(n_nodes=4)
    F = torch.from_numpy(cfg["F"]).cuda()
    res, kern = {}, {}
    for prec in ("fp64", "fp32"):
        plan = dgfs.Plan(cfg["masses"], cfg["omega"], cfg["alpha"], cfg["N"], cfg["L"], cfg["Nrho"],
                         sphere=cfg["sphere"], M=cfg["M"], R=cfg["R"], precision=prec)
        ws = dgfs.workspace(plan, 4, dgfs.OP_RHS)
        out = torch.empty_like(F)
        t = _time_cuda(lambda: dgfs.rhs(plan, F, out=out, project=(prec == "fp32"), ws=ws),
                       max(1, args.steps // 2), 1)
        res[prec] = 36 / t
        dgfs.profile_enable(True)
        dgfs.rhs(plan, F, out=out, project=(prec == "fp32"), ws=ws)
        torch.cuda.synchronize()
        kern[prec] = {k: round(v[1], 3) for k, v in sorted(dgfs.profile_read().items())}
        dgfs.profile_enable(False)
        del plan, ws
        torch.cuda.empty_cache()
    return {"metric": "collision evals/s, 3-species VSS N=48^3 M=32 N_rho=24", "value": round(res["fp64"], 1),
            "unit": "collision evals/s", "fp32_mixed": round(res["fp32"], 1),
            "kernels_ms_per_pass": kern, "n_gpus": 1, "dtype": "f64",
            "data": "synthetic", "config": {"workload": cfg["name"], "nodes": 4, "pairs": 9}}


def bench_box2d(args):
    """The precision workload's 2-D shape: 16 x 8 elements with P = 1 (512
    nodes) on the unit square, four diffuse walls, three species (masses 1,
    2, 4), VSS alpha = 1.4, N = 48, Fibonacci M = 32, N_rho = 24.  One
    forward-Euler step (the 2-D transport plus 512 x 9 collision
    evaluations) in FP32-mixed with the FP64 projection and in FP64."""
    import torch
    from paper_1903_04670_amd import dgfs, workloads as wl
    cfg = wl.precision_vss(n_nodes=512)
    F0 = torch.from_numpy(cfg["F"]).cuda()
    del cfg["F"]
    walls = {"left": ((0.0, -0.3, 0.0), 1.0), "right": ((0.0, 0.3, 0.0), 1.0),
             "bottom": ((0.2, 0.0, 0.0), 1.0), "top": ((-0.2, 0.0, 0.0), 1.0)}
    mesh = dgfs.make_mesh2d(16, 8, periodic=(False, False), walls=walls)
    res, kern = {}, {}
    for prec in ("fp32", "fp64"):
        plan = dgfs.Plan(cfg["masses"], cfg["omega"], cfg["alpha"], cfg["N"], cfg["L"], cfg["Nrho"],
                         sphere=cfg["sphere"], M=cfg["M"], R=cfg["R"], dg_order=1, precision=prec)
        ws = dgfs.workspace(plan, 512, dgfs.OP_STEP)
        F = F0.clone()
        project = prec == "fp32"
        t = _time_cuda(lambda: dgfs.step_2d(plan, F, 1e-4, mesh, project=project, euler=True, ws=ws), 1, 1)
        res[prec] = 512 * 9 / t
        dgfs.profile_enable(True)
        dgfs.step_2d(plan, F, 1e-4, mesh, project=project, euler=True, ws=ws)
        torch.cuda.synchronize()
        kern[prec] = {k: round(v[1], 3) for k, v in sorted(dgfs.profile_read().items())}
        dgfs.profile_enable(False)
        del plan, ws, F
        torch.cuda.empty_cache()
    return {"metric": "collision evals/s in a 2-D box step, 3-species VSS N=48^3 M=32 N_rho=24, 512 nodes",
            "value": round(res["fp64"], 1), "unit": "collision evals/s", "fp32_mixed": round(res["fp32"], 1),
            "kernels_ms_per_step": kern, "n_gpus": 1, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "2-D box 16x8 elements P=1, " + cfg["name"], "nodes": 512, "pairs": 9}}


# Table 1 cells whose P100 FP64 time per evaluation the paper prints
# (Sec. 3.2, Table 1): (N, N_rho, M, seconds).  Context only.
TABLE1_TIMES = [(16, 8, 6, 0.00056), (16, 8, 12, 0.00085), (24, 6, 12, 0.00114), (32, 8, 12, 0.00287),
                (32, 16, 12, 0.00541), (32, 32, 12, 0.01057), (48, 24, 12, 0.02556), (56, 56, 12, 0.09303)]


def bench_table1(args):
    """The accuracy study's shapes (equal masses, L = 12, constant kernel:
    omega = 1) in FP64: the latency of one evaluation (one node, one ordered
    pair, one call) and the throughput of 64 nodes in one call, beside the
    paper's printed time per evaluation on its GPU (another machine:
    context, not a target).  The input is a Maxwellian; the time does not
    depend on the values."""
    import numpy as np
    import torch
    from paper_1903_04670_amd import dgfs, workloads as wl
    rows = []
    for N, Nr, M, paper_s in TABLE1_TIMES:
        f = wl.maxwellian(N, 12.0, 1.0)
        plan = dgfs.Plan([1.0, 1.0], np.ones((2, 2)), np.ones((2, 2)), N, 12.0, Nr,
                         sphere="octahedron" if M == 6 else "icosahedron")
        one = torch.from_numpy(f[None]).cuda()
        many = one.expand(64, N, N, N).contiguous()
        ws1, ws64 = dgfs.workspace(plan, 1), dgfs.workspace(plan, 64)
        o1, o64 = torch.empty_like(one), torch.empty_like(many)
        t1 = _time_cuda(lambda: dgfs.collide(plan, 0, 1, one, one, out=o1, ws=ws1), 20, 3)
        t64 = _time_cuda(lambda: dgfs.collide(plan, 0, 1, many, many, out=o64, ws=ws64), 5, 1)
        rows.append({"N": N, "N_rho": Nr, "M": M, "latency_ms": round(t1 * 1e3, 4),
                     "evals_per_s_64_nodes": round(64 / t64, 1), "paper_ms_per_eval": paper_s * 1e3})
        del plan, ws1, ws64
        torch.cuda.empty_cache()
    return {"metric": "Table 1 shapes: latency of one evaluation and 64-node throughput (FP64)",
            "value": rows[4]["evals_per_s_64_nodes"], "unit": "collision evals/s (N=32, N_rho=16, M=12, 64 nodes)",
            "rows": rows, "n_gpus": 1, "dtype": "f64", "data": "synthetic (Maxwellian)",
            "config": {"workload": "accuracy-study shapes, equal masses, omega = 1, L = 12"}}


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.workload != "couette":
        if args.gpus != 1:
            print("bench.py measures one GPU only.", file=sys.stderr)
            sys.exit(2)
        fn = {"vjp": bench_vjp, "batched": bench_batched, "vss": bench_vss, "table1": bench_table1,
              "box2d": bench_box2d}[args.workload]
        print(json.dumps(fn(args)), flush=True)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the collision hot path is benchmarked on a single "
              "MI355X; sharding across GPUs is described in the design notes, not implemented.", file=sys.stderr)
        sys.exit(2)
    cfg, evals_per_step, res = run(args)
    r64, r32, rns = res["fp64"], res["fp32"], res.get("fp64_nosym")
    n64, n32 = res["fp64_nyq"], res["fp32_nyq"]
    value = evals_per_step / (r64["ms"] / 1e3)
    gpp, gpq, gterms = gain_schedule(cfg)
    roof = gain_roofline(cfg, r64, "double", 8, args.steps, evals_per_step, gpp, gpq, gterms, FP64_PEAK_TFLOPS)
    roof32 = gain_roofline(cfg, r32, "float", 4, args.steps, evals_per_step, gpp, gpq, gterms, FP32_PEAK_TFLOPS)
    roof32["issue_ceiling_tflops"] = FP32_UNPACKED_TFLOPS
    roof32["issue_ceiling_frac"] = round(roof32["fp_tflops"] / FP32_UNPACKED_TFLOPS, 4)
    value32 = evals_per_step / (r32["ms"] / 1e3)
    path = {}
    for prec, v in (("fp64", value), ("fp32", value32)):
        b = measured_path_bytes(prec)
        path[prec] = None if b is None else {"bytes_per_eval": b, "GBps": round(v * b / 1e9, 1),
                                             "frac": round(v * b / (HBM_PEAK_GBS * 1e9), 4)}
    line = {
        "metric": "collision evals/s at N=32^3 (FP64; FP32-mixed beside it)",
        "value": round(value, 1),
        "unit": "collision evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r64["ms"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "couette 2 species N=32 M=12 Nrho=16 K=16 P=3 (64 nodes), SSP-RK3 step",
                   "evals_per_step": evals_per_step, "nodes": 64, "pairs": 4},
        "fp32_mixed": {"value": round(value32, 1), "ms_per_step": round(r32["ms"], 3),
                       "projection": "fp64", "dtype": "f32 transforms, f64 moments/projection"},
        "graph_replay": {"fp64_evals_per_s": round(evals_per_step / (r64["ms_graph"] / 1e3), 1),
                         "fp32_mixed_evals_per_s": round(evals_per_step / (r32["ms_graph"] / 1e3), 1)},
        "kernels_ms_per_step": {k: round(v[1] / args.steps, 4) for k, v in sorted(r64["kern"].items())},
        "kernels_ms_per_step_fp32": {k: round(v[1] / args.steps, 4) for k, v in sorted(r32["kern"].items())},
        "roofline": roof,
        "roofline_fp32_mixed": roof32,
        "path_hbm": {
            "what": "whole path (every kernel of a step): rocprofv3-measured HBM bytes per evaluation "
                    "(FETCH_SIZE + WRITE_SIZE, copy-calibrated) x evals/s, against 8 TB/s; null when the "
                    "kernels changed since the counters were taken",
            "fp64": path["fp64"], "fp32_mixed": path["fp32"]},
        "model_equivalent": {
            "what": "not a roofline fraction: the HBM rate a per-term cost model (one HBM round trip of an "
                    "N^3 complex intermediate per (r, m) term plus three real N^3 arrays) would need for the "
                    "measured evals/s; this design moves fewer bytes (sum over m before the forward transform, "
                    "shared x-shifted arrays, reused gain sums), see path_hbm",
            "bytes_per_eval_fp64": model_bytes_per_eval(cfg["N"], cfg["M"], cfg["Nrho"], 8),
            "bytes_per_eval_fp32_mixed": model_bytes_per_eval(cfg["N"], cfg["M"], cfg["Nrho"], 4),
            "fp64_TBps": round(value * model_bytes_per_eval(cfg["N"], cfg["M"], cfg["Nrho"], 8) / 1e12, 3),
            "fp32_mixed_TBps": round(value32 * model_bytes_per_eval(cfg["N"], cfg["M"], cfg["Nrho"], 4) / 1e12,
                                     3)},
        "no_symmetry": None if rns is None else {
            "what": "FP64 step with the reuse of gain sums turned off: every ordered pair sums over all "
                    "M = 12 directions (48 direction terms per node instead of 24); the rate of a workload "
                    "without this one's antipodal sphere set and equal R_pq = R_qp",
            "fp64_evals_per_s": round(evals_per_step / (rns["ms"] / 1e3), 1),
            "graph_replay_fp64_evals_per_s": round(evals_per_step / (rns["ms_graph"] / 1e3), 1),
            "direction_terms_per_node": cfg["ns"] * cfg["ns"] * cfg["M"]},
        "nyquist_zero": {
            "what": "variant operator, not the headline: the gain's translates drop the Nyquist planes of "
                    "fft(f), so u1, u2 are real and one complex transform gives both (real-packed k_gain_yz)",
            "fp64_evals_per_s": round(evals_per_step / (n64["ms"] / 1e3), 1),
            "fp32_mixed_evals_per_s": round(evals_per_step / (n32["ms"] / 1e3), 1),
            "graph_replay": {"fp64_evals_per_s": round(evals_per_step / (n64["ms_graph"] / 1e3), 1),
                             "fp32_mixed_evals_per_s": round(evals_per_step / (n32["ms_graph"] / 1e3), 1)},
            "k_gain_yz_avg_launch_ms": {
                "fp64": round(n64["kern"]["k_gain_yz"][1] / max(n64["kern"]["k_gain_yz"][0], 1), 4),
                "fp32_mixed": round(n32["kern"]["k_gain_yz"][1] / max(n32["kern"]["k_gain_yz"][0], 1), 4)},
            "kernels_ms_per_step": {k: round(v[1] / args.steps, 4) for k, v in sorted(n64["kern"].items())},
            "kernels_ms_per_step_fp32": {k: round(v[1] / args.steps, 4) for k, v in sorted(n32["kern"].items())}},
        "finite": all(r["finite"] for r in res.values()),
        "schedule": ("default" if not args.autotune else
                     {k: dict(zip(("chunk_evals", "shift_split", "gain_x_fuse"), v["sched"])) for k, v in res.items()}),
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
