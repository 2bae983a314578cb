"""Benchmark of the NSFR hot path on one MI355X.

Workload (one "step"): one full right-hand-side evaluation nsfr_rhs -- the
entropy-conserving two-point volume flux differencing, the surface fluxes and
the weight-adjusted inverse of the FR-modified mass with c = c_HU, writing
dU/dt -- of the inviscid Taylor-Green vortex on a 16^3-element periodic box
warped by the paper's nonsymmetric map (beta = 1/5), p = 3 LGL, Mach 0.1, FP64.
State, metric terms and output are resident in HBM.

value = DOF-updates per second per right-hand side = nodes * K / t, with t the
HIP-event time of K back-to-back nsfr_rhs launches on the launching stream.

Also reported:
  * roofline: the stage kernel (one launch per rhs) against the HBM roof,
    160 algorithmic bytes per node (U 40 + metric columns 72 + 1/(W J) 8 +
    dU/dt 40) over the average launch time of the timed region; the HBM bytes
    measured with rocprofv3 counters on the same kernel source (null once the
    source changed); the FP64 VALU rate from rocprofv3 instruction counters;
  * extra: the median per-launch rhs time (>= 200 launches after 20 warm-ups)
    for p = 3, 4, 5 on 16^3 and on the HBM-resident 32^3 mesh; the RK4 step
    (four fused stage launches from a HIP graph); the adjoint: t_vjp / t_rhs
    at c = 0 and c = c_HU and the 50-step gradient time over the 50-step
    forward time on the 24^3, p = 4 mesh; the 64-flow ensemble (seed 0) in one
    persistent launch per RK stage against the same flows launched one after
    the other;
  * cpu_baseline: the oracle on the host cores for a bounded sample, all
    threads and one thread, with the CPU model.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--quick]
"""
import argparse
import hashlib
import json
import os
import statistics
import sys
import time

import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, published
FP64_PEAK_TFS = 78.6         # MI355X FP64 vector, published
# algorithmic bytes per node of one right-hand side: read U (40) and the metric
# terms (9 C + 1/(WJ): 80), write dU/dt (40)
RHS_BYTES_PER_NODE = 160.0
# one fused RK4 stage, averaged over the four stages: every stage reads its
# stage state (40) and the metric terms (80); stage 1 writes acc and Y (80);
# stages 2-3 read U^n and acc and write acc and Y (160); stage 4 reads acc and
# writes U (80): (200 + 280 + 280 + 200) / 4 = 240
STAGE_BYTES_PER_NODE = 240.0


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("stage.hip", "nsfr_device.h"):
        with open(os.path.join(ROOT, "paper_2312_07725_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_counters(workload_key):
    """rocprofv3 counter figures of the stage kernel for one workload, stored in
    profiles/stage_counters.json with the hash of the kernel source they were
    taken on; None if absent or the kernel changed since."""
    path = os.path.join(ROOT, "profiles", "stage_counters.json")
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    e = d.get(workload_key)
    if e and e.get("kernel_hash") == kernel_source_hash():
        return e
    return None


def log(msg):
    """Progress line on stderr (the JSON result line goes to stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def timed(fn, reps, stream):
    """HIP-event time (s) of fn(reps) on `stream`, synchronised on both sides."""
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    fn(reps)
    end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end) / 1e3


def per_launch(fn, reps, stream):
    """Per-launch HIP-event times (s) of reps calls of fn()."""
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for i in range(reps):
        fn()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    return [ev[i].elapsed_time(ev[i + 1]) / 1e3 for i in range(reps)]


def rhs_stats(nsfr, inputs, p, ne, c, reps=200, warm=20, quad="lgl", overint=0, scheme="nsfr"):
    g = nsfr.NSFR(p, ne, beta=0.2, c=c, quad=quad, overint=overint, scheme=scheme)
    U = inputs.tgv_state(g.node_coords().cpu()).cuda().contiguous()
    out = g.empty()
    st = torch.cuda.current_stream()
    for _ in range(warm):
        g.rhs(U, out)
    ts = per_launch(lambda: g.rhs(U, out), reps, st)
    med = statistics.median(ts)
    return g, U, {"p": p, "elements": ne ** 3, "nodes": g.n_nodes, "rhs_median_us": med * 1e6,
                  "rhs_mean_us": statistics.fmean(ts) * 1e6, "dof_updates_per_s": g.n_nodes / med,
                  "frac_hbm_roof": RHS_BYTES_PER_NODE * g.n_nodes / med / 1e9 / HBM_PEAK_GBS}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(p, ne, c, budget_s=15.0, budget_1_s=8.0):
    """The oracle (plain PyTorch CPU, FP64) on the host: full right-hand sides
    of the same workload, repeated until about budget_s seconds have elapsed,
    with all of torch's threads and then with one thread."""
    import oracle
    from paper_2312_07725_amd import inputs
    s = oracle.Scheme(p, (ne, ne, ne), beta=0.2, c=c)
    U = inputs.tgv_state(s.X)
    nodes = s.mesh.E * s.mesh.n ** 3

    def run(budget):
        s.rhs(U)   # warm-up (allocator, thread pool)
        n, t0 = 0, time.perf_counter()
        while True:
            s.rhs(U)
            n += 1
            el = time.perf_counter() - t0
            if el > budget:
                return n, el
    threads = torch.get_num_threads()
    n, el = run(budget_s)
    torch.set_num_threads(1)
    n1, el1 = run(budget_1_s)
    torch.set_num_threads(threads)
    return {"value": nodes * n / el, "unit": "DOF-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} full right-hand sides of the {ne}^3 p={p} warped TGV (c=c_HU) on the host, "
                      f"{el:.1f} s with {threads} threads; {n1} in {el1:.1f} s with 1 thread",
            "value_1_thread": nodes * n1 / el1, "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}


def adjoint_stats(nsfr, inputs, st, c, ne=24, p=4, nsteps=50):
    from paper_2312_07725_amd import adjoint
    g, U, fw = rhs_stats(nsfr, inputs, p, ne, c, reps=100, warm=10)
    lam = inputs.normal_like(U.shape, 1).cuda()
    gout = g.empty()
    for _ in range(10):
        g.rhs_vjp(U, lam, gout)
    tv = statistics.median(per_launch(lambda: g.rhs_vjp(U, lam, gout), 100, st))
    res = {"c": c, "rhs_median_us": fw["rhs_median_us"], "vjp_median_us": tv * 1e6,
           "vjp_over_rhs": tv * 1e6 / fw["rhs_median_us"]}
    if nsteps:
        dt = g.cfl_dt(U, 0.1)
        adjoint.integrate(g, U, dt, 2)
        adjoint.kinetic_energy_gradient(g, U, dt, 2)
        tf = timed(lambda k: adjoint.integrate(g, U, dt, k), nsteps, st)
        tg = timed(lambda k: adjoint.kinetic_energy_gradient(g, U, dt, k), nsteps, st)
        res.update({"steps": nsteps, "forward_ms": tf * 1e3, "gradient_ms": tg * 1e3, "gradient_over_forward": tg / tf})
    del g, U
    return res


def ensemble_stats(nsfr, inputs, st, steps=20):
    """64 TGV flows (seed 0): K RK4 steps in one persistent launch per stage
    (HIP graph) against the same flows' single-flow graphs run in turn."""
    draws = inputs.ensemble_draws(64, seed=0)
    cfgs = [nsfr.make_config(p, ne, beta=0.2, c=nsfr.c_hu(p)) for (ne, p, m) in draws]
    ens = nsfr.Ensemble(cfgs)
    U = ens.empty()
    singles = []
    for i, (ne, p, mach) in enumerate(draws):
        g = nsfr.NSFR(p, ne, beta=0.2, c=nsfr.c_hu(p))
        ens.flow_view(U, i).copy_(inputs.tgv_state(g.node_coords().cpu(), 1.4, mach))
        singles.append(g)
    dts = torch.empty(64, dtype=torch.float64, device="cuda")
    for i, g in enumerate(singles):
        g.cfl_dt(ens.flow_view(U, i).contiguous(), 0.1, out=dts[i:i + 1])
    nodes = sum(g.n_nodes for g in singles)
    work = ens.empty(3)
    ens.rk4_run(U, dts, 2, work=work)
    t_ens = timed(lambda k: ens.rk4_run(U, dts, k, work=work), steps, st)
    flows = [(g, ens.flow_view(U, i).contiguous().clone(), dts[i:i + 1].contiguous(), g.work(3))
             for i, g in enumerate(singles)]
    for g, Ui, dti, wi in flows:
        g.rk4_run(Ui, dti, None, 2, wi)

    def seq(k):
        for g, Ui, dti, wi in flows:
            g.rk4_run(Ui, dti, None, k, wi)
    t_seq = timed(seq, steps, st)
    del ens, singles, flows
    return {"flows": 64, "seed": 0, "nodes": nodes, "steps": steps,
            "ensemble_dof_updates_per_s_per_stage": 4 * nodes * steps / t_ens,
            "sequential_dof_updates_per_s_per_stage": 4 * nodes * steps / t_seq,
            "ensemble_over_sequential": t_seq / t_ens}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--p", type=int, default=3)
    ap.add_argument("--ne", type=int, default=16)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--quick", action="store_true", help="headline only: skip the extra measurements")
    ap.add_argument("--extra", default="all",
                    help="comma-separated extra blocks to run (rhs_16cubed, rhs_32cubed, adjoint, ensemble, gl, "
                         "scheme_cost) or 'all'")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain elementwise copy of 2 x 1 GiB (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (multi-GPU sharding is "
                                   "described, not built)"}))
        sys.exit(2)
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)

    from paper_2312_07725_amd import nsfr, inputs
    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.add(src, 0.0, out=dst)   # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del src, dst
    p, ne = args.p, args.ne
    c = nsfr.c_hu(p)
    g = nsfr.NSFR(p, ne, beta=0.2, c=c)
    nodes = g.n_nodes
    U = inputs.tgv_state(g.node_coords().cpu()).cuda().contiguous()
    out = g.empty()
    st = torch.cuda.current_stream()

    def steps(k):
        for _ in range(k):
            g.rhs(U, out)

    steps(args.warmup)
    t = timed(steps, args.steps, st)
    ms_per_step = 1e3 * t / args.steps
    value = nodes * args.steps / t
    med = statistics.median(per_launch(lambda: g.rhs(U, out), args.steps, st))

    # dominant kernel: the stage kernel, one launch per rhs
    t_kernel = t / args.steps
    achieved = RHS_BYTES_PER_NODE * nodes / t_kernel / 1e9
    key = f"rhs_p{p}_ne{ne}"
    ctr = load_counters(key)
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": ctr["hbm_bytes_per_launch"] if ctr else None,
            "kernel": f"stage_kernel<{p},true,0> (mode RHS)", "avg_launch_us": t_kernel * 1e6,
            "median_launch_us": med * 1e6, "algorithmic_bytes_per_launch": RHS_BYTES_PER_NODE * nodes,
            "fp64_tflops": None, "fp64_frac": None}
    if ctr and ctr.get("fp64_flop_per_launch"):
        tf = ctr["fp64_flop_per_launch"] / t_kernel / 1e12
        roof["fp64_tflops"], roof["fp64_frac"] = tf, tf / FP64_PEAK_TFS

    d = g.diagnostics(U).cpu()
    extra = {"entropy_rate_rel": abs(float(d[0])) / float(d[1]), "unphysical_nodes": g.check_state(U),
             "nodes": nodes, "rhs_median_us": med * 1e6, "kernel_source_hash": kernel_source_hash()}
    blocks = {"rhs_16cubed", "rhs_32cubed", "adjoint", "ensemble", "gl", "scheme_cost"}
    want = blocks if args.extra == "all" else set(args.extra.split(","))
    if want - blocks:
        raise SystemExit(f"unknown extra blocks {sorted(want - blocks)}")
    if not args.quick:
        del g, U, out
    if not args.quick and "rhs_16cubed" in want:
        log("rhs_16cubed")
        extra["rhs_16cubed"] = {}
        for pp in (3, 4, 5):
            gg, UU, r = rhs_stats(nsfr, inputs, pp, 16, nsfr.c_hu(pp))
            extra["rhs_16cubed"][f"p{pp}"] = r
            if pp == 3:   # the RK4 step of the same mesh, from a HIP graph
                dt = gg.cfl_dt(UU, 0.1)
                work = gg.work(3)
                gg.rk4_run(UU, dt, None, 10, work)
                ts = timed(lambda k: gg.rk4_run(UU, dt, None, k, work), 100, st)
                extra["rk4_16cubed_p3"] = {"step_us": ts / 100 * 1e6, "dof_updates_per_s_per_stage":
                                           4 * gg.n_nodes * 100 / ts,
                                           "frac_hbm_roof_stage": STAGE_BYTES_PER_NODE * gg.n_nodes * 400 / ts
                                           / 1e9 / HBM_PEAK_GBS}
            del gg, UU
        gg, UU, r = rhs_stats(nsfr, inputs, 3, 16, 0.0)
        extra["rhs_16cubed"]["p3_c0"] = r
        del gg, UU
    if not args.quick and "gl" in want:
        log("gl")
        # uncollocated: Gauss-Legendre rule with q = p + 1 + overint points
        # (entropy projection kernel + hybridised stage kernel per rhs)
        extra["rhs_16cubed_gl"] = {}
        for pp, ov in ((3, 0), (3, 1), (4, 0), (5, 0), (5, 3)):
            gg, UU, r = rhs_stats(nsfr, inputs, pp, 16, nsfr.c_hu(pp), reps=100, warm=10, quad="gl", overint=ov)
            del r["frac_hbm_roof"]
            r["q"] = pp + 1 + ov
            if "rhs_16cubed" in extra:
                r["vs_lgl_same_p"] = r["rhs_median_us"] / extra["rhs_16cubed"][f"p{pp}"]["rhs_median_us"]
            extra["rhs_16cubed_gl"][f"p{pp}_q{pp + 1 + ov}"] = r
            del gg, UU
    if not args.quick and "scheme_cost" in want:
        log("scheme_cost")
        # the paper's cost comparison (Sec. 7.4) on these kernels: NSFR-EC with
        # c_DG, conservative DG (Roe) and DG overintegrated to 2 (p + 1) points,
        # all on the Gauss-Legendre rule, warped TGV, one rhs
        extra["scheme_cost_gl"] = {}
        for ne_ in (8, 16):
            for pp in (3, 4, 5):
                t = {}
                for name, sch, ov in (("nsfr", "nsfr", 0), ("dg", "dg", 0), ("dg_overint", "dg", pp + 1)):
                    gg, UU, r = rhs_stats(nsfr, inputs, pp, ne_, 0.0, reps=50, warm=5, quad="gl", overint=ov,
                                          scheme=sch)
                    t[name] = r["rhs_median_us"]
                    del gg, UU
                extra["scheme_cost_gl"][f"ne{ne_}_p{pp}"] = {
                    "rhs_us": t, "nsfr_over_dg": t["nsfr"] / t["dg"], "dg_overint_over_nsfr": t["dg_overint"] / t["nsfr"]}
    if not args.quick and "rhs_32cubed" in want:
        log("rhs_32cubed")
        extra["rhs_32cubed"] = {}   # working sets of 0.3-1.1 GB: beyond the 256 MB last-level cache
        for pp in (3, 4, 5):
            gg, UU, r = rhs_stats(nsfr, inputs, pp, 32, nsfr.c_hu(pp), reps=200, warm=10)
            extra["rhs_32cubed"][f"p{pp}"] = r
            del gg, UU
        torch.cuda.empty_cache()
    if not args.quick and "adjoint" in want:
        log("adjoint")
        extra["adjoint_24cubed_p4"] = {"c0": adjoint_stats(nsfr, inputs, st, 0.0),
                                       "c_hu": adjoint_stats(nsfr, inputs, st, nsfr.c_hu(4), nsteps=0)}
        torch.cuda.empty_cache()
    if not args.quick and "ensemble" in want:
        log("ensemble")
        extra["ensemble"] = ensemble_stats(nsfr, inputs, st)

    cpu = None
    if not args.no_cpu:
        log("cpu_baseline")
        cpu = cpu_baseline(p, ne, c)

    line = {
        "metric": "FP64 DOF-updates/s per rhs (p=3..5) + %roofline; adjoint/forward cost ratio",
        "value": value, "unit": "DOF-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"inviscid TGV, {ne}^3 periodic hexahedra warped by the nonsymmetric map "
                               f"(beta=0.2), p={p} LGL, c=c_HU, Chandrashekar EC flux with Ranocha pressure fix, "
                               f"one full right-hand side (volume, surface, weight-adjusted mass inverse) per step",
                   "p": p, "elements": ne ** 3, "nodes": nodes, "mach": 0.1},
        "roofline": roof, "cpu_baseline": cpu, "extra": extra,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
