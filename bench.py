"""Benchmark of the NSFR hot path on one MI355X.

Workload (one "step"): one classical RK4 step -- four fused stage kernels, each
evaluating the full right-hand side (entropy-conserving two-point volume flux
differencing, surface fluxes, weight-adjusted inverse of the FR-modified mass
with c = c_HU) and the RK combination -- of the inviscid Taylor-Green vortex
on a 16^3-element periodic box warped by the paper's nonsymmetric map
(beta = 1/5), p = 3, FP64. Steps are replayed from a HIP graph.

value = DOF-updates per second per right-hand side = 4 * nodes * K / t.

Also reported: the dominant kernel against the HBM roofline (algorithmic
bytes / measured average stage-kernel time), the oracle on the host cores for
a bounded sample, single-rhs throughput for p = 3..5, and the adjoint/forward
cost ratio on the 24^3, p = 4 adjoint workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--quick]
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, published
FP64_PEAK_TFS = 78.6         # MI355X FP64 vector, published
# algorithmic bytes per node of one fused RK stage (average of the four stages):
# every stage reads its stage state (40 B) and the metric terms (9 C + 1/(WJ): 80 B);
# stage 1 writes acc and Y2 (80); stages 2-3 read U^n and acc and write acc and Y (160);
# stage 4 reads acc and writes U (80). (200 + 280 + 280 + 200) / 4 = 240.
STAGE_BYTES_PER_NODE = 240.0
RHS_BYTES_PER_NODE = 160.0   # U 40 + metrics 80 + dU/dt 40


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("stage.hip", "nsfr_device.h"):
        with open(os.path.join(ROOT, "paper_2312_07725_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload_key):
    """HBM bytes per launch measured with rocprofv3 counters (FETCH_SIZE and
    WRITE_SIZE), stored under profiles/ together with the hash of the kernel
    source they were taken on; null if the kernel changed since."""
    path = os.path.join(ROOT, "profiles", "stage_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        e = d.get(workload_key)
        if e and e.get("kernel_hash") == kernel_source_hash():
            return e["hbm_bytes_per_launch"]
    except Exception:
        return None
    return None


def timed(fn, reps, stream):
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    fn(reps)
    end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end) / 1e3


def rhs_throughput(nsfr, inputs, p, ne, c, reps=200, warm=20):
    g = nsfr.NSFR(p, ne, beta=0.2, c=c)
    U = inputs.tgv_state(g.node_coords().cpu()).cuda().contiguous()
    out = g.empty()
    st = torch.cuda.current_stream()

    def run(k):
        for _ in range(k):
            g.rhs(U, out)
    run(warm)
    t = timed(run, reps, st)
    return g, U, t / reps


def cpu_baseline(p, ne, c, budget_s=15.0):
    """The oracle (plain PyTorch CPU, FP64) on the host: full right-hand sides
    of the same workload, repeated until about budget_s seconds have elapsed."""
    import oracle
    from paper_2312_07725_amd import inputs
    s = oracle.Scheme(p, (ne, ne, ne), beta=0.2, c=c)
    U = inputs.tgv_state(s.X)
    s.rhs(U)   # warm-up (allocator, thread pool)
    n, t0 = 0, time.perf_counter()
    while True:
        s.rhs(U)
        n += 1
        el = time.perf_counter() - t0
        if el > budget_s:
            break
    nodes = s.mesh.E * s.mesh.n ** 3
    return {"value": nodes * n / el, "unit": "DOF-updates/s", "cores": torch.get_num_threads(),
            "kind": "oracle",
            "sample": f"{n} full right-hand sides of the {ne}^3 p={p} warped TGV (c=c_HU) on the host, {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--p", type=int, default=3)
    ap.add_argument("--ne", type=int, default=16)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--quick", action="store_true", help="skip the extra p / adjoint measurements")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain elementwise copy of 2 x 1 GiB (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
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
    dt = g.cfl_dt(U, 0.1)
    work = g.work(3)
    st = torch.cuda.current_stream()

    def steps(k):
        g.rk4_run(U, dt, None, k, work)

    steps(args.warmup)
    torch.cuda.synchronize()
    t = timed(steps, args.steps, st)
    ms_per_step = 1e3 * t / args.steps
    value = 4.0 * nodes * args.steps / t
    d = g.diagnostics(U).cpu()
    entropy_rel = abs(float(d[0])) / float(d[1])
    bad = g.check_state(U)

    # dominant kernel: the fused stage kernel, 4 launches per step
    t_kernel = t / (4 * args.steps)
    achieved = STAGE_BYTES_PER_NODE * nodes / t_kernel / 1e9
    key = f"p{p}_ne{ne}"
    traffic = load_traffic(key)
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": f"stage_kernel<{p},true,0>", "avg_launch_us": t_kernel * 1e6,
            "algorithmic_bytes_per_launch": STAGE_BYTES_PER_NODE * nodes}

    extra = {"entropy_rate_rel_after_run": entropy_rel, "unphysical_nodes": bad, "nodes": nodes}
    if not args.quick:
        per_p = {}
        for pp in (3, 4, 5):
            gg, UU, tr = rhs_throughput(nsfr, inputs, pp, ne, nsfr.c_hu(pp))
            per_p[f"p{pp}"] = {"rhs_us": tr * 1e6, "dof_updates_per_s": gg.n_nodes / tr,
                               "frac_hbm_roof": RHS_BYTES_PER_NODE * gg.n_nodes / tr / 1e9 / HBM_PEAK_GBS}
            del gg, UU
        gg, UU, tr0 = rhs_throughput(nsfr, inputs, p, ne, 0.0)
        per_p[f"p{p}_c0"] = {"rhs_us": tr0 * 1e6, "dof_updates_per_s": gg.n_nodes / tr0}
        extra["rhs_16cubed"] = per_p
        # a mesh whose working set exceeds the 256 MB last-level cache
        gg, UU, tr = rhs_throughput(nsfr, inputs, p, 32, c, reps=50)
        extra["rhs_32cubed"] = {"p": p, "rhs_us": tr * 1e6, "dof_updates_per_s": gg.n_nodes / tr,
                                "frac_hbm_roof": RHS_BYTES_PER_NODE * gg.n_nodes / tr / 1e9 / HBM_PEAK_GBS}
        del gg, UU
        # adjoint / forward cost on the 24^3, p = 4 adjoint workload
        ga, Ua, tf = rhs_throughput(nsfr, inputs, 4, 24, 0.0, reps=100)
        lam = inputs.normal_like(Ua.shape, 1).cuda()
        gout = ga.empty()

        def vj(k):
            for _ in range(k):
                ga.rhs_vjp(Ua, lam, gout)
        vj(10)
        tv = timed(vj, 100, st) / 100
        extra["adjoint"] = {"workload": "TGV 24^3 warped beta=0.2, p=4, c=0", "rhs_us": tf * 1e6,
                            "vjp_us": tv * 1e6, "vjp_over_rhs": tv / tf}
        del ga, Ua

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(p, ne, c)

    line = {
        "metric": "FP64 DOF-updates/s per rhs (p=3..5) + %roofline; adjoint/forward cost ratio",
        "value": value, "unit": "DOF-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"inviscid TGV, {ne}^3 periodic hexahedra warped by the nonsymmetric map "
                               f"(beta=0.2), p={p} LGL, c=c_HU, Chandrashekar EC flux with Ranocha pressure fix, "
                               f"RK4 step (4 fused rhs stages) from a HIP graph",
                   "p": p, "elements": ne ** 3, "nodes": nodes, "mach": 0.1, "cfl": 0.1},
        "roofline": roof, "cpu_baseline": cpu, "extra": extra,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
