"""Benchmark: GCP-CROWN domains bounded per second on one MI355X.

Default workload (--workload mlp784): MLP 784-256x6-10, weights N(0, 2/fan_in),
x0 ~ U[0,1]^784, eps = 0.015, 9 margin spec rows, 1024 BaB domains with 1-8
splits each, 200 LP-implied cuts over 2-6 neurons of >= 2 layers.  One step
bounds one batch: it resets alpha/beta/gamma and the Adam state to their
starting values, runs 20 projected Adam iterations (bound pass + adjoint +
update, all on the device) and the certifying pass (fp32 GEMMs, fp64
reductions, margin check).  value = domains per second over the timed steps.

Other workloads: --workload cnn (CNN-A shape, 2048 domains, 500 cuts),
--workload resnet (ResNet, 4096 domains, 1000 cuts), --workload batch (64
uneven MLP instances in grouped launches, compared with one gcp_optimize per
instance).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--mode bf16|fp32] [--workload mlp784|cnn|resnet|batch]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {  # MI355X published dense peaks
    "hbm_GBps": 8000.0,
    "bf16_TFLOPs": 2500.0,
    "fp32_TFLOPs": 157.3,
    "fp64_TFLOPs": 78.6,
    # fp32 FMAs on the vector ALUs without packed math (the build leaves it
    # off): 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP x 2.4 GHz
    "fp32_valu_TFLOPs": 78.6,
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mode", choices=["bf16", "fp32"], default="fp32",
                    help="GEMM precision of the 20 ascent iterations (the certifying pass is fp32/fp64 either way)")
    ap.add_argument("--domains", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the fp32-mode comparison run")
    ap.add_argument("--cpu-domains", type=int, default=None)
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="first run a plain device copy of this many MiB (HBM counter calibration)")
    ap.add_argument("--no-profile", action="store_true", help="do not time kernels with events")
    ap.add_argument("--graph", action="store_true", help="replay the Adam iteration as a captured hipGraph")
    ap.add_argument("--workload", choices=["mlp784", "cnn", "resnet", "batch", "bab"], default="mlp784")
    ap.add_argument("--roots", choices=["crown", "ibp"], default="crown",
                    help="root pre-activation bounds of the workload: the stored fp64 CROWN bounds or interval bounds")
    ap.add_argument("--retune", action="store_true",
                    help="autotune every GEMM/conv tile afresh instead of starting from the shipped MI355X choices")
    ap.add_argument("--persist", action="store_true",
                    help="run the Adam iterations as one persistent dataflow launch (GCP_FLAG_PERSIST; dense nets; "
                         "with --workload batch every instance shares that launch)")
    ap.add_argument("--explicit-pi", action="store_true",
                    help="optimise pi of every unstable neuron too (gcp_optimize_pi) instead of Lemma A.1's pi*")
    a = ap.parse_args()
    if a.domains is None:
        a.domains = {"mlp784": 1024, "cnn": 2048, "resnet": 4096, "batch": 0, "bab": 1024}[a.workload]
    if a.cpu_domains is None:
        a.cpu_domains = {"mlp784": 384, "cnn": 96, "resnet": 16, "batch": 0, "bab": 0}[a.workload]
    return a


WORKLOADS = {
    "mlp784": "GCP-CROWN bound optimisation, MLP 784-256x6-10, {B} BaB domains x 9 spec rows, 200 cuts, "
       "1-8 splits/domain, 20 Adam iterations + fp32/fp64 certifying pass",
    "cnn": "GCP-CROWN bound optimisation, CNN Conv(3,16,4,s2)-Conv(16,32,4,s2)-2048-100-10 on 3x32x32, {B} BaB "
       "domains x 9 spec rows, 500 cuts, 1-8 splits/domain, 20 Adam iterations + certifying pass",
    "resnet": "GCP-CROWN bound optimisation, ResNet stem16-blocks16/32/64-linear10 on 3x32x32, {B} BaB domains x 9 "
       "spec rows, 1000 cuts, 1-8 splits/domain, 20 Adam iterations + certifying pass",
}


def use_tuned_tiles():
    """Start from the tile choices the autotuner made on MI355X for these
    workloads (paper_2208_05740_amd/tuned_tiles_gfx950.txt), so that every run
    launches the same kernels as the committed profiles; shapes not listed are
    tuned as usual.  The library appends to the cache file, so it gets a copy."""
    import shutil
    import tempfile
    if "GCP_TILE_CACHE" in os.environ:
        return
    src = os.path.join(ROOT, "paper_2208_05740_amd", "tuned_tiles_gfx950.txt")
    if not os.path.exists(src):
        return
    fd, dst = tempfile.mkstemp(prefix="gcp_tiles_", suffix=".txt")
    os.close(fd)
    shutil.copyfile(src, dst)
    os.environ["GCP_TILE_CACHE"] = dst


def main():
    args = parse()
    if not args.retune:
        use_tuned_tiles()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); sharding the BaB domains "
              "of a call across GPUs is not implemented.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2208_05740_amd import binding as B
    from workloads import gen

    dev = torch.device("cuda:0")
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "bab":
        return bench_bab(args)
    prob = gen.make_workload(args.workload, 0, B=args.domains, roots=args.roots)
    P = B.Problem(prob, device=dev)
    M = P.M
    # starting point: CROWN-adaptive alpha, beta ~ U[0,1] on used split slots, gamma = 0
    a_vec = torch.tensor(gen.crown_alpha_init(prob.lu), dtype=torch.float32, device=dev)
    alpha0 = a_vec.expand(M, -1).contiguous()
    beta0 = torch.tensor(prob.beta.reshape(M, -1), dtype=torch.float32, device=dev)
    gamma0 = torch.zeros(M, P.N, dtype=torch.float32, device=dev)
    alpha, beta, gamma = alpha0.clone(), beta0.clone(), gamma0.clone()
    pi = args.explicit_pi
    state = torch.zeros(B.adam_state_size(M, P.n_I, P.K, P.N, explicit_pi=pi), dtype=torch.float32, device=dev)
    bound = torch.empty(M, dtype=torch.float64, device=dev)
    ver = torch.empty(M, dtype=torch.uint8, device=dev)
    rho0 = torch.tensor(gen.rho_init(prob.lu), dtype=torch.float32, device=dev).expand(M, -1).contiguous()
    rho = rho0.clone()
    o = prob.opt
    use_graph = [args.graph]

    def step(mode, explicit=pi):
        alpha.copy_(alpha0)
        beta.copy_(beta0)
        gamma.copy_(gamma0)
        state.zero_()
        kw = dict(iters=o["iters"], lr_alpha=o["lr_alpha"], lr_mult=o["lr_mult"], decay=o["decay"], b1=o["adam_b1"],
                  b2=o["adam_b2"], adam_eps=o["adam_eps"], mode=mode | (B.GCP_FLAG_PERSIST if args.persist else 0),
                  use_graph=use_graph[0])
        if explicit:
            rho.copy_(rho0)
            b, v = B.optimize_pi(P.net, P.x0, P.eps, P.C, P.splits, P.cuts, alpha, beta, gamma, rho, state, **kw)
            bound.copy_(b)
            ver.copy_(v)
        else:
            B.optimize(P.net, P.x0, P.eps, P.C, P.splits, P.cuts, alpha, beta, gamma, state, bound_out=bound,
                       verified_out=ver, **kw)

    def timed(mode, steps, warmup):
        for _ in range(warmup):
            step(mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step(mode)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    if args.copy_probe_mb:
        src = torch.ones(args.copy_probe_mb << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    def measure(mode, steps, warmup):
        """Timed steps, then (unless --no-profile) the same steps again with
        every library launch bracketed by HIP events on its stream (the
        markers slow the run, so the timed value comes from the first
        region); returns the time, the kernel classes, the final bounds and
        the final parameters of the last step."""
        dt = timed(mode, steps, warmup)
        kp, dtp = None, None
        if not args.no_profile:
            B.profile_enable(True)
            use_graph[0] = False     # per-kernel events need eager launches
            dtp = timed(mode, steps, 0)
            use_graph[0] = args.graph
            B.profile_enable(False)
            kp = B.profile_read()
        torch.cuda.synchronize()
        par = tuple(t.cpu().numpy().astype(np.float64) for t in (alpha, beta, gamma))
        return dt, kp, dtp, bound.cpu().numpy().copy(), par

    def kernel_table(kp):
        return {k: {"launches": v["launches"], "avg_us": round(1e3 * v["ms"] / v["launches"], 2)}
                for k, v in sorted(kp.items(), key=lambda kv: -kv[1]["ms"])[:8]}

    mode = B.GCP_MODE_BF16 if args.mode == "bf16" else B.GCP_MODE_FP32
    dt, kprof, dt_prof, bound_main, par_main = measure(mode, args.steps, args.warmup)
    value = args.domains * args.steps / dt
    out = {
        "metric": "BaB domains bounded/sec (fwd+adjoint iter) at fixed bound accuracy; % MFMA/HBM peak",
        "value": value,
        "unit": "domains/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1000.0 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.mode,
        "data": "synthetic",
        "config": {
            "workload": WORKLOADS[args.workload].format(B=args.domains),
            "domains": args.domains, "spec_rows": prob.S, "rows": M, "n_unstable": P.n_I,
            "root_bounds": "fp64 CROWN (stored)" if args.roots == "crown" else "interval arithmetic",
            "cuts": P.N, "split_slots": P.K, "iters": o["iters"], "graph_replay": args.graph,
            "domain_iters_per_s": value * o["iters"],
            "relaxation": "explicit pi (rho optimised)" if pi else "Lemma A.1 pi*",
            "final_bound_mean": float(bound_main.mean()),
            "verified_rows": int((bound_main >= 0).sum()),
        },
    }
    if kprof:
        # the adjoint's a_hat: stored by the bound pass, or rebuilt per layer
        # (the library recomputes only where the stored copies would not fit)
        out["config"]["a_hat"] = ("recomputed" if any(k.split(".")[0] in ("ahat", "convT_ahat") for k in kprof)
                                  else "stored")
    if args.workload == "resnet" and not args.no_compare:
        # the ResNet configuration's own form: a_hat recomputed in the adjoint
        # (bitwise equal results: the recomputing GEMM sums in the same order)
        dtr = timed(mode | B.GCP_FLAG_RECOMPUTE, max(1, args.steps // 2), 1)
        torch.cuda.synchronize()
        out["config"]["recompute_form"] = {
            "value": args.domains * max(1, args.steps // 2) / dtr,
            "ms_per_step": dtr * 1000.0 / max(1, args.steps // 2),
            "final_bound_equals_stored": bool(np.array_equal(bound.cpu().numpy(), bound_main)),
        }
    if pi:
        # the same optimisation with Lemma A.1's pi*, for the bound it reaches
        step(mode, explicit=False)
        torch.cuda.synchronize()
        closed = bound.cpu().numpy().copy()
        out["config"]["lemma_pi_final_bound_mean"] = float(closed.mean())
        out["config"]["rows_tighter_than_lemma_pi"] = float(np.mean(bound_main > closed))
        out["config"]["lemma_pi_verified_rows"] = int((closed >= 0).sum())
    copy_bw = None
    if kprof:
        out["roofline"] = roofline(kprof, args.mode)
        out["roofline"]["instrumented_ms_per_step"] = dt_prof * 1000.0 / args.steps
        copy_bw = copy_bandwidth()
        out["roofline"]["achievable_copy_GBps"] = copy_bw
        out["config"]["kernels"] = kernel_table(kprof)
    flagged = None
    if not pi and mode == B.GCP_MODE_FP32:
        flagged, out["outward"] = outward(B, P, alpha, beta, gamma, bound_main)
    if not pi:
        out["oracle_error"] = oracle_error(prob, bound_main, par_main, 0, flagged=flagged)
    if not args.no_compare:
        other = B.GCP_MODE_FP32 if mode == B.GCP_MODE_BF16 else B.GCP_MODE_BF16
        osteps = max(1, args.steps // 2)
        dt2, kprof2, dt_prof2, bound_other, par_other = measure(other, osteps, 1)
        rel = np.abs(bound_main - bound_other) / np.maximum(np.abs(bound_other), 1e-30)
        om = {
            "dtype": "fp32" if other == B.GCP_MODE_FP32 else "bf16",
            "value": args.domains * osteps / dt2,
            "final_bound_rel_diff_max": float(rel.max()),
            "final_bound_rel_diff_median": float(np.median(rel)),
            "final_bound_mean": float(bound_other.mean()),
        }
        if not pi:
            if args.mode == "fp32":
                om.update(scaled_diff(prob, bound_main, bound_other, par_main))
            else:
                om.update(scaled_diff(prob, bound_other, bound_main, par_other))
        if kprof2:
            om["roofline"] = roofline(kprof2, om["dtype"])
            om["roofline"]["instrumented_ms_per_step"] = dt_prof2 * 1000.0 / osteps
            om["roofline"]["achievable_copy_GBps"] = copy_bw
            om["kernels"] = kernel_table(kprof2)
        if not pi:
            om["oracle_error"] = oracle_error(prob, bound_other, par_other, 0)
        out["config"]["other_mode"] = om
    if not args.no_cpu_baseline:
        cb, g_oracle, rows = cpu_baseline([prob], args.cpu_domains)
        out["cpu_baseline"] = cb
        if not pi:
            out["oracle_opt_gap"] = opt_gap(prob, bound_main, g_oracle, rows)
            if not args.no_compare:
                out["config"]["other_mode"]["oracle_opt_gap"] = opt_gap(prob, bound_other, g_oracle, rows)
    print(json.dumps(out))


def outward(B, P, alpha, beta, gamma, certified, reps=5):
    """The certifying pass at the final parameters with GCP_FLAG_OUTWARD
    (every bound minus its rounding slack) beside the plain one: verified
    rows and the time of each form (HIP events around `reps` calls)."""
    import numpy as np
    import torch

    def run(mode):
        return B.bound(P.net, P.x0, P.eps, P.C, P.splits, P.cuts, alpha, beta, gamma, mode=mode, verified=True)

    times = {}
    for name, mode in (("plain", B.GCP_MODE_FP32), ("outward", B.GCP_MODE_FP32 | B.GCP_FLAG_OUTWARD)):
        run(mode)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            g, v, _ = run(mode)
        e1.record()
        torch.cuda.synchronize()
        times[name] = e0.elapsed_time(e1) / reps
        if name == "plain":
            plain = g.cpu().numpy()
        else:
            flagged, vf = g.cpu().numpy(), v.cpu().numpy()
    return flagged, {
        "certified_equals_plain_pass": bool(np.array_equal(plain, certified)),
        "verified_rows": int(vf.sum()), "verified_rows_plain": int((certified >= 0).sum()),
        "slack_rel_max": float(np.max((certified - flagged) / np.maximum(np.abs(certified), 1e-300))),
        "slack_rel_median": float(np.median((certified - flagged) / np.maximum(np.abs(certified), 1e-300))),
        "ms_certifying_pass": times["plain"], "ms_certifying_pass_outward": times["outward"]}


def oracle_error(prob, bound, par, seed, n=64, flagged=None):
    """Error of the device's certified bounds against the FP64 oracle at the
    device's final parameters, on a sample of rows (n random rows and the
    last 8): max |d| / max(|g|, T) (T = sum of the magnitudes of every term
    of the bound) and max |d| / |g|.  With ``flagged`` (the GCP_FLAG_OUTWARD
    bounds at the same parameters) also how far those lie below the exact
    value and their slack, in units of T."""
    import numpy as np

    from oracle import gcp_oracle as O
    M = bound.size
    rng = np.random.default_rng(seed)
    rows = np.unique(np.concatenate([rng.choice(M - 8, size=min(n, M - 8), replace=False), np.arange(M - 8, M)]))
    a, b, c = (x[rows] for x in par)
    ref = O.bound(prob, a, b, c, rows=rows, flat=True)
    T = O.error_scale(prob, a, b, c, rows=rows, flat=True)
    d = np.abs(bound[rows] - ref)
    res = {"rows_sampled": int(rows.size), "max_rel_err_T": float((d / np.maximum(np.abs(ref), T)).max()),
           "max_rel_err": float((d / np.abs(ref)).max()),
           "rows_above_exact": int((bound[rows] > ref).sum()),
           "sample": f"{rows.size} rows ({min(n, M - 8)} seeded random + the last 8), oracle bound (fp64) at the "
                     "device's final alpha, beta, gamma"}
    if flagged is not None:
        res["outward_rows_above_exact"] = int((flagged[rows] > ref).sum())
        res["outward_max_minus_exact_T"] = float(((flagged[rows] - ref) / T).max())
        res["outward_slack_T_max"] = float(((bound[rows] - flagged[rows]) / T).max())
    return res


def scaled_diff(prob, b32, b16, par32, max_rows=20000):
    """bf16 against fp32 final bounds relative to max(|g|, T), T = the sum of
    the magnitudes of every term of the fp32 run's bound (the oracle's error
    scale at its final parameters), over every row (or a seeded sample of
    max_rows rows)."""
    import numpy as np

    from oracle import gcp_oracle as O
    M = b32.size
    rows = np.arange(M) if M <= max_rows else np.sort(np.random.default_rng(1).choice(M, max_rows, replace=False))
    a, b, c = (x[rows] for x in par32)
    T = O.error_scale(prob, a, b, c, rows=rows, flat=True)
    d = np.abs(b16[rows] - b32[rows]) / np.maximum(np.abs(b32[rows]), T)
    return {"final_bound_diff_max_over_T": float(d.max()), "final_bound_diff_rows": int(rows.size)}


def opt_gap(prob, bound, g_oracle, rows):
    """Final certified bound of the device run against the oracle's own
    20-iteration fp64 optimisation from the same start, on the rows the CPU
    baseline optimised: (device - oracle) / max(|oracle|, T)."""
    import numpy as np

    from oracle import gcp_oracle as O
    del O
    rel = (bound[rows] - g_oracle) / np.maximum(np.abs(g_oracle), 1e-30)
    return {"rows": int(rows.size), "max_abs_rel_gap": float(np.abs(rel).max()), "mean_rel_gap": float(rel.mean()),
            "note": "(device final bound - oracle 20-step optimum) / |oracle|, same start and Adam settings"}


def copy_bandwidth(mib=2048, reps=5):
    """Achievable HBM bandwidth on this device: a plain device-to-device copy
    of `mib` MiB (read + write bytes over the best of `reps` event-timed runs)."""
    import torch
    src = torch.ones(mib << 18, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None or ms < best else best
    del src, dst
    return 2.0 * (mib << 20) / (best * 1e-3) / 1e9


def roofline(kprof, dtype):
    """Dominant kernel class (largest total time in the timed region) against
    the published MI355X peak of the resource its arithmetic intensity binds
    it to.  Algorithmic work per launch: its FLOPs (the GEMMs' 2 M N K) and
    its optimiser-state bytes (alpha read in the bound pass, alpha and its
    Adam moments read and written in the adjoint, multipliers with their
    moments in their update, the split mask); intensity = FLOPs / those
    bytes, compared with the ridge of the kernel's operand type.  `achieved`
    = the bound resource's algorithmic amount per launch over the launch's
    average event-timed duration.  The every-operand-once byte figure is
    reported beside it."""
    name, k = max(kprof.items(), key=lambda kv: kv[1]["ms"])
    secs = k["ms"] * 1e-3
    mf_peak = PEAKS["bf16_TFLOPs"] if ".bf16" in name else PEAKS["fp32_TFLOPs"]
    ridge = mf_peak * 1e12 / (PEAKS["hbm_GBps"] * 1e9)
    alg = k.get("alg_bytes", 0.0)
    ai = k["flops"] / alg if alg else float("inf")
    n = k["launches"]
    r = {"kernel": name, "launches": n, "avg_us": 1e6 * secs / n,
         "algorithmic_bytes_per_launch": alg / n, "flops_per_launch": k["flops"] / n,
         "operand_bytes_per_launch": k["bytes"] / n, "operand_GBps": k["bytes"] / secs / 1e9,
         "arith_intensity": ai, "ridge": ridge}
    if ".direct" in name:
        # the direct transposed conv does its FMAs on the vector ALUs
        ach = k["flops"] / secs / 1e12
        peak = PEAKS["fp32_valu_TFLOPs"]
        r.update(bound="alu", achieved=ach, peak=peak, unit="TFLOP/s", frac=ach / peak)
    elif ai < ridge:
        ach = alg / secs / 1e9
        r.update(bound="hbm", achieved=ach, peak=PEAKS["hbm_GBps"], unit="GB/s", frac=ach / PEAKS["hbm_GBps"])
    else:
        ach = k["flops"] / secs / 1e12
        r.update(bound="mfma", achieved=ach, peak=mf_peak, unit="TFLOP/s", frac=ach / mf_peak)
    r["traffic"] = measured_traffic(name)
    return r


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    runs (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter's
    reading for a plain copy of known size), or None when no record exists
    for this kernel or the kernel source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    from paper_2208_05740_amd.profiling import source_sha
    if rec.get("source_sha") != source_sha():
        return None
    k = rec.get("kernels", {}).get(kernel)
    if not k:
        return None
    return k["fetch_kib"] * 1024 * rec["fetch_scale"] + k["write_kib"] * 1024 * rec["write_scale"]


def oracle_start(prob, rows):
    """Starting parameters of the bench for a row subset, in float64: the
    CROWN-adaptive alpha, the problem's beta and gamma."""
    import numpy as np

    from workloads import gen
    a = np.broadcast_to(gen.crown_alpha_init(prob.lu), (rows.size, len(gen.crown_alpha_init(prob.lu)))).copy()
    b = prob.beta.reshape(prob.B * prob.S, -1)[rows].astype(np.float64)
    c = prob.gamma.reshape(prob.B * prob.S, -1)[rows].astype(np.float64)
    return a, b, c


def cpu_baseline(probs, nd, runs=3):
    """The FP64 oracle (as it stands) on the first `nd` domains of each given
    problem, the same 20-iteration optimisation + final bound, on the host
    cores this process may run on (torch and BLAS threads set to that
    count); the median of `runs` runs.  Returns the record, the oracle's
    final bounds of the first problem's rows, and those rows."""
    import numpy as np
    import torch
    from threadpoolctl import threadpool_limits

    from oracle import gcp_oracle as O
    cores = len(os.sched_getaffinity(0))
    torch.set_num_threads(cores)
    times, g_first, rows_first = [], None, None
    with threadpool_limits(limits=cores):
        for _ in range(runs):
            t0 = time.perf_counter()
            total = 0
            for i, prob in enumerate(probs):
                k = min(nd, prob.B)
                rows = np.arange(k * prob.S)
                a, b, c = oracle_start(prob, rows)
                g, *_ = O.optimize(prob, alpha=a, beta=b, gamma=c, rows=rows, flat=True)
                if i == 0:
                    g_first, rows_first = g, rows
                total += k
            times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    what = probs[0].name if len(probs) == 1 else f"{len(probs)} instances"
    rec = {"value": total / dt, "unit": "domains/s", "cores": cores, "kind": "oracle",
           "sample": f"first {nd} domains of {what} ({total} domains), same 20-iteration optimisation + final "
                     f"bound in float64; median of {runs} runs: {dt:.1f} s ({', '.join(f'{t:.1f}' for t in times)})"}
    return rec, g_first, rows_first


def bench_bab(args):
    """gcp_bab on one property of the 784-256x6-10 MLP (the spec row with the
    largest root bound, 200 cuts): `domains` domains per bounding call,
    splits up to depth 16, a budget of `steps` full batches.  One untimed
    run of the same search first (it tunes every batch shape the search
    meets), then the timed one; beside it gcp_optimize alone on one full
    batch of the same shape, the rate the search would reach without its
    own work."""
    import numpy as np
    import torch

    from paper_2208_05740_amd import binding as B
    from workloads import gen

    dev = torch.device("cuda:0")
    mode = B.GCP_MODE_BF16 if args.mode == "bf16" else B.GCP_MODE_FP32
    prob = gen.make_workload("mlp784", 0, B=1, roots=args.roots)
    P = B.Problem(prob, device=dev)
    a0 = torch.tensor(gen.crown_alpha_init(prob.lu), dtype=torch.float32, device=dev).expand(P.M, -1).contiguous()
    z = lambda n: torch.zeros(P.M, n, dtype=torch.float32, device=dev)  # noqa: E731
    sp0 = B.Splits(P.net, gen.Splits(np.full((1, 0), -1, np.int32), np.zeros((1, 0), np.int32),
                                     np.zeros((1, 0), np.int8)))
    root, _, _ = B.bound(P.net, P.x0, P.eps, P.C, sp0, P.cuts, a0, z(0), z(P.N), mode=B.GCP_MODE_FP32)
    s = int(torch.argmax(root).item())
    c_row = P.C[s].contiguous()
    o = prob.opt
    budget = args.domains * args.steps
    kw = dict(cuts=P.cuts, batch=args.domains, max_depth=16, max_domains=budget, max_pool=1 << 22, retries=0,
              iters=o["iters"], lr_alpha=o["lr_alpha"], lr_mult=o["lr_mult"], decay=o["decay"], mode=mode)
    for _ in range(max(args.warmup, 1)):
        B.bab(P.net, P.x0, P.eps, c_row, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = B.bab(P.net, P.x0, P.eps, c_row, **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # the bounding call alone at the full batch shape (one spec row per domain)
    sp = B.Splits(P.net, gen.Splits(np.full((args.domains, 16), -1, np.int32), np.zeros((args.domains, 16), np.int32),
                                    np.ones((args.domains, 16), np.int8)))
    al = torch.tensor(gen.crown_alpha_init(prob.lu), dtype=torch.float32, device=dev).expand(args.domains, -1)
    al = al.contiguous()
    be = torch.zeros(args.domains, 16, dtype=torch.float32, device=dev)
    ga = torch.zeros(args.domains, P.N, dtype=torch.float32, device=dev)
    st = torch.zeros(B.adam_state_size(args.domains, P.n_I, 16, P.N), dtype=torch.float32, device=dev)

    def opt():
        B.optimize(P.net, P.x0, P.eps, c_row.reshape(1, -1), sp, P.cuts, al.clone(), be.clone(), ga.clone(),
                   st.zero_(), iters=o["iters"], lr_alpha=o["lr_alpha"], lr_mult=o["lr_mult"], decay=o["decay"],
                   mode=mode)
    opt()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(3):
        opt()
    torch.cuda.synchronize()
    opt_rate = 3 * args.domains / (time.perf_counter() - t1)
    value = res["bounded"] / dt
    out = {
        "metric": "BaB domains bounded/sec (fwd+adjoint iter) at fixed bound accuracy; % MFMA/HBM peak",
        "value": value, "unit": "domains/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1000.0 / max(res["rounds"], 1), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.mode, "data": "synthetic",
        "config": {
            "workload": f"branch and bound (gcp_bab) on one property of the MLP 784-256x6-10 (spec row {s}, the "
                        f"largest root bound), 200 cuts, {args.domains} domains per bounding call, depth <= 16, "
                        f"budget {budget} domains, 20 Adam iterations + certifying pass per call",
            "root_bound": float(root[s].item()), "result": res,
            "ms_per_round": dt * 1000.0 / max(res["rounds"], 1),
            "optimize_only_domains_per_s": opt_rate,
            "search_efficiency": value / opt_rate,
            "note": "one spec row per domain (the headline line counts 9 per domain); ms_per_step is per round; "
                    "the ramp-up rounds (1, 2, 4, ... domains) are inside the timed search",
        },
    }
    print(json.dumps(out))


def bench_batch(args):
    """Config 4: 64 uneven MLP instances.  value = domains/s of the grouped
    batch (gcp_optimize_batch); the same steps with one gcp_optimize call per
    instance are timed beside it, and their final bounds must be identical."""
    import numpy as np
    import torch

    from paper_2208_05740_amd import binding as B
    from workloads import gen
    dev = torch.device("cuda:0")
    probs = gen.make_batch(seed=0)
    Ps = [B.Problem(p, device=dev) for p in probs]
    o = probs[0].opt
    mode = B.GCP_MODE_BF16 if args.mode == "bf16" else B.GCP_MODE_FP32
    items = []
    for p, P in zip(probs, Ps):
        a0 = torch.tensor(gen.crown_alpha_init(p.lu), dtype=torch.float32, device=dev).expand(P.M, -1).contiguous()
        b0 = torch.tensor(p.beta.reshape(P.M, -1), dtype=torch.float32, device=dev)
        items.append(dict(P=P, a0=a0, b0=b0, alpha=a0.clone(), beta=b0.clone(),
                          gamma=torch.zeros(P.M, P.N, dtype=torch.float32, device=dev),
                          state=torch.zeros(B.adam_state_size(P.M, P.n_I, P.K, P.N), dtype=torch.float32, device=dev),
                          bound=torch.empty(P.M, dtype=torch.float64, device=dev),
                          verified=torch.empty(P.M, dtype=torch.uint8, device=dev)))

    def reset():
        for it in items:
            it["alpha"].copy_(it["a0"])
            it["beta"].copy_(it["b0"])
            it["gamma"].zero_()
            it["state"].zero_()

    use_graph = [args.graph]

    def step_batched():
        reset()
        B.optimize_batch(items, iters=o["iters"], lr_alpha=o["lr_alpha"], lr_mult=o["lr_mult"], decay=o["decay"],
                         b1=o["adam_b1"], b2=o["adam_b2"], adam_eps=o["adam_eps"],
                         mode=mode | (B.GCP_FLAG_PERSIST if args.persist else 0), use_graph=use_graph[0])

    def step_single():
        reset()
        for it in items:
            P = it["P"]
            B.optimize(P.net, P.x0, P.eps, P.C, P.splits, P.cuts, it["alpha"], it["beta"], it["gamma"], it["state"],
                       iters=o["iters"], lr_alpha=o["lr_alpha"], lr_mult=o["lr_mult"], decay=o["decay"],
                       b1=o["adam_b1"], b2=o["adam_b2"], adam_eps=o["adam_eps"], mode=mode,
                       bound_out=it["bound"], verified_out=it["verified"])

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    dt = timed(step_batched, args.steps, args.warmup)
    bounds_b = [it["bound"].cpu().numpy().copy() for it in items]
    kprof = None
    if not args.no_profile:
        # per-kernel event timing needs kernels that do not overlap: the
        # instrumented replay runs the large instances one after another
        prev = os.environ.get("GCP_BATCH_STREAMS")
        os.environ["GCP_BATCH_STREAMS"] = "1"
        B.profile_enable(True)
        use_graph[0] = False
        dt_prof = timed(step_batched, args.steps, 0)
        use_graph[0] = args.graph
        B.profile_enable(False)
        kprof = B.profile_read()
        if prev is None:
            del os.environ["GCP_BATCH_STREAMS"]
        else:
            os.environ["GCP_BATCH_STREAMS"] = prev
    dts = timed(step_single, args.steps, 1)
    bounds_s = [it["bound"].cpu().numpy().copy() for it in items]
    same = all(np.array_equal(x, y) for x, y in zip(bounds_b, bounds_s))
    dom = sum(p.B for p in probs)
    value = dom * args.steps / dt
    out = {
        "metric": "BaB domains bounded/sec (fwd+adjoint iter) at fixed bound accuracy; % MFMA/HBM peak",
        "value": value, "unit": "domains/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1000.0 / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.mode, "data": "synthetic",
        "config": {
            "workload": f"GCP-CROWN batch: {len(probs)} MLP instances (depth 3-9, width 64-1024, input 784/3072, "
                        f"16-4096 domains log-uniform, 50-1000 cuts, 9 spec rows), "
                        f"{'one persistent launch' if args.persist else 'grouped launches'}, 20 Adam "
                        f"iterations + certifying pass",
            "persistent_launch": bool(args.persist),
            "instances": len(probs), "domains": dom, "rows": sum(P.M for P in Ps), "graph_replay": args.graph,
            "per_instance_launches": {"value": dom * args.steps / dts, "ms_per_step": dts * 1000.0 / args.steps},
            "speedup_vs_per_instance": dts / dt,
            "final_bounds_identical": bool(same),
        },
    }
    if kprof:
        out["roofline"] = roofline(kprof, args.mode)
        out["roofline"]["instrumented_ms_per_step"] = dt_prof * 1000.0 / args.steps
        out["config"]["kernels"] = {k: {"launches": v["launches"], "avg_us": round(1e3 * v["ms"] / v["launches"], 2)}
                                    for k, v in sorted(kprof.items(), key=lambda kv: -kv[1]["ms"])[:8]}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(probs[:8], 16)[0]
    print(json.dumps(out))


if __name__ == "__main__":
    main()
