"""Benchmark of the CPIC hot path on one MI355X.

Workload (the N=1 line): one synthetic MV-model Glasma event on a 512^2
lattice, L = 6 fm, g^2 mu = 2 GeV, m = 0.2 GeV, Lambda = 10 GeV, 50 colour
sheets, dtau = a/8 (1024 steps to 1.5 fm/c), with 1e5 charm quarks
(m = 1.27 GeV, p_T = 0, formed at 0.1 fm/c), double precision.  A step is one
leapfrog update of the fields plus the push of every formed particle plus
the broadening sums.  The initial condition is built on the GPU before the
timed region; W warm-up steps (past the formation step) are not timed, then
K steps are timed with a barrier and synchronisation on both sides.

Extra keys report the same event in single precision (reunitarisation every
16 steps) and the batched multi-event mode; the CPU oracle is timed on a
bounded sample of the same workload on the host cores.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
HBARC_GEV_FM = 0.1973269804
FP64_VALU_TFLOPS = 78.6
BYTES_PER_SITE = {"f64": 68 * 2 * 8, "f32": 68 * 2 * 4}     # read + write of U1 U2 phi E1 E2 pi
PART_REALS_RW = 2 * 18 + 2 * 2                               # particle record read+write (reals + 2 int cells)


def glasma_512(precision, N=512, L=6.0, seed=3):
    import paper_2303_05599_amd as cp
    return dict(N=N, L_fm=L, g2mu_GeV=2.0, m_ir_GeV=0.2, uv_GeV=10.0, n_sheets=50, dtau_over_a=0.125,
                tau_max_fm=1.5, seed=seed, precision=precision, reunit_every=16, record_every=8)


def charm(n=100_000, seed=4):
    return dict(n=n, mass_GeV=1.27, pT_min_GeV=0.0, pT_max_GeV=0.0, azimuth_uniform=1, tau_form_fm=0.1, rep=0,
                seed=seed)


def run_event(precision, steps, warmup):
    import torch
    import paper_2303_05599_amd as cp
    ctx = cp.Context(glasma_512(precision), charm())
    t0 = time.perf_counter()
    ctx.init_mv()
    t_ic = time.perf_counter() - t0
    ctx.step(warmup)
    ctx.sync()
    tune_report = ctx.tune(5)
    launch = ctx.get_launch()
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(steps)
    ctx.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tm = ctx.timing()
    ctx.set_timing(False)
    d = ctx.diagnostics()
    obs = ctx.observables()
    # graph-replayed rate over the rest of the run (not the headline number)
    n_left = min(256, 1024 - ctx.n)
    t0 = time.perf_counter()
    ctx.evolve((ctx.n + n_left) * 0.125 * 6.0 / 512 * (1 - 1e-12))
    ctx.sync()
    graph_ms = (time.perf_counter() - t0) * 1e3 / max(n_left, 1)
    ctx.close()
    return dict(wall=wall, t_ic=t_ic, timing=tm, diag=d, obs=obs, graph_ms_per_step=graph_ms, launch=launch,
                tune_report=tune_report)


def batch_events(precision, n_events=64, seed=5):
    """Uneven batch: N uniform over {128, 256, 384, 512}, L = 6 fm (dtau = a/8, 2N steps to
    1.5 fm/c), g2mu ~ U[1.5, 2.5] GeV, m = 0.1 g2mu, Lambda = 10 GeV, 50 sheets; 1e4..1e5
    beauty quarks (m = 4.18 GeV, formed at 1/(2m)) with p_T ~ U[0, 5] GeV; event e seeded 1000 + e."""
    rng = np.random.default_rng(seed)
    Ns = rng.choice([128, 256, 384, 512], n_events)
    g2mu = rng.uniform(1.5, 2.5, n_events)
    npart = rng.integers(10_000, 100_001, n_events)
    tau_form = HBARC_GEV_FM / (2 * 4.18)
    gl = [dict(N=int(Ns[e]), L_fm=6.0, g2mu_GeV=float(g2mu[e]), m_ir_GeV=0.1 * float(g2mu[e]), uv_GeV=10.0,
               n_sheets=50, dtau_over_a=0.125, tau_max_fm=1.5, seed=1000 + e, precision=precision,
               reunit_every=16, record_every=8) for e in range(n_events)]
    pl = [dict(n=int(npart[e]), mass_GeV=4.18, pT_min_GeV=0.0, pT_max_GeV=5.0, azimuth_uniform=1,
               tau_form_fm=tau_form, rep=0, seed=1000 + e) for e in range(n_events)]
    return gl, pl


def run_batch(fp64_launch):
    """FP32 events batched (one launch per kernel and step over all events, graph-replayed)
    against FP64 and FP32 events run one at a time; initial conditions untimed."""
    import torch
    import paper_2303_05599_amd as cp
    gl32, pl = batch_events(cp.FP32)
    site_updates = sum(g["N"] ** 2 * 2 * g["N"] for g in gl32)
    pushes = 0
    b = cp.Batch(gl32, pl)
    t0 = time.perf_counter()
    b.init_mv()
    t_ic = time.perf_counter() - t0
    tune = b.tune(5)
    b.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run()
    b.sync()
    t_batch = time.perf_counter() - t0
    obs32 = [b.observables(e) for e in range(len(gl32))]
    launch = b.get_launch()
    b.close()

    def plain(precision, launch=None):
        gl, _ = batch_events(precision)
        total, last = 0.0, []
        for g, p in zip(gl, pl):
            ctx = cp.Context(g, p)
            ctx.init_mv()
            if launch:
                ctx.set_launch(launch["bx"], launch["by"], launch["xcd_remap"], launch["waves"],
                               launch["variant"])
            ctx.sync()
            t0 = time.perf_counter()
            ctx.evolve(1e9)
            ctx.sync()
            total += time.perf_counter() - t0
            last.append(ctx.observables()[-1])
            ctx.close()
        return total, last
    t64, obs64 = plain(cp.FP64, fp64_launch)
    t32p, _ = plain(cp.FP32)
    rel_pT = [abs(o32[-1, 1] / o64[1] - 1) for o32, o64 in zip(obs32, obs64)]
    rel_pL = [abs(o32[-1, 2] / o64[2] - 1) for o32, o64 in zip(obs32, obs64)]
    for g, p in zip(gl32, pl):
        a_fm = g["L_fm"] / g["N"]
        n_form = math.ceil(p["tau_form_fm"] / (0.125 * a_fm) - 1e-9)
        pushes += p["n"] * (2 * g["N"] - n_form)
    n = len(gl32)
    return {"workload": f"{n} MV events, N in {{128,256,384,512}}, L=6 fm, 2N steps, 50 sheets, "
                        "1e4..1e5 beauty quarks each (pT 0..5 GeV), FP32 with reunitarisation every 16 steps",
            "events_per_s_fp32_batched": n / t_batch, "events_per_s_fp64_plain": n / t64,
            "events_per_s_fp32_plain": n / t32p,
            "speedup_fp32_batched_vs_fp64_plain": t64 / t_batch,
            "site_updates_per_s_fp32_batched": site_updates / t_batch,
            "pushes_per_s_fp32_batched": pushes / t_batch,
            "seconds": {"fp32_batched": t_batch, "fp64_plain": t64, "fp32_plain": t32p, "batch_ic": t_ic},
            "dpT2_rel_err_fp32_batched_vs_fp64": {"max": max(rel_pT), "mean": float(np.mean(rel_pT))},
            "dpL2_rel_err_fp32_batched_vs_fp64": {"max": max(rel_pL), "mean": float(np.mean(rel_pL))},
            "launch": launch, "tuner_choice": tune.strip().splitlines()[-1]}


def cpu_baseline(n_steps=6, n_part=100_000):
    """The oracle on the host cores: 512^2 MV event (one colour sheet; the
    initial condition is not timed), n_steps leapfrog steps with the push of
    n_part charm quarks active from the first step."""
    import oracle
    N, L = 512, 6.0
    a = oracle.lattice_spacing(L, N)
    st = oracle.mv_initial_condition(N, L, 2.0, 0.2, 10.0, 1, 3)
    P = oracle.particles_init(N, n_part, 4, 0.0, 0.0, True, 0)
    run = oracle.Run(N, 0.125, st, P, mhat=1.27 * a, n_form=0)
    run.step()      # n = 0 (no kick), untimed
    t0 = time.perf_counter()
    for _ in range(n_steps):
        run.step()
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=N * N * n_steps / dt, unit="site-updates/s", cores=cores, kind="oracle",
                pushes_per_s=n_part * n_steps / dt,
                sample=f"512^2 MV event (1 sheet, IC untimed), {n_steps} steps incl. push of {n_part} charm quarks, "
                       f"{dt:.1f} s wall")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=512)
    ap.add_argument("--warmup", type=int, default=96)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true", help="skip the FP32 and batched runs")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64",
                    help="precision of the headline run (profiling)")
    ap.add_argument("--tune-report", default=None, help="write the launch tuner's table to this file")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy (reference for the HBM counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(4):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 256 << 20, "copy_bytes_written": 256 << 20, "launches": 4}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (events shard across GPUs "
              f"without communication, see the design notes)", file=sys.stderr)
        sys.exit(2)
    if args.warmup + args.steps > 1024:
        sys.exit("warmup + steps must not exceed the 1024 steps to tau = 1.5 fm/c")
    import torch
    import paper_2303_05599_amd as cp
    torch.cuda.set_device(0)
    V = 512 * 512
    res = run_event(cp.FP64 if args.precision == "fp64" else cp.FP32, args.steps, args.warmup)
    tm = res["timing"]
    ms_per_step = res["wall"] * 1e3 / args.steps
    site_rate = V * args.steps / res["wall"]
    push_rate = 100_000 * args.steps / res["wall"]
    field_avg_s = tm["field_ms"] / max(tm["n_field"], 1) * 1e-3
    push_avg_s = tm["push_ms"] / max(tm["n_push"], 1) * 1e-3
    achieved = BYTES_PER_SITE["f64"] * V / field_avg_s / 1e9
    out = {
        "metric": "site-updates/s + particle-pushes/s at 512^2, % HBM peak; FP32-batched vs FP64",
        "value": site_rate,
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "MV Glasma 512^2, L=6 fm, g2mu=2 GeV, 50 sheets, dtau=a/8, 1e5 charm quarks "
                               "(m=1.27 GeV, pT=0, tau_form=0.1 fm/c), FP64",
                   "lattice": 512, "particles": 100_000, "precision": "fp64"},
        "pushes_per_s": push_rate,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "field_step_kernel<double>", "avg_launch_us": field_avg_s * 1e6,
                     "bytes_per_launch": BYTES_PER_SITE["f64"] * V},
        "push_kernel": {"avg_launch_us": push_avg_s * 1e6, "pushes_per_s_kernel": 100_000 / push_avg_s},
        "graph_ms_per_step": res["graph_ms_per_step"],
        "launch": res["launch"],
        "ic_seconds": res["t_ic"],
        "gauss_max": res["diag"][1], "unitarity_max": res["diag"][6],
        "dpT2_GeV2_last": float(res["obs"][-1, 1]), "dpL2_GeV2_last": float(res["obs"][-1, 2]),
    }
    if not args.no_extras:
        r32 = run_event(cp.FP32, args.steps, args.warmup)
        t32 = r32["timing"]
        f32_avg = t32["field_ms"] / max(t32["n_field"], 1) * 1e-3
        out["fp32"] = {"site_updates_per_s": V * args.steps / r32["wall"],
                       "pushes_per_s": 100_000 * args.steps / r32["wall"],
                       "ms_per_step": r32["wall"] * 1e3 / args.steps,
                       "field_avg_launch_us": f32_avg * 1e6,
                       "field_GBs": BYTES_PER_SITE["f32"] * V / f32_avg / 1e9,
                       "field_frac_hbm": BYTES_PER_SITE["f32"] * V / f32_avg / 1e9 / HBM_PEAK_GBS,
                       "push_avg_launch_us": t32["push_ms"] / max(t32["n_push"], 1) * 1e3,
                       "launch": r32["launch"],
                       "dpT2_rel_vs_fp64": float(abs(r32["obs"][-1, 1] / res["obs"][-1, 1] - 1)),
                       "dpL2_rel_vs_fp64": float(abs(r32["obs"][-1, 2] / res["obs"][-1, 2] - 1))}
        out["batch"] = run_batch(res["launch"])
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    if args.tune_report:
        with open(args.tune_report, "w") as f:
            f.write(res["tune_report"])
    print(json.dumps(out))


if __name__ == "__main__":
    main()
