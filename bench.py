"""Benchmark of the CPIC hot path on one MI355X.

Workload (the N=1 line): one synthetic MV-model Glasma event on a 512^2
lattice, L = 6 fm, g^2 mu = 2 GeV, m = 0.2 GeV, Lambda = 10 GeV, 50 colour
sheets, dtau = a/8 (1024 steps to 1.5 fm/c), with 1e5 charm quarks
(m = 1.27 GeV, p_T = 0, formed at 0.1 fm/c), double precision.  A step is one
leapfrog update of the fields plus the push of every formed particle plus
the broadening sums.  Untimed, in this order: the initial condition (built on
the GPU); max(W, n_form + 1) warm-up steps, so that every later step pushes
the particles; the launch tuner; a kernel-timing stretch (eager launches with
HIP events attached to every kernel: the per-kernel times of the roofline
entries); the capture of the step graphs and an alignment of the start to
four steps before a particle reordering (every 16 steps), so that K = 20
steps hold one reordering and K = 16 m + 4 hold m + 1.  Timed: K steps of the
production path (cpic_evolve: the library's HIP graphs, one per stretch
between reorderings, all captured before the timed region) and the
readout of the broadening samples (their fixed-order reduction and copy to
the host), with synchronisation on both sides.

Extra keys report the same event in single precision (reunitarisation every
16 steps), the jets workload (the same event in single precision with 1e6
near-light-like quarks and the light-like path integral of Sec. V.B) and
the batched multi-event mode; the CPU oracle is timed on a bounded sample of
the same workload on the host cores.
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
# Algorithmic bytes per unit of work (per site-update of the field kernel, per
# particle push): the field update reads and writes the 68 reals of a site
# (U_x, U_y, phi, E_x, E_y, pi); the push moves its record (about 17 words
# each way), the six force fields at one site (48 reals), phi at the cell (8)
# and a link on one step in eight.  The library keeps only the first two rows
# of each link (12 of its 18 reals), so its field update moves 56 + 56 reals
# of state per site: that figure is reported beside the full-link one.
SITE_BYTES = {"f64": 68 * 2 * 8, "f32": 68 * 2 * 4}
SITE_BYTES_TWO_ROW = {"f64": 56 * 2 * 8, "f32": 56 * 2 * 4}
PUSH_BYTES = {"f64": 730, "f32": 370}
# light-like paths, per path and step: the Wilson line (18 reals) read, the
# three integrated forces (24 reals) read and written, the x link crossed
# (once per 1/dt steps, counted every step: 12 reals of its two rows) and
# the five force-table vectors at the path's cell (40 reals)
JET_BYTES = {"f64": 118 * 8, "f32": 118 * 4}
# force table, per site: the two links (24 reals of their rows), phi (8), E
# and pi at both half steps (48) read; the six field vectors (48) written
TABLE_BYTES = {"f64": 128 * 8, "f32": 128 * 4}
SORT_EVERY = 16          # steps between reorderings of moving particles (the library's constant)
WATCH_EVERY = 64         # steps between the drift watchdog's checks (the library's default)
DTAU_FM = 0.125 * 6.0 / 512
# SU(2) variant: a site holds 20 reals (two quaternion links, phi, E_x, E_y,
# pi), read and written once; a push moves its record (13 words each way: the
# SU(2) columns), the six force fields at one site (18 reals), phi at the cell
# (3) and a link (4 reals) every eighth step
SITE_BYTES_SU2 = {"f64": 20 * 2 * 8, "f32": 20 * 2 * 4}
PUSH_BYTES_SU2 = {"f64": (26 + 18 + 3 + 0.5) * 8, "f32": (26 + 18 + 3 + 0.5) * 4}
# calibrated HBM counter readings per workload (rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE)
PMC_SUMMARIES = {w: os.path.join(ROOT, "profiles", f"pmc_{w}.txt")
                 for w in ("512_fp64", "512_fp32", "jets_512_fp32", "su2_512_fp64", "color_log_512_fp64")}
KERNEL_SOURCES = os.path.join(ROOT, "paper_2303_05599_amd", "csrc")


def glasma_512(precision, N=512, L=6.0, seed=3, n_colors=3):
    return dict(N=N, L_fm=L, g2mu_GeV=2.0, m_ir_GeV=0.2, uv_GeV=10.0, n_sheets=50, dtau_over_a=0.125,
                tau_max_fm=1.5, seed=seed, precision=precision, reunit_every=16, record_every=8, n_colors=n_colors)


def charm(n=100_000, seed=4, color_update=0):
    return dict(n=n, mass_GeV=1.27, pT_min_GeV=0.0, pT_max_GeV=0.0, azimuth_uniform=1, tau_form_fm=0.1, rep=0,
                seed=seed, color_update=color_update)


def jet_quarks(n=1_000_000, seed=4):
    """Near-light-like quarks: m = 0.01 GeV, p_T = 10 GeV, uniform azimuth, formed at tau = 0."""
    return dict(n=n, mass_GeV=0.01, pT_min_GeV=10.0, pT_max_GeV=10.0, azimuth_uniform=1, tau_form_fm=0.0, rep=0,
                seed=seed)


def formation_step(particles):
    """n_form = ceil(tau_form / dtau) at 512^2, as the library rounds it."""
    f = particles["tau_form_fm"] / DTAU_FM
    return math.ceil(f - 1e-9 * f)


def plan_steps(steps, warmup, n_form, n_max=1024):
    """Untimed steps before the timed region: the warm-up (at least up to the
    first push step), the kernel-timing stretch (up to 128 steps) and the
    graph and alignment steps (at most 2 x 15 + 35 + 48; see run_event)."""
    w = max(warmup, n_form + 1)
    spare = n_max - w - steps - 114
    if spare < 16:
        sys.exit(f"--steps {steps} with a warm-up of {w} steps (past formation at step {n_form}) leaves no room for "
                 f"the kernel-timing stretch within the {n_max} steps to tau = 1.5 fm/c")
    return w, min(128, spare)


def run_event(precision, steps, warmup, tune=True, particles=None, jets=False, n_colors=3, fixed=None, nt=None,
              push=None):
    """One 512^2 event: IC (timed separately), warm-up steps at least to the
    first push step, the launch tuner, a kernel-timing stretch (eager launches
    with HIP events attached to each kernel: the per-kernel times of the
    roofline entries), graph capture and alignment, then the timed region:
    `steps` steps of the production path (the HIP graphs of cpic_evolve)
    and the readout of the samples.  The timed region comes
    last, so a profiler's last `steps` dispatches of each kernel are exactly
    the timed ones."""
    import torch
    import paper_2303_05599_amd as cp
    p = particles or charm()
    ctx = cp.Context(glasma_512(precision, n_colors=n_colors), p)
    if jets:
        ctx.enable_jets(x_offset=0.3)
    if push is not None:
        ctx.set_push_mode(cp.PUSH_TILE if push == "tile" else cp.PUSH_GATHER)
    t0 = time.perf_counter()
    ctx.init_mv()
    t_ic = time.perf_counter() - t0
    w, n_kt = plan_steps(steps, warmup, formation_step(p))
    ctx.step(w)
    ctx.sync()
    if fixed:
        ctx.set_launch(fixed[0], fixed[1], 1, 1, 3)
        tune_report = f"fixed compressed-tile launch {fixed[0]}x{fixed[1]}\n"
    else:
        tune_report = ctx.tune(5) if tune else "not tuned (library defaults)\n"
    if nt is not None:
        ctx.set_store_policy(nt)
    launch = ctx.get_launch()
    launch["logq"] = p.get("color_update", 0) == cp.COLOR_LOG
    launch["push_mode"] = {cp.PUSH_TABLE: "table", cp.PUSH_TILE: "tile"}.get(ctx.push_mode(), "gather")
    # kernel timing (eager launches); not the headline rate
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(n_kt)
    ctx.sync()
    eager_ms = (time.perf_counter() - t0) * 1e3 / n_kt
    tm = ctx.timing()
    if jets:
        tm.update(ctx.jets_timing())
    ctx.set_timing(False)
    # graph capture: cpic_evolve replays one graph per stretch between
    # reordering points (multiples of 16).  The timed region starts four steps
    # before such a point; the same stretch pattern (4, 16, the remainder) is
    # run once untimed from the same alignment, which captures every graph the
    # timed region replays
    ctx.step((SORT_EVERY - 4 - ctx.n % SORT_EVERY) % SORT_EVERY)
    pre = steps if steps <= 4 + SORT_EVERY else 4 + SORT_EVERY + (steps - 4) % SORT_EVERY
    ctx.evolve((ctx.n + pre) * DTAU_FM * (1 - 1e-12))
    ctx.step((SORT_EVERY - 4 - ctx.n % SORT_EVERY) % SORT_EVERY)
    # a region shorter than the drift watchdog's interval starts where it holds
    # no check (one in WATCH_EVERY steps, about 40 us at this size): its rate
    # is then the steady one, as in a long region, where the checks amortise
    while steps < WATCH_EVERY and (ctx.n + steps) // WATCH_EVERY > ctx.n // WATCH_EVERY:
        ctx.step(SORT_EVERY)
    # the samples taken so far are summed now, so that the readout in the
    # timed region reduces only the samples of the timed steps
    ctx.observables()
    if jets:
        ctx.jet_observables()
    ctx.sync()
    untimed = ctx.n
    # timed region: the production path and the readout of the samples
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.evolve((ctx.n + steps) * DTAU_FM * (1 - 1e-12))
    obs = ctx.observables()
    jobs = ctx.jet_observables() if jets else None
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    d = ctx.diagnostics()
    transport = ctx.transport()
    jet_transport = ctx.jet_transport() if jets else None
    ctx.close()
    return dict(wall=wall, t_ic=t_ic, timing=tm, diag=d, obs=obs, jet_obs=jobs, eager_ms_per_step=eager_ms,
                transport=transport, jet_transport=jet_transport,
                kernel_timing_steps=n_kt, launch=launch, tune_report=tune_report, untimed_steps=untimed,
                warmup_steps=w)


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
    """FP32 events batched (one launch per kernel and step over the events of a launch group,
    graph-replayed; the library's default two launch lanes run groups side by side) against
    FP64 and FP32 events run one at a time; initial conditions untimed."""
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
            "speedup_fp32_batched_vs_fp32_plain": t32p / t_batch,
            "speedup_fp32_batched_vs_fp64_plain": t64 / t_batch,
            "site_updates_per_s_fp32_batched": site_updates / t_batch,
            "pushes_per_s_fp32_batched": pushes / t_batch,
            "seconds": {"fp32_batched": t_batch, "fp64_plain": t64, "fp32_plain": t32p, "batch_ic": t_ic},
            "dpT2_rel_err_fp32_batched_vs_fp64": {"max": max(rel_pT), "mean": float(np.mean(rel_pT))},
            "dpL2_rel_err_fp32_batched_vs_fp64": {"max": max(rel_pL), "mean": float(np.mean(rel_pL))},
            "launch": launch, "tuner_choice": tune.strip().splitlines()[-1]}


def run_jets(steps, warmup, V, tune=True, fixed=None):
    """The jets workload: the 512^2 event in FP32 with 1e6 near-light-like quarks
    and the light-like path integral over all 512^2 starting sites (the
    limit the quarks are compared with); the same timed region as the
    headline run."""
    import paper_2303_05599_amd as cp
    n_part = 1_000_000
    r = run_event(cp.FP32, steps, warmup, tune, jet_quarks(n_part), jets=True, fixed=fixed)
    k = rooflines(r, "fp32", n_part, V, "jets_512_fp32")
    last, lj = r["obs"][-1], r["jet_obs"][-1]
    return {"workload": "MV Glasma 512^2 (as above) in FP32 with reunitarisation every 16 steps, 1e6 quarks "
                        "m=0.01 GeV, pT=10 GeV, uniform azimuth, formed at tau=0, plus one light-like path "
                        "along +x per site",
            "ms_per_step": r["wall"] * 1e3 / steps,
            "site_updates_per_s": V * steps / r["wall"],
            "pushes_per_s": n_part * steps / r["wall"],
            "path_steps_per_s": V * steps / r["wall"],
            "eager_ms_per_step": r["eager_ms_per_step"],
            "kernels": k, "launch": r["launch"],
            "tau_fm": float(last[0]),
            "quarks_GeV2": {"dpT2": float(last[1]), "dpL2": float(last[2]), "dp_par2": float(last[3]),
                            "dp_perp2": float(last[4]),
                            # the library's transport export (cpic_transport)
                            "anisotropy_L_over_T": float(r["transport"][-1, 6]),
                            "kappa_T_GeV2_c_per_fm": float(r["transport"][-1, 1]),
                            "kappa_L_GeV2_c_per_fm": float(r["transport"][-1, 2])},
            "light_like_GeV2": {"dpx2": float(lj[1]), "dpy2": float(lj[2]), "dpz2": float(lj[3]),
                                "anisotropy_z_over_y": float(r["jet_transport"][-1, 5]),
                                "qhat_y_GeV2_c_per_fm": float(r["jet_transport"][-1, 2]),
                                "qhat_z_GeV2_c_per_fm": float(r["jet_transport"][-1, 3])}}


def run_color_log(steps, warmup, V, ref=None, tune=True):
    """The headline event with the alternative colour update of Sec. III.B
    (charges stepped by dQ/dt = i[Q, A.v] with A from the matrix logarithm of
    the links) over the same timed region; its broadening next to the
    rotation's."""
    import paper_2303_05599_amd as cp
    n_part = 100_000
    r = run_event(cp.FP64, steps, warmup, tune, charm(n_part, color_update=cp.COLOR_LOG))
    k = rooflines(r, "fp64", n_part, V, "color_log_512_fp64")
    out = {"workload": "the headline event (FP64) with the charges updated from the matrix logarithm of the links",
           "ms_per_step": r["wall"] * 1e3 / steps,
           "pushes_per_s": n_part * steps / r["wall"],
           "push_kernel": k["push"], "launch": r["launch"],
           "casimir_q2_max_drift": float(r["diag"][8])}
    if ref is not None:
        out["dpT2_rel_vs_rotation"] = float(r["obs"][-1, 1] / ref["obs"][-1, 1] - 1)
        out["dpL2_rel_vs_rotation"] = float(r["obs"][-1, 2] / ref["obs"][-1, 2] - 1)
    return out


def run_su2(steps, warmup, V):
    """The headline event and charm quarks in the SU(2) variant (links as
    quaternions, Darboux charges), FP64, the same timed region."""
    import paper_2303_05599_amd as cp
    n_part = 100_000
    r = run_event(cp.FP64, steps, warmup, False, charm(n_part), n_colors=2)
    tm = r["timing"]
    pmc = read_pmc_summary(PMC_SUMMARIES["su2_512_fp64"])
    out = {"workload": "MV Glasma 512^2 as the headline event, gauge group SU(2), 1e5 charm quarks, FP64",
           "ms_per_step": r["wall"] * 1e3 / steps,
           "site_updates_per_s": V * steps / r["wall"],
           "pushes_per_s": n_part * steps / r["wall"], "kernels": {}}
    for key, ms, k, unit_bytes, units, name in (
            ("field", tm["field_ms"], tm["n_field"], SITE_BYTES_SU2["f64"], V, "su2_field_kernel<double>"),
            ("push", tm["push_ms"], tm["n_push"], PUSH_BYTES_SU2["f64"], n_part, "su2_push_kernel<double>")):
        secs = ms / max(k, 1) * 1e-3
        ach = unit_bytes * units / secs / 1e9
        out["kernels"][key] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": ach / HBM_PEAK_GBS, "traffic": None, "kernel": name,
                               "avg_launch_us": secs * 1e6, "bytes_per_unit": unit_bytes, "units_per_launch": units}
        if pmc and name in pmc:
            fe, wr = pmc[name]
            out["kernels"][key].update(traffic=fe + wr, traffic_read=fe, traffic_written=wr)
    out["dpT2_GeV2_last"] = float(r["obs"][-1, 1])
    out["gauss_max"] = float(r["diag"][1])
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads():
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        return int(env)
    return len(os.sched_getaffinity(0))


def oracle_rates(N, st, P, mhat, steps, threads):
    """Site-updates/s and pushes/s of the oracle over `steps` steps (the first,
    n = 0, untimed) on `threads` OpenMP threads, field step and push timed apart."""
    import oracle
    oracle.set_threads(threads)
    run = oracle.Run(N, 0.125, st, P, mhat=mhat, n_form=0)
    run.step()
    run.t_field = run.t_push = 0.0
    for _ in range(steps):
        run.step()
    wall = run.t_field + run.t_push
    return {"threads": threads, "steps": steps, "seconds": wall,
            "site_updates_per_s": N * N * steps / wall, "pushes_per_s": P.shape[0] * steps / wall,
            "field_s_per_step": run.t_field / steps, "push_s_per_step": run.t_push / steps,
            "field_GBps_at_1088B": N * N * 1088 / (run.t_field / steps) / 1e9,
            "push_GBps_at_730B": P.shape[0] * 730 / (run.t_push / steps) / 1e9}


def cpu_baseline(n_steps=40, n_steps_single=2, n_part=100_000):
    """The oracle on the host cores.  The headline value is the 512^2 event
    with 1e5 charm quarks (config 2; one colour sheet for the untimed initial
    condition, the push active from the first step) over n_steps steps on all
    cores.  The table adds one thread against all cores for config 2 (a
    shorter sample) and for the whole config 1 run (32^2, 43 steps, 1024
    static quarks), each with the field step and the push timed apart."""
    import oracle
    cores = host_threads()
    N, L = 512, 6.0
    a = oracle.lattice_spacing(L, N)
    st = oracle.mv_initial_condition(N, L, 2.0, 0.2, 10.0, 1, 3)
    P = oracle.particles_init(N, n_part, 4, 0.0, 0.0, True, 0)
    all2 = oracle_rates(N, st, P, 1.27 * a, n_steps, cores)
    one2 = oracle_rates(N, st, P, 1.27 * a, n_steps_single, 1)
    st1 = oracle.mv_initial_condition(32, 6.0, 2.0, 0.2, 10.0, 1, 1)
    P1 = oracle.particles_init(32, 1024, 2, 0.0, 0.0, True, 0)
    all1 = oracle_rates(32, st1, P1, math.inf, 42, cores)
    one1 = oracle_rates(32, st1, P1, math.inf, 42, 1)
    oracle.set_threads(cores)
    return dict(value=all2["site_updates_per_s"], unit="site-updates/s", cores=cores, kind="oracle",
                pushes_per_s=all2["pushes_per_s"], cpu_model=cpu_model(),
                sample=f"512^2 MV event (1 sheet, IC untimed), {n_steps} steps incl. push of {n_part} charm quarks, "
                       f"{all2['seconds']:.1f} s on {cores} threads",
                table={"config2_512_fp64_1e5_charm": {"all_cores": all2, "one_thread": one2},
                       "config1_32_fp64_1024_static": {"all_cores": all1, "one_thread": one1}})


def _rms_rel(a, ref):
    a, ref = np.asarray(a, dtype=np.float64), np.asarray(ref, dtype=np.float64)
    return float(np.sqrt(np.mean((a - ref) ** 2) / np.mean(ref ** 2)))


def cpu_baseline_fp32_accuracy(n_compare=2000):
    """The oracle side of the single-precision accuracy keys (part of the
    CPU-baseline leg, the only leg that runs the oracle).  The oracle pushes
    the first n_compare particles of an event (particles are independent given
    the fields), from its own initial condition of the same seeds; the GPU
    records of the same particles give the same broadening sums.

    (a) The batch's first two 128^2 events (FP32, batched), to their end.
    (b) Error growth: the FP32 charm setup of the headline (m = 1.27 GeV,
        pT = 0, formed at 0.1 fm/c, 50 sheets, reunitarisation and charge
        renormalisation every 16 steps) on a 128^2 lattice, L = 6 fm, to
        1.5 fm/c (256 steps), the errors after 32, 64, 128, 256 steps, with
        the FP64 GPU path beside it.  (512^2 is beyond the oracle's budget
        here: 67 M site-updates per 256 steps.)"""
    import oracle
    import paper_2303_05599_amd as cp
    oracle.set_threads(host_threads())

    def oracle_event(g, p, n_compare):
        N, L = g["N"], g["L_fm"]
        a = oracle.lattice_spacing(L, N)
        st = oracle.mv_initial_condition(N, L, g["g2mu_GeV"], g["m_ir_GeV"], g["uv_GeV"], g["n_sheets"], g["seed"])
        P = oracle.particles_init(N, p["n"], p["seed"], p["pT_min_GeV"] * a, p["pT_max_GeV"] * a, True, 0)
        f = p["tau_form_fm"] / (0.125 * L / N)
        n_form = math.ceil(f - 1e-9 * f)  # as the library rounds the formation step
        return oracle.Run(N, 0.125, st, P[:n_compare], mhat=p["mass_GeV"] * a, n_form=n_form), a

    def errors(run, a, recs, state=None):
        k = recs.shape[0]
        ref = run.observe() / (k * a * a)
        got = oracle.particles_observe(run.n * 0.125, run.mhat, False, recs) / (k * a * a)
        e = {"dpT2_rel_err": float(abs(got[0] / ref[0] - 1)), "dpL2_rel_err": float(abs(got[1] / ref[1] - 1)),
             "momentum_rms_rel_err": _rms_rel(recs[:, 3:6], run.P[:, 3:6]),
             "dpT2_GeV2": float(ref[0]), "dpL2_GeV2": float(ref[1])}
        if state is not None:
            e["E_rms_rel_err"] = _rms_rel(state["E"], run.st["E"])
            e["U_rms_rel_err"] = _rms_rel(state["U"].view(np.float64), run.st["U"].view(np.float64))
        return e

    t0 = time.perf_counter()
    gl32, pl = batch_events(cp.FP32)
    idx = [e for e in range(len(gl32)) if gl32[e]["N"] == 128][:2]
    b = cp.Batch([gl32[e] for e in idx], [pl[e] for e in idx])
    b.init_mv()
    b.run()
    b.sync()
    batch = []
    for j, e in enumerate(idx):
        g, p = gl32[e], pl[e]
        recs = b.get_state(j, cp.STATE_PARTICLES, (p["n"], 20))[:n_compare]
        run, a = oracle_event(g, p, n_compare)
        for _ in range(b.n(j)):
            run.step()
        batch.append(dict(event=e, steps=run.n, **errors(run, a, recs)))
    b.close()

    N, L = 128, 6.0
    g = dict(N=N, L_fm=L, g2mu_GeV=2.0, m_ir_GeV=0.2, uv_GeV=10.0, n_sheets=50, dtau_over_a=0.125, tau_max_fm=1.5,
             seed=7, reunit_every=16, record_every=8)
    p = charm(10_000)
    ctxs = {prec: cp.Context(dict(g, precision=prec), p) for prec in (cp.FP32, cp.FP64)}
    for c in ctxs.values():
        c.init_mv()
    run, a = oracle_event(g, p, n_compare)
    growth = []
    for k in (32, 64, 128, 256):  # (the quarks form at step 18)
        while run.n < k:
            run.step()
        row = {"steps": k, "tau_fm": k * 0.125 * L / N}
        for prec, c in ctxs.items():
            c.step(k - c.n)
            recs = c.get_state(cp.STATE_PARTICLES)[:n_compare]
            row["fp32" if prec == cp.FP32 else "fp64"] = errors(run, a, recs, c.state())
        growth.append(row)
    for c in ctxs.values():
        c.close()
    return {"batch_fp32_vs_oracle_128": {"events": batch, "particles_compared": n_compare,
                                         "dpT2_rel_err_max": max(r["dpT2_rel_err"] for r in batch),
                                         "dpL2_rel_err_max": max(r["dpL2_rel_err"] for r in batch)},
            "error_growth_fp32_vs_oracle": {"workload": "the headline's FP32 charm setup on 128^2 (L = 6 fm, 50 "
                                                        "sheets, 1e4 quarks, the first 2000 compared)",
                                            "rows": growth},
            "seconds": time.perf_counter() - t0}


def kernel_source_hash():
    """sha256 over the device code (the translation units that define kernels,
    the headers except the host-side context, the compiler flags): a stored
    counter reading is only used for the kernels it was taken on."""
    import hashlib
    sys.path.insert(0, ROOT)
    from paper_2303_05599_amd import build as libbuild
    h = hashlib.sha256(" ".join(libbuild.FLAGS[:-2]).encode())
    for name in sorted(os.listdir(KERNEL_SOURCES)):
        path = os.path.join(KERNEL_SOURCES, name)
        if not name.endswith((".hip", ".h")) or name == "ctx.h":
            continue
        with open(path, "rb") as f:
            data = f.read()
        if name.endswith(".hip") and b"__global__" not in data:
            continue  # host code only
        h.update(name.encode() + b"\0" + data)
    return h.hexdigest()


def read_pmc_summary(path):
    """kernel name -> (fetch bytes, write bytes) per dispatch, or None when the
    summary is missing or was taken on other kernel sources."""
    if not os.path.exists(path):
        return None
    d = {}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#") and "=" in line:
                k, v = line.split("=", 1)
                d[k.strip()] = v.strip()
    if d.get("source_sha256") != kernel_source_hash():
        return None
    out = {}
    for k, v in d.items():
        if k.endswith(".kernel"):
            key = k[:-len(".kernel")]
            out[v] = (float(d[key + ".fetch_bytes"]), float(d[key + ".write_bytes"]))
    return out


def kernel_names(launch, precision):
    t = "double" if precision == "fp64" else "float"
    v = launch["variant"]
    if v == 4:
        cp = 2 if launch.get("nt_store") else 0
        return (f"fused_kernel<{t}, {launch['bx']}, {launch['by']}, {cp}>", f"straggler_kernel<{t}>",
                f"jet_kernel<{t}>")
    if v == 3:
        cp = 2 if launch.get("nt_store") else 0
        field = f"field_ctile_kernel<{t}, {launch['bx']}, {launch['by']}, {cp}>"
    elif v == 2:
        field = f"field_tile_kernel<{t}, {launch['bx']}, {launch['by']}>"
    elif v == 1:
        field = "field_link_kernel" + ("" if launch["waves"] == 1 else f"_w{launch['waves']}") + f"<{t}>"
    else:
        field = "field_step_kernel" + ("" if launch["waves"] == 1 else f"_w{launch['waves']}") + f"<{t}>"
    if launch.get("push_mode") == "table":
        push = f"force_table_kernel<{t}> + push_table_kernel<{t}>"
    else:
        push = f"push_kernel<{t}, {launch['push_lanes']}, {'true' if launch.get('logq') else 'false'}>"
    return field, push, f"jet_kernel<{t}>"


def rooflines(res, precision, n_part, V, pmc_workload=None):
    """Per-kernel roofline entries from the live HIP-event kernel times; HBM
    traffic from the counter summary of `pmc_workload` where it holds the
    same kernel (a push shown as "a + b" adds both kernels' traffic)."""
    tm = res["timing"]
    dt = "f64" if precision == "fp64" else "f32"
    field_s = tm["field_ms"] / max(tm["n_field"], 1) * 1e-3
    push_s = tm["push_ms"] / max(tm["n_push"], 1) * 1e-3
    fname, pname, jname = kernel_names(res["launch"], precision)
    out = {}
    if res["launch"]["variant"] == 4:
        # the fused step: the tile kernel updates every site and pushes the
        # particles still in their tile; the straggler kernel pushes the rest
        # (counted on the device over the timed launches)
        strag = tm["straggler_pushes"] / max(tm["n_push"], 1)
        entries = [("fused", fname, field_s, SITE_BYTES[dt] * V + PUSH_BYTES[dt] * (n_part - strag), 1,
                    f"step ({V} site-updates at {SITE_BYTES[dt]} B + {n_part - strag:.0f} particle-pushes at "
                    f"{PUSH_BYTES[dt]} B)"),
                   ("stragglers", pname, push_s, PUSH_BYTES[dt], strag, "particle-push")]
    else:
        entries = [("field", fname, field_s, SITE_BYTES[dt], V, "site-update"),
                   ("push", pname, push_s, PUSH_BYTES[dt], n_part, "particle-push")]
    if tm.get("n_jets"):
        entries.append(("jets", jname, tm["jets_ms"] / tm["n_jets"] * 1e-3, JET_BYTES[dt], V, "path-step"))
    for key, name, secs, unit_bytes, units, unit in entries:
        bpl = unit_bytes * units
        ach = bpl / secs / 1e9
        out[key] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": ach / HBM_PEAK_GBS, "traffic": None, "kernel": name,
                    "avg_launch_us": secs * 1e6, "bytes_per_launch": bpl,
                    "bytes_per_unit": unit_bytes, "units_per_launch": units, "work_unit": unit}
    if "ctile" in fname:
        # the same launch priced with the two-row link storage it works on
        two = SITE_BYTES_TWO_ROW[dt] * V
        out["field"].update(bytes_per_unit_two_row_links=two // V, frac_two_row_links=two / field_s / 1e9 / HBM_PEAK_GBS)
    pmc = read_pmc_summary(PMC_SUMMARIES[pmc_workload or "512_" + precision])
    for e in out.values():
        parts = e["kernel"].split(" + ")
        if pmc and all(k in pmc for k in parts):
            fe, wr = sum(pmc[k][0] for k in parts), sum(pmc[k][1] for k in parts)
            e.update(traffic=fe + wr, traffic_read=fe, traffic_written=wr)
    return out


def pmc_summary(out_path, fetch_dirs, write_dirs, copy_fetch_dir, copy_write_dir, command, title):
    """Condense rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE of a bench workload,
    comma-separated directories when several launch shapes were profiled, and
    of the 256 MiB copy) into the key = value summary read above: every field,
    push and light-like kernel with at least 16 dispatches, by name."""
    import csv
    import glob

    def per_kernel(dirs, counter):
        # per kernel, the dispatches of the run in which it ran most often: a
        # run with a fixed tile also runs the default tile in its warm-up
        kern = {}
        for d in dirs.split(","):
            by, run = {}, {}
            for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
                for r in csv.DictReader(open(f)):
                    if r["Counter_Name"] == counter:
                        key = (r["Kernel_Name"], int(r["Dispatch_Id"]))
                        by[key] = by.get(key, 0.0) + float(r["Counter_Value"])
            for (name, _), v in sorted(by.items(), key=lambda kv: kv[0][1]):
                run.setdefault(short(name), []).append(v)
            for name, v in run.items():
                if len(v) > len(kern.get(name, [])):
                    kern[name] = v
        return kern

    def short(name):
        return name.replace("void ", "").replace("cpic::", "").split("(")[0]

    cf, cw = per_kernel(copy_fetch_dir, "FETCH_SIZE"), per_kernel(copy_write_dir, "WRITE_SIZE")
    copy_kernel = max(cf, key=lambda k: max(cf[k]))
    copy_bytes = 256 << 20
    f_fetch = copy_bytes / (max(cf[copy_kernel]) * 1024)
    f_write = copy_bytes / (max(cw[copy_kernel]) * 1024)
    kf, kw = per_kernel(fetch_dirs, "FETCH_SIZE"), per_kernel(write_dirs, "WRITE_SIZE")
    lines = [f"# rocprofv3 PMC summary: HBM traffic per dispatch, {title}.",
             "# FETCH_SIZE and WRITE_SIZE (KiB per dispatch, mean of the last 16 dispatches of each",
             "# kernel: the timed region) are scaled by the ratio of the bytes a 256 MiB device copy",
             "# moves to what the same counters read for it.",
             "# commands (from /tmp, TMPDIR=/tmp; R = repository root):"]
    lines += ["#   " + c.strip() for c in command.split(";")]
    lines += [f"source_sha256 = {kernel_source_hash()}",
              f"copy_kernel = {copy_kernel}",
              f"copy_fetch_kib = {max(cf[copy_kernel]):.1f}", f"copy_write_kib = {max(cw[copy_kernel]):.1f}",
              f"copy_fetch_factor = {f_fetch:.4f}", f"copy_write_factor = {f_write:.4f}"]
    i = 0
    for name in sorted(kf):
        if not any(p in name for p in ("field_", "push_", "force_table", "jet_kernel", "fused_", "straggler_")) \
                or "diag" in name:
            continue
        if len(kf[name]) < 16 or len(kw.get(name, [])) < 16:
            continue
        fe, wr = kf[name][-16:], kw[name][-16:]
        fkib, wkib = sum(fe) / 16, sum(wr) / 16
        lines += [f"k{i}.kernel = {name}", f"k{i}.fetch_kib = {fkib:.1f}", f"k{i}.write_kib = {wkib:.1f}",
                  f"k{i}.fetch_bytes = {fkib * 1024 * f_fetch:.0f}",
                  f"k{i}.write_bytes = {wkib * 1024 * f_write:.0f}"]
        i += 1
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def trace_summary(out_path, trace_dir, command, last, top=12):
    """Markdown table of a rocprofv3 --kernel-trace --stats run, with the mean
    over each kernel's last `last` dispatches (the bench's timed region)."""
    import csv
    import glob
    f = glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True)[0]
    rows = list(csv.DictReader(open(f)))
    durs = {}
    for tf in glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True):
        for r in csv.DictReader(open(tf)):
            durs.setdefault(r["Kernel_Name"], []).append(
                (int(r["Start_Timestamp"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    lines = ["# rocprofv3 kernel statistics", "", "Command (from /tmp, TMPDIR=/tmp; R = repository root):", "",
             "```", command, "```", "",
             f"`timed us` is the mean over the kernel's last {last} dispatches, which are the bench's timed steps.",
             "", "| kernel | calls | total ms | average us | timed us | % |", "|---|---|---|---|---|---|"]
    for r in rows[:top]:
        name = r["Name"].replace("void ", "").replace("cpic::", "").split("(")[0]
        d = sorted(durs.get(r["Name"], []))[-last:]
        timed = f"{sum(x for _, x in d) / len(d) / 1e3:.2f}" if d else "-"
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} | {timed} | {float(r['Percentage']):.1f} |")
    with open(out_path, "w") as fo:
        fo.write("\n".join(lines) + "\n")
    print("\n".join(lines))


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
    ap.add_argument("--pmc-summary", nargs=5, metavar=("OUT", "FETCH_DIRS", "WRITE_DIRS", "COPY_FETCH_DIR",
                                                       "COPY_WRITE_DIR"),
                    help="condense rocprofv3 --pmc output directories into a profiles/ summary (FETCH_DIRS and "
                         "WRITE_DIRS: comma-separated, one directory per profiled run)")
    ap.add_argument("--trace-summary", nargs=3, metavar=("OUT", "TRACE_DIR", "TIMED_STEPS"),
                    help="condense a rocprofv3 --kernel-trace --stats directory into a markdown table")
    ap.add_argument("--command", default="", help="command line recorded in a summary")
    ap.add_argument("--title", default="", help="workload named in a counter summary")
    ap.add_argument("--launch", nargs=2, type=int, metavar=("BX", "BY"), default=None,
                    help="fix the compressed-tile field launch instead of tuning (counter runs of a tuned shape)")
    ap.add_argument("--nt", type=int, choices=[0, 1], default=None,
                    help="fix the store policy of the field update's new state (1: non-temporal) after tuning")
    ap.add_argument("--jets-only", action="store_true",
                    help="run only the jets workload and print its JSON (for profiling; not the benchmark line)")
    ap.add_argument("--leg", choices=["su2", "color-log"], default=None,
                    help="run only the SU(2) or the colour-logarithm leg and print its JSON (for profiling; not "
                         "the benchmark line)")
    ap.add_argument("--push", choices=["tile", "gather"], default=None,
                    help="push mode before tuning (default: the library's; the tuner tries the fused step only "
                         "from the tile mode)")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the library's default launch shapes (for counter runs, where the tuner's timings "
                         "are distorted by the serialised dispatches)")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary, args.command, args.title)
        return
    if args.trace_summary:
        out, tdir, last = args.trace_summary
        trace_summary(out, tdir, args.command, int(last))
        return
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
    import torch
    import paper_2303_05599_amd as cp
    torch.cuda.set_device(0)
    V = 512 * 512
    n_part = 100_000
    if args.jets_only:
        print(json.dumps(run_jets(args.steps, args.warmup, V, not args.no_tune, args.launch)))
        return
    if args.leg == "su2":
        print(json.dumps(run_su2(args.steps, args.warmup, V)))
        return
    if args.leg == "color-log":
        print(json.dumps(run_color_log(args.steps, args.warmup, V, tune=not args.no_tune)))
        return
    res = run_event(cp.FP64 if args.precision == "fp64" else cp.FP32, args.steps, args.warmup, not args.no_tune,
                    fixed=args.launch, nt=args.nt, push=args.push)
    ms_per_step = res["wall"] * 1e3 / args.steps
    site_rate = V * args.steps / res["wall"]
    push_rate = n_part * args.steps / res["wall"]
    kern = rooflines(res, args.precision, n_part, V)
    dominant = max(kern, key=lambda k: kern[k]["avg_launch_us"])
    dt = "f64" if args.precision == "fp64" else "f32"
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
        "dtype": dt,
        "data": "synthetic",
        "config": {"workload": "MV Glasma 512^2, L=6 fm, g2mu=2 GeV, 50 sheets, dtau=a/8, 1e5 charm quarks "
                               f"(m=1.27 GeV, pT=0, tau_form=0.1 fm/c), {args.precision.upper()}",
                   "lattice": 512, "particles": n_part, "precision": args.precision},
        "pushes_per_s": push_rate,
        "roofline": dict(kern[dominant], dominant=dominant),
        "kernels": kern,
        "eager_ms_per_step": res["eager_ms_per_step"], "kernel_timing_steps": res["kernel_timing_steps"],
        "warmup_steps_run": res["warmup_steps"], "first_timed_step": res["untimed_steps"],
        "watchdog_checks_in_timed_region": (res["untimed_steps"] + args.steps) // WATCH_EVERY
                                           - res["untimed_steps"] // WATCH_EVERY,
        "watchdog_every": WATCH_EVERY,
        "timed_region": "K steps of cpic_evolve (HIP graphs of up to 16 steps between the particle reorderings "
                        "every 16 steps; the drift watchdog's checks every 64 steps) and the readout of the broadening samples (fixed-order reduction and copy to the host)",
        "launch": res["launch"],
        "ic_seconds": res["t_ic"],
        "gauss_max": res["diag"][1], "unitarity_max": res["diag"][6],
        "dpT2_GeV2_last": float(res["obs"][-1, 1]), "dpL2_GeV2_last": float(res["obs"][-1, 2]),
        "kappa_T_last": float(res["transport"][-1, 1]), "kappa_L_last": float(res["transport"][-1, 2]),
        "anisotropy_L_over_T_last": float(res["transport"][-1, 6]),
    }
    t_start = time.perf_counter()

    def progress(leg):
        print(f"bench: {leg} done at {time.perf_counter() - t_start:.0f} s", file=sys.stderr, flush=True)

    progress("headline FP64")
    if not args.no_extras:
        r32 = run_event(cp.FP32, args.steps, args.warmup)
        k32 = rooflines(r32, "fp32", n_part, V)
        out["fp32"] = {"site_updates_per_s": V * args.steps / r32["wall"],
                       "pushes_per_s": n_part * args.steps / r32["wall"],
                       "ms_per_step": r32["wall"] * 1e3 / args.steps,
                       "eager_ms_per_step": r32["eager_ms_per_step"],
                       "kernels": k32,
                       "launch": r32["launch"],
                       "dpT2_rel_vs_fp64": float(abs(r32["obs"][-1, 1] / res["obs"][-1, 1] - 1)),
                       "dpL2_rel_vs_fp64": float(abs(r32["obs"][-1, 2] / res["obs"][-1, 2] - 1))}
        progress("FP32")
        out["jets"] = run_jets(args.steps, args.warmup, V)
        progress("jets")
        out["color_log"] = run_color_log(args.steps, args.warmup, V, res)
        progress("colour logarithm")
        out["su2"] = run_su2(args.steps, args.warmup, V)
        progress("SU(2)")
        out["batch"] = run_batch(res["launch"])
        progress("batch")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
        progress("CPU baseline")
        if not args.no_extras:
            out["fp32_vs_oracle"] = cpu_baseline_fp32_accuracy()
            progress("FP32 against the oracle")
    if args.tune_report:
        with open(args.tune_report, "w") as f:
            f.write(res["tune_report"])
    print(json.dumps(out))


if __name__ == "__main__":
    main()
