"""Benchmark: timestep throughput of the Ohta-Kawasaki Newton-Krylov solve on
one MI355X.

A step is one timestep of the whole hot path (Newton residual, FGMRES with the
matching-Schur block preconditioner, Jacobian applies, updates) over the
configured synthetic field.  Prints ONE JSON line.

Default workload (the headline): 3D unit cube, Q1 hex on a uniform 256^3
mesh (16,974,593 nodes, 33,949,186 DOFs), eps=0.01, sigma=1000, m=0.1,
theta=1, dt=2e-5, u0 = m + 0.05*U(-1,1) seeded (seed 2), w0 = 0.  `value` is
the FP64 path's throughput; the mixed-precision form (FP32 preconditioner,
FP64 FGMRES, residual, Jacobian and M_E(u)) is timed beside it on the same
input, with its error against the FP64 path after every step, and so is
Newton with preconditioned MINRES on the symmetric rearrangement of the
Newton system (FP64; --linear-solver fgmres leaves it out).  All are
timed with no profiling events in the timed region; kernel-class rooflines
come from a profiled rerun of the same timesteps.  --config 3d128 (4.29M
DOFs) and 2d64 are the smaller cases of the same recipe.

Other workloads:
  --config sweep64  64 independent 2D instances, N uniform over
                    {128,256,512,1024}, eps~U[0.01,0.05], sigma~logU[10,1000],
                    m~U[-0.4,0.4], dt=eps^2/2 (seeds 4000+i), mixed precision,
                    one batched timestep against the sum of the 64 solo runs.
  --config robustness  the paper's robustness experiments (Sec. 4) on Q1:
                    Table 2 analogue (2D, eps in {0.02,0.01,0.005}, N = 2/eps,
                    dt = eps^2) and Table 1 analogue (3D N in {16..128}, eps =
                    0.02, dt = 4e-4), m = 0.4, sigma = 100, theta = 1/2, cosine
                    initial condition; average FGMRES iterations per Newton step
                    for the default solver and the paper's preset.
  --config paper    the paper's experiment (Sec. 4) on Q1: 3D N = --paper-n
                    (25*2^k; 100 by default, 400 = 129M DOFs), m = 0.4,
                    eps = 0.02, sigma = 100, theta = 1/2, dt = eps^2, cosine
                    initial condition, w0 from (okb), paper solver preset
                    (2 Richardson iterations of S~^-1, 5 V-cycles); --steps of
                    the T = 300 dt run.
  --config serve    256 resident simulations (70% 2D N in {256..2048}, 30% 3D
                    N in {64,128}; seeds 5000+s), one Poisson stream of
                    timestep requests (seed 5999) at --rates req/s for
                    --duration s each, mixed precision; p50/p99 latency
                    (arrival to done) and sustained DOFs/s.
"""
import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
TARGET_FRAC = 0.60     # roofline fraction asked of the stencil and V-cycle kernels
# kernel classes timed in the profiled region of the single-problem benchmark (ok.h)
K_CHEB_MASS, K_MG_SMOOTH, K_KRYLOV = 1, 2, 5
KERNELS = {
    K_KRYLOV: ("krylov", "Gram-Schmidt chain of one Arnoldi step of FGMRES; algorithmic bytes: "
                         "3 two-field vectors per projection (w and v_i read, w written), "
                         "i = 0..j",
               ("paper_1603_04570_amd/csrc/k_krylov.hip", "paper_1603_04570_amd/csrc/ok_internal.h",
                "paper_1603_04570_amd/csrc/engine.hip")),
    K_CHEB_MASS: ("cheb_pair", "Chebyshev-Jacobi iterations on M, two per launch (the autotuned "
                               "one of k_strip2/k_cheb2t/k_cheb2); algorithmic bytes: x, r, d "
                               "read and written once per launch (6 words/node)",
                  ("paper_1603_04570_amd/csrc/k_stencil_impl.h",
                   "paper_1603_04570_amd/csrc/k_strip2.h",
                   "paper_1603_04570_amd/csrc/ok_internal.h",
                   "paper_1603_04570_amd/csrc/engine.hip")),
    K_MG_SMOOTH: ("vcycle_smoother", "finest-level V-cycle smoothing passes (fused pre-smoothing + "
                                     "residual and fused post-smoothing, in FP64 strips with the "
                                     "coarse-grid correction interpolated in the same pass; the "
                                     "autotuned one of k_strip2/k_mg2t/k_mg2, or the one-iteration "
                                     "kernels); algorithmic bytes: 3 words/node per fused pass, "
                                     "plus the coarse correction (2^-d words/node) when folded",
                  ("paper_1603_04570_amd/csrc/k_stencil_impl.h",
                   "paper_1603_04570_amd/csrc/k_strip2.h",
                   "paper_1603_04570_amd/csrc/ok_internal.h",
                   "paper_1603_04570_amd/csrc/engine.hip")),
}


def stored_traffic(kernel_class, config):
    """HBM bytes per launch of a kernel class measured with hardware counters
    (profiles/<kernel>_<config>_traffic.txt), or None when there is no such
    record or the kernel sources changed since it was taken."""
    import hashlib
    tag, _, sources = KERNELS[kernel_class]
    path = os.path.join(ROOT, "profiles", f"{tag}_{config}_traffic.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if line.startswith("#") or ":" not in line:
            continue
        k, v = line.split(":", 1)
        rec[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in sources:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if rec.get("source_sha256") != h.hexdigest():
        return None
    return float(rec["traffic_bytes_per_dispatch"])


def roofline_of(P, kernel_class, config, fp64):
    launches, kms, kbytes = P.profile_read(kernel_class)
    if not launches:
        return None, 0.0
    avg_s = kms / launches * 1e-3
    per_launch = kbytes / launches
    ach = per_launch / avg_s / 1e9
    return ({"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": round(ach / HBM_PEAK_GBS, 4),
             "traffic": stored_traffic(kernel_class, config) if fp64 else None,
             "kernel": KERNELS[kernel_class][1], "bytes_per_launch": per_launch,
             "avg_us": round(avg_s * 1e6, 2), "launches": launches,
             "total_ms": round(kms, 3)}, kms)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def cpu_baseline(cfg, its_per_step, newton_per_step):
    """The FP64 CSR oracle on one host core, on a bounded sample of the same
    workload: one residual evaluation and `sample_its` FGMRES iterations of
    the first Newton solve of timestep 1 (assembly excluded, as setup is on
    the GPU), each timed, then scaled to one timestep of the GPU run:
    (Newton iterations + 1) residuals and its FGMRES iterations."""
    from oracle.okref import Oracle
    from paper_1603_04570_amd.inputs import dofs, noise_state
    dim, n = cfg["dim"], cfg["n"]
    sample_its = 1 if dofs(dim, n) > 10_000_000 else 4
    t_setup = time.perf_counter()
    o = Oracle(dim, n, cfg["eps"], cfg["sigma"], cfg["m"], cfg["dt"], cfg["theta"],
               gmres_restart=sample_its, gmres_max_restarts=0)
    t_setup = time.perf_counter() - t_setup
    u, w = noise_state(dim, n, cfg["m"], cfg["seed"])
    t0 = time.perf_counter()
    F, _ = o.residual(u, w, u)
    t_res = time.perf_counter() - t0
    t0 = time.perf_counter()
    x, its, st = o.fgmres(u, -F)
    t_fg = time.perf_counter() - t0
    per_it = t_fg / max(its, 1)
    step_s = (newton_per_step + 1.0) * t_res + its_per_step * per_it
    return {"value": dofs(dim, n) / step_s, "unit": "DOFs/s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle (serial FP64, assembled CSR) on {dim}D {n}^{dim}, the same "
                       f"workload and seed: one residual ({t_res:.2f} s) and {its} FGMRES "
                       f"iteration(s) of the first Newton solve ({t_fg:.1f} s), scaled to "
                       f"{newton_per_step + 1:.2f} residuals and {its_per_step:.2f} FGMRES "
                       f"iterations per timestep (the GPU run's averages); assembly "
                       f"{t_setup:.1f} s excluded; one thread on host {cpu_model()}, "
                       f"nproc {os.cpu_count()}")}


def calibrate_copy(torch, mib=1024, reps=5):
    """A plain elementwise copy (y = -x, FP64) of `mib` MiB: it reads and writes
    exactly that many bytes, so hardware byte counters of this kernel give the
    scale from counter units to bytes."""
    n = mib * 2**20 // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    torch.neg(x, out=y)  # load the kernel before timing
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        torch.neg(x, out=y)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "reps": reps,
                      "avg_ms": ms, "GBs": 2 * n * 8 / ms / 1e6}), flush=True)


def _params(ok, spec, precision):
    return ok.default_params(dim=spec["dim"], n=spec["n"], eps=spec["eps"], sigma=spec["sigma"],
                             m=spec["m"], dt=spec["dt"], theta=spec["theta"], precision=precision)


def _base_line(metric_value, steps, warmup, ms_per_step, dtype, config):
    return {"metric": "timestep DOFs/s", "value": metric_value, "unit": "DOFs/s", "n_gpus": 1,
            "steps": steps, "warmup": warmup, "ms_per_step": ms_per_step,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic", "config": config}


def bench_sweep(args, torch, ok):
    """Batched sweep: all 64 instances advance one timestep per step in
    grouped launches (classes by N on streams of their own, FGMRES iterations
    replayed from captured graphs), against the sum of the solo runs."""
    from paper_1603_04570_amd.inputs import dofs, noise_state, sweep_instance
    prec = ok.OK_FP64 if args.precision == "fp64" else ok.OK_MIXED
    specs = [sweep_instance(i) for i in range(64)]
    plist = [_params(ok, s, prec) for s in specs]
    init = [noise_state(s["dim"], s["n"], s["m"], s["seed"]) for s in specs]
    init = [(torch.from_numpy(u).cuda(), torch.from_numpy(w).cuda()) for u, w in init]
    B = ok.Batch(plist)
    tuned = 0 if args.no_autotune else B.autotune()

    def reset():
        for i, (u, w) in enumerate(init):
            B.set_state(i, u, w)
        torch.cuda.synchronize()

    reset()
    for _ in range(args.warmup):
        B.timestep(1)
    reset()
    t0 = time.perf_counter()
    st = B.timestep(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    total = sum(dofs(s["dim"], s["n"]) for s in specs)
    # the same instances one at a time (same launch mode, warm)
    solo = 0.0
    solo_its = []
    for i, s in enumerate(specs):
        P = ok.Problem(plist[i])
        P.use_graphs(True)
        u, w = init[i][0].clone(), init[i][1].clone()
        P.timestep(u, w, 1)  # warm: graphs captured, code loaded
        u.copy_(init[i][0])
        w.copy_(init[i][1])
        torch.cuda.synchronize()
        a = time.perf_counter()
        ss = P.timestep(u, w, args.steps)
        torch.cuda.synchronize()
        solo += time.perf_counter() - a
        solo_its.append(ss.its())
        assert ss.its() == st[i].its(), (i, ss.its(), st[i].its())
    fp64 = None
    if prec == ok.OK_MIXED:  # the same batch on the plain FP64 path
        B64 = ok.Batch([_params(ok, s, ok.OK_FP64) for s in specs])
        if not args.no_autotune:
            B64.autotune()
        for i, (u, w) in enumerate(init):
            B64.set_state(i, u, w)
        B64.timestep(1)
        for i, (u, w) in enumerate(init):
            B64.set_state(i, u, w)
        torch.cuda.synchronize()
        a = time.perf_counter()
        B64.timestep(args.steps)
        torch.cuda.synchronize()
        fp64 = time.perf_counter() - a
        B64.close()
    sizes = sorted({s["n"] for s in specs})
    out = _base_line(total * args.steps / elapsed, args.steps, args.warmup,
                     elapsed * 1e3 / args.steps, "f64" if prec == ok.OK_FP64 else "f64+f32",
                     {"workload": "sweep64: 64 x 2D Q1, N in {128,256,512,1024} (seeds 4000+i), "
                                  "eps~U[.01,.05], sigma~logU[10,1000], m~U[-.4,.4], "
                                  "dt=eps^2/2, theta=1",
                      "dofs": total, "instances": 64,
                      "instances_per_N": {str(n): sum(s["n"] == n for s in specs) for n in sizes},
                      "global_batch": 64, "parallelism": "none (1 GPU)"})
    out.update({"classes": B.classes(), "solo_sum_s": solo, "batched_s": elapsed,
                "vs_solo_sum": solo / elapsed, "autotuned_shapes": tuned,
                "fp64_batched_s": fp64, "vs_fp64_batched": (fp64 / elapsed) if fp64 else None,
                "fgmres_its_total": sum(sum(x.its()) for x in st), "roofline": None})
    return out


def bench_paper(args, torch, ok):
    """The paper's experiment on Q1, timed over --steps timesteps after one
    warm-up step (the state is reset to u0, w0 afterwards)."""
    from paper_1603_04570_amd.inputs import cosine_state, dofs
    n = args.paper_n
    p = ok.default_params(dim=3, n=n, eps=0.02, sigma=100.0, m=0.4, dt=4e-4, theta=0.5,
                          schur_richardson=2, mg_cycles=5,
                          precision=ok.OK_MIXED if args.precision == "mixed" else ok.OK_FP64)
    P = ok.Problem(p)
    u0, _ = cosine_state(3, n, 0.4)
    u0d = torch.from_numpy(u0).cuda()
    w0d = P.initial_w(u0d)
    tuned = 0 if args.no_autotune else P.autotune()
    u, w = u0d.clone(), w0d.clone()
    for _ in range(args.warmup):
        P.timestep(u, w, 1)
    u.copy_(u0d)
    w.copy_(w0d)
    torch.cuda.synchronize()
    # chunks of at most 100 timesteps: each chunk's stats hold every Newton
    # iteration's FGMRES count (the per-call history is bounded)
    its, newton, step_ms = [], [], []
    t0 = time.perf_counter()
    done = 0
    while done < args.steps:
        k = min(100, args.steps - done)
        st = P.timestep(u, w, k)
        its += st.its()
        newton += st.per_step()
        step_ms += st.ms()
        done += k
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    nd = dofs(3, n)
    out = _base_line(nd * args.steps / el, args.steps, args.warmup, el * 1e3 / args.steps,
                     "f64" if args.precision != "mixed" else "f64+f32",
                     {"workload": f"paper: Sec. 4 experiment on Q1, 3D N={n} ({nd} DOFs), m=0.4, "
                                  "eps=0.02, sigma=100, theta=1/2, dt=eps^2, cosine u0, w0 from "
                                  "(okb), 2 Richardson iterations of S~^-1, 5 V-cycles",
                      "dofs": nd, "global_batch": 1, "parallelism": "none (1 GPU)"})
    step_ms = np.array(step_ms)
    out.update({"latency_ms": {"p50": float(np.percentile(step_ms, 50)),
                               "p99": float(np.percentile(step_ms, 99))},
                "horizon": f"{args.steps} timesteps = {args.steps * 4e-4:g} time units",
                "newton_its": newton, "fgmres_its": its,
                "fgmres_per_newton": round(float(np.mean(its)), 2),
                "fgmres_per_newton_max": int(max(its)),
                "paper_reference_its": 8.0, "autotuned_shapes": tuned, "roofline": None})
    return out


def bench_robustness(args, torch, ok):
    """Average FGMRES iterations per Newton step (the paper's Tables 1-2
    measure) and timestep throughput, per case and solver preset."""
    from paper_1603_04570_amd.inputs import cosine_state, dofs, table1_cases, table2_cases
    presets = {"default": {}, "paper": dict(schur_richardson=2, mg_cycles=5)}
    steps = args.steps
    rows, tot_dofs, tot_s = [], 0.0, 0.0
    for table, cases in (("table2_eps", table2_cases()),
                         ("table1_refinement", table1_cases(3, (16, 32, 64, 128)))):
        for case in cases:
            for name, pre in presets.items():
                p = ok.default_params(dim=case["dim"], n=case["n"], eps=case["eps"],
                                      sigma=case["sigma"], m=case["m"], dt=case["dt"],
                                      theta=case["theta"], **pre)
                P = ok.Problem(p)
                u0, w0 = cosine_state(case["dim"], case["n"], case["m"])
                u, w = torch.from_numpy(u0).cuda(), torch.from_numpy(w0).cuda()
                P.autotune()
                P.timestep(u.clone(), w.clone(), 1)  # warm
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st = P.timestep(u, w, steps)
                torch.cuda.synchronize()
                el = time.perf_counter() - t0
                nd = dofs(case["dim"], case["n"])
                tot_dofs += nd * steps
                tot_s += el
                its = st.its()
                rows.append({"table": table, "dim": case["dim"], "n": case["n"],
                             "eps": case["eps"], "dt": case["dt"], "solver": name,
                             "newton_its": st.newton_its, "fgmres_its": its,
                             "fgmres_per_newton": round(float(np.mean(its)), 2),
                             "dofs_per_s": nd * steps / el})
                print(f"{table} N={case['n']} eps={case['eps']} {name}: "
                      f"{rows[-1]['fgmres_per_newton']} its/Newton", file=sys.stderr, flush=True)
    return {"metric": "timestep DOFs/s", "value": tot_dofs / tot_s, "unit": "DOFs/s",
            "n_gpus": 1, "steps": steps, "warmup": 1, "ms_per_step": tot_s * 1e3 / len(rows) / steps,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": "robustness: paper's Sec. 4 workload on Q1 (m=0.4, sigma=100, "
                                   "theta=1/2, cosine IC, w0=0); Table 2 analogue 2D eps sweep "
                                   "N=2/eps dt=eps^2; Table 1 analogue 3D N=16..128 eps=0.02 "
                                   "dt=4e-4", "parallelism": "none (1 GPU)"},
            "paper_reference_its": 8.0, "cases": rows, "roofline": None}


def bench_serve(args, torch, ok):
    """Serving loop: resident simulations, Poisson timestep requests,
    admission by HBM budget, continuous batching (native worker threads)."""
    from paper_1603_04570_amd.inputs import noise_state, poisson_arrivals, serving_simulation
    prec = ok.OK_FP64 if args.precision == "fp64" else ok.OK_MIXED
    sims = [serving_simulation(s) for s in range(256)]
    plist = [_params(ok, s, prec) for s in sims]
    cfg = ok.server_config(max_queue=args.max_queue, max_slots_per_pool=16)
    S = ok.Server(plist, int(args.budget_gib * 2**30), config=cfg)
    for i, s in enumerate(sims):
        u0, w0 = noise_state(s["dim"], s["n"], s["m"], s["seed"])
        S.set_state(i, torch.from_numpy(u0).cuda(), torch.from_numpy(w0).cuda())
    torch.cuda.synchronize()
    dofs_of = [2 * (s["n"] + 1) ** s["dim"] for s in sims]
    S.start()
    # warm-up: one request per class (pools created, code loaded, graphs captured)
    firsts = {}
    for i, s in enumerate(sims):
        firsts.setdefault((s["dim"], s["n"]), i)
    for i in firsts.values():
        S.submit(i, 1)
    got = 0
    while got < len(firsts):
        got += len(S.poll(4096, wait_s=1.0))
    runs = []
    for rate in [float(r) for r in args.rates.split(",")]:
        S.reset_stats()
        count = max(1, int(rate * args.duration))
        t, sim = poisson_arrivals(rate, count, len(sims), seed=5999)
        t0 = S.now() + 0.2
        for k in range(count):
            S.submit(int(sim[k]), 1, t0 + float(t[k]))
        res, last = [], time.perf_counter()
        while len(res) < count:
            res += S.poll(65536, wait_s=1.0)
            if time.perf_counter() - last > 10:
                print(f"serve rate {rate}: {len(res)}/{count} requests finished", file=sys.stderr,
                      flush=True)
                last = time.perf_counter()
        st = S.stats()
        done = [r for r in res if r["status"] == 0]
        lat = np.array([r["t_done"] - r["t_arrival"] for r in done]) * 1e3
        t_end = max(r["t_done"] for r in done) if done else t0
        dof_steps = sum(dofs_of[r["sim"]] * r["steps_done"] for r in done)
        runs.append({"offered_rate": rate, "requests": count, "completed": len(done),
                     "rejected": st["rejected"], "deferred": st["deferred"],
                     "failed": st["failed"],
                     "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
                     "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
                     "dofs_per_s": dof_steps / max(t_end - t0, 1e-9),
                     "completed_per_s": len(done) / max(t_end - t0, 1e-9),
                     "busy_s": st["busy_s"], "wall_s": t_end - t0, "ticks": st["ticks"],
                     "max_active": st["max_active"], "max_queue_seen": st["max_queue_seen"],
                     "pools_created": st["pools_created"], "pools_freed": st["pools_freed"],
                     "peak_pool_bytes": st["peak_bytes"],
                     "newton_its_mean": float(np.mean([r["newton_its"] for r in done]))
                     if done else None,
                     "fgmres_its_mean": float(np.mean([r["fgmres_its"] for r in done]))
                     if done else None})
    S.stop(drain=True)
    S.close()
    head = runs[-1]
    out = _base_line(head["dofs_per_s"], head["completed"], 0,
                     head["wall_s"] * 1e3 / max(head["completed"], 1),
                     "f64" if prec == ok.OK_FP64 else "f64+f32",
                     {"workload": "serve: 256 simulations (70% 2D N in {256,512,1024,2048}, 30% "
                                  "3D N in {64,128}; seeds 5000+s), Poisson timestep requests "
                                  f"(seed 5999) at {head['offered_rate']} req/s for "
                                  f"{args.duration} s, queue bound {args.max_queue}, pool budget "
                                  f"{args.budget_gib} GiB",
                      "simulations": 256, "global_batch": "continuous",
                      "parallelism": "none (1 GPU)"})
    out.update({"latency_ms": {"p50": head["p50_ms"], "p99": head["p99_ms"]},
                "serving": runs, "roofline": None})
    return out


def _single_params(ok, cfg, precision, solver=0):
    return ok.default_params(dim=cfg["dim"], n=cfg["n"], eps=cfg["eps"], sigma=cfg["sigma"],
                             m=cfg["m"], dt=cfg["dt"], theta=cfg["theta"], precision=precision,
                             linear_solver=solver)


def _side_by_side(torch, Pa, Pb, u0d, w0d, steps):
    """Both problems stepped from the same initial state: relative 2-norm
    difference of each field after each step, Pa against Pb."""
    ua, wa, ub, wb = u0d.clone(), w0d.clone(), u0d.clone(), w0d.clone()
    per_step = []
    for k in range(steps):
        Pa.timestep(ua, wa, 1)
        Pb.timestep(ub, wb, 1)
        per_step.append({"step": k + 1,
                         "u": float(torch.linalg.vector_norm(ua - ub) /
                                    torch.linalg.vector_norm(ub)),
                         "w": float(torch.linalg.vector_norm(wa - wb) /
                                    torch.linalg.vector_norm(wb))})
    return {"per_step": per_step, "max_u": max(p["u"] for p in per_step),
            "max_w": max(p["w"] for p in per_step)}


def _tune(args, ok, P, cfg):
    """Autotunes problem P, or pins the launch shapes a --save-shapes run wrote
    (--load-shapes: counter runs under a profiler then use the shapes the
    untraced run picked, not those of their own slowed autotuner).  With
    --save-shapes, the table's entries for the configuration's grids are
    merged into that file.  Returns the number of entries set."""
    if args.load_shapes:
        with open(args.load_shapes) as f:
            entries = json.load(f)
        for e in entries:
            ok.set_launch_shape(e["dim"], e["n"], e["kernel"], e["precision"], e["items"],
                                e["threads"], e["zchunks"])
        tuned = len(entries)
    else:
        tuned = 0 if args.no_autotune else P.autotune()
    if args.save_shapes:
        table = {}
        if os.path.exists(args.save_shapes):
            with open(args.save_shapes) as f:
                for e in json.load(f):
                    table[(e["dim"], e["n"], e["kernel"], e["precision"])] = e
        n = cfg["n"]
        while n >= 1:
            for kernel in range(ok.OK_SHAPE_STENCIL, ok.OK_SHAPE_MG_POST_STRIP + 1):
                for prec in (ok.OK_FP64, ok.OK_MIXED):
                    items, threads, zchunks = ok.get_launch_shape(cfg["dim"], n, kernel, prec)
                    key = (cfg["dim"], n, kernel, prec)
                    if items:
                        table[key] = {"dim": cfg["dim"], "n": n, "kernel": kernel,
                                      "precision": prec, "items": items, "threads": threads,
                                      "zchunks": zchunks}
            if n % 2:
                break
            n //= 2
        with open(args.save_shapes, "w") as f:
            json.dump(sorted(table.values(), key=lambda e: (e["n"], e["kernel"], e["precision"])),
                      f, indent=0)
    return tuned


def _timed_run(args, torch, ok, cfg, prec, u0d, w0d, solver=0):
    """One problem of the configuration in precision `prec`: autotuned,
    --warmup untimed timesteps from the initial state, then --steps timesteps
    from the same initial state timed between two device synchronisations
    (no profiling events in the timed region)."""
    P = ok.Problem(_single_params(ok, cfg, prec, solver), device=u0d.device)
    tuned = _tune(args, ok, P, cfg)
    if args.graphs:
        P.use_graphs(True)
    u, w = u0d.clone(), w0d.clone()
    for _ in range(args.warmup):
        P.timestep(u, w, 1)
    u.copy_(u0d)
    w.copy_(w0d)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = P.timestep(u, w, args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    return P, stats, elapsed, tuned


def _latency(torch, P, u0d, w0d, steps):
    """Per-timestep wall times (HIP events around each step) over `steps`
    consecutive timesteps from the initial state."""
    u, w = u0d.clone(), w0d.clone()
    ms = []
    while len(ms) < steps:
        k = min(steps - len(ms), 256)
        st = P.timestep(u, w, k)
        ms += st.ms()
    torch.cuda.synchronize()
    a = np.array(ms)
    return {"samples": len(ms), "p50": float(np.percentile(a, 50)),
            "p99": float(np.percentile(a, 99)), "max": float(a.max()), "mean": float(a.mean())}


def _profiled(torch, ok, P, u0d, w0d, steps, config, fp64):
    """Kernel-class timing in a profiled region: the same timesteps from the
    same initial state as the timed region, run again with HIP-event
    brackets on the launch stream around every launch chain of the three
    kernel classes."""
    P.profile_enable(ok.OK_K_KRYLOV, ok.OK_K_CHEB_MASS, ok.OK_K_MG_SMOOTH)
    u, w = u0d.clone(), w0d.clone()
    torch.cuda.synchronize()
    P.timestep(u, w, steps)
    torch.cuda.synchronize()
    out = {}
    for cls in (K_KRYLOV, K_CHEB_MASS, K_MG_SMOOTH):
        r, _ = roofline_of(P, cls, config, fp64)
        if r:
            r["window"] = f"profiled region: the {steps} timed timesteps rerun with event brackets"
            if cls in (K_CHEB_MASS, K_MG_SMOOTH):
                r["target_frac"] = TARGET_FRAC
                r["meets_target"] = r["frac"] >= TARGET_FRAC
        out[KERNELS[cls][0]] = r
    P.profile_enable()
    return out


def bench_single(args, torch, ok, cfg):
    """One problem of a named configuration: FP64 timed (the value), the
    mixed-precision form timed beside it, per-step latency, the mixed path's
    error against the FP64 path per step, kernel-class rooflines and the
    oracle's CPU baseline."""
    from paper_1603_04570_amd.inputs import dofs, noise_state
    dev = torch.device("cuda:0")
    u0, w0 = noise_state(cfg["dim"], cfg["n"], cfg["m"], cfg["seed"])
    u0d, w0d = torch.from_numpy(u0).to(dev), torch.from_numpy(w0).to(dev)
    nd = dofs(cfg["dim"], cfg["n"])
    precs = ["fp64", "mixed"] if args.precision in (None, "both") else [args.precision]
    runs = {}
    for prec in precs:
        pcode = ok.OK_FP64 if prec == "fp64" else ok.OK_MIXED
        P, st, el, tuned = _timed_run(args, torch, ok, cfg, pcode, u0d, w0d)
        lat = _latency(torch, P, u0d, w0d, args.latency_steps) if args.latency_steps > 0 else None
        prof = None if args.no_profile else _profiled(torch, ok, P, u0d, w0d, args.steps,
                                                      args.config, prec == "fp64")
        runs[prec] = dict(P=P, stats=st, elapsed=el, tuned=tuned, latency=lat, prof=prof)
        print(f"{args.config} {prec}: {nd * args.steps / el / 1e6:.1f}M DOFs/s, "
              f"{el * 1e3 / args.steps:.2f} ms/step", file=sys.stderr, flush=True)
    head = runs[precs[0]]
    st, el = head["stats"], head["elapsed"]
    roofline, kernels = None, None
    if head["prof"]:
        kernels = head["prof"]
        timed = [r for r in kernels.values() if r]
        if timed:  # the dominant kernel class by summed time
            roofline = max(timed, key=lambda r: r["total_ms"])
    out = _base_line(nd * args.steps / el, args.steps, args.warmup, el * 1e3 / args.steps,
                     "f64" if precs[0] == "fp64" else "f64+f32",
                     {"workload": f"{args.config}: {cfg['dim']}D Q1 {cfg['n']}^{cfg['dim']} "
                                  f"eps={cfg['eps']} sigma={cfg['sigma']} m={cfg['m']} "
                                  f"dt={cfg['dt']} theta={cfg['theta']} seed={cfg['seed']} "
                                  f"precision={precs[0]}",
                      "dofs": nd, "nodes": nd // 2, "global_batch": 1,
                      "parallelism": "none (1 GPU)"})
    step_ms = np.array(st.ms())
    out.update({
        "latency_ms": {"p50": float(np.percentile(step_ms, 50)),
                       "p99": float(np.percentile(step_ms, 99)), "samples": len(step_ms),
                       "long_run": head["latency"]},
        "newton_its": st.per_step(), "fgmres_its": st.its(),
        "roofline": roofline, "roofline_kernels": kernels,
        "autotuned_shapes": head["tuned"]})
    if "mixed" in runs and precs[0] != "mixed":
        mx = runs["mixed"]
        ms_step = np.array(mx["stats"].ms())
        out["mixed"] = {
            "value": nd * args.steps / mx["elapsed"], "unit": "DOFs/s", "dtype": "f64+f32",
            "ms_per_step": mx["elapsed"] * 1e3 / args.steps,
            "vs_fp64": el / mx["elapsed"],
            "latency_ms": {"p50": float(np.percentile(ms_step, 50)),
                           "p99": float(np.percentile(ms_step, 99)), "samples": len(ms_step),
                           "long_run": mx["latency"]},
            "newton_its": mx["stats"].per_step(), "fgmres_its": mx["stats"].its(),
            "roofline_kernels": mx["prof"]}
        # the mixed and the FP64 path stepped side by side from the same
        # initial state: relative error of each field after each step
        err = _side_by_side(torch, mx["P"], head["P"], u0d, w0d, args.steps)
        err["error"] = ("relative 2-norm of each field after each step, against the FP64 path "
                        "from the same initial state (both Newton-converged to the same "
                        "tolerance)")
        out["mixed"]["error_vs_fp64"] = err
    if args.linear_solver == "both" and precs[0] == "fp64":
        # Newton's linear solve by preconditioned MINRES on the symmetric
        # rearrangement (FP64), timed the same way beside the FGMRES headline
        Pm, mst, mel, _ = _timed_run(args, torch, ok, cfg, ok.OK_FP64, u0d, w0d,
                                     ok.OK_SOLVER_MINRES)
        print(f"{args.config} fp64 minres: {nd * args.steps / mel / 1e6:.1f}M DOFs/s, "
              f"{mel * 1e3 / args.steps:.2f} ms/step", file=sys.stderr, flush=True)
        ms_step = np.array(mst.ms())
        err = _side_by_side(torch, Pm, head["P"], u0d, w0d, args.steps)
        err["error"] = ("relative 2-norm of each field after each step, against the FGMRES "
                        "path from the same initial state")
        out["minres"] = {
            "value": nd * args.steps / mel, "unit": "DOFs/s", "dtype": "f64",
            "ms_per_step": mel * 1e3 / args.steps, "vs_fgmres": el / mel,
            "latency_ms": {"p50": float(np.percentile(ms_step, 50)),
                           "p99": float(np.percentile(ms_step, 99)), "samples": len(ms_step)},
            "newton_its": mst.per_step(), "minres_its": mst.its(),
            "error_vs_fgmres": err}
        del Pm
    for r in runs.values():
        del r["P"]
    if not args.no_cpu_baseline:
        per = st.fgmres_its_total / max(st.steps_done, 1)
        out["cpu_baseline"] = cpu_baseline(cfg, per, st.newton_its / max(st.steps_done, 1))
    return out


def kernel_probe(args, torch, ok, cfg):
    """The preconditioner's kernels alone, in the shapes the autotuner picks:
    --kernel-probe V-cycles of S^ and Chebyshev applications on M on a seeded
    right-hand side of the configuration's finest grid (not a benchmark line:
    a workload for hardware-counter runs of those kernels)."""
    from paper_1603_04570_amd.inputs import uniform01
    prec = ok.OK_MIXED if args.precision == "mixed" else ok.OK_FP64
    P = ok.Problem(_single_params(ok, cfg, prec))
    tuned = _tune(args, ok, P, cfg)
    nodes = (cfg["n"] + 1) ** cfg["dim"]
    r = torch.from_numpy(uniform01(5, nodes) - 0.5).cuda()
    x = torch.empty_like(r)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.kernel_probe):
        P.mg_apply(r, x)
    for _ in range(args.kernel_probe):
        P.cheb_mass(r, x)
    torch.cuda.synchronize()
    return {"kernel_probe": args.config, "precision": "mixed" if prec else "fp64",
            "applications": args.kernel_probe, "autotuned_shapes": tuned,
            "seconds": time.perf_counter() - t0}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="3d256",
                    help="3d256 (default), 3d128, 2d64, sweep64, serve, robustness, paper")
    ap.add_argument("--precision", choices=["both", "fp64", "mixed"], default=None,
                    help="single-problem configs: both (default; value = FP64), fp64 or mixed; "
                         "sweep64/serve: mixed by default")
    ap.add_argument("--latency-steps", type=int, default=100,
                    help="single-problem configs: timesteps of the p50/p99 latency run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--save-shapes", metavar="FILE",
                    help="single-problem configs: write the autotuned launch shapes of the "
                         "configuration's grids to FILE (JSON; merged with what it holds)")
    ap.add_argument("--load-shapes", metavar="FILE",
                    help="single-problem configs: pin the launch shapes of FILE instead of "
                         "autotuning")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain copy kernel of known size (for counter scaling)")
    ap.add_argument("--no-fuse", action="store_true",
                    help="run every Chebyshev iteration (on M and in the smoothers) in a pass of its own")
    ap.add_argument("--no-fold-prolong", action="store_true",
                    help="add the multigrid coarse-grid correction in a pass of its own instead "
                         "of inside the strip post-smoother")
    ap.add_argument("--issue-ahead", action="store_true",
                    help="issue each FGMRES iteration before the previous one's stop test is read")
    ap.add_argument("--linear-solver", choices=["both", "fgmres"], default="both",
                    help="single-problem configs: also time Newton with MINRES on the symmetric "
                         "system beside the FGMRES value (both, the default) or not (fgmres)")
    ap.add_argument("--gram-schmidt", choices=["icwy", "mgs"], default="icwy",
                    help="Arnoldi orthogonalisation: icwy (default; two passes, modified "
                         "Gram-Schmidt in inverse compact WY form) or mgs (one pass per "
                         "projection)")
    ap.add_argument("--kernel-probe", type=int, default=0, metavar="K",
                    help="single-problem configs: instead of timesteps, autotune and run K "
                         "V-cycles (ok_mg_apply) and K Chebyshev applications on M "
                         "(ok_cheb_mass) on the finest grid, for hardware-counter runs")
    ap.add_argument("--trace-ranges", action="store_true",
                    help="ROCTX ranges per timestep, Newton and FGMRES iteration "
                         "(for rocprofv3 --marker-trace)")
    ap.add_argument("--graphs", action="store_true",
                    help="replay captured FGMRES iterations (single-problem configs)")
    ap.add_argument("--rates", default="2000", help="serve: offered request rates (req/s)")
    ap.add_argument("--paper-n", type=int, default=100, help="paper: elements per direction")
    ap.add_argument("--duration", type=float, default=8.0, help="serve: seconds of arrivals")
    ap.add_argument("--budget-gib", type=float, default=160.0, help="serve: pool HBM budget")
    ap.add_argument("--max-queue", type=int, default=256, help="serve: queue bound")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch
    if args.calibrate_copy:
        calibrate_copy(torch)
        return
    from paper_1603_04570_amd import ok
    from paper_1603_04570_amd.inputs import CONFIGS

    if args.no_fuse:
        ok.set_option(ok.OK_OPT_FUSE_CHEB, 0)
        ok.set_option(ok.OK_OPT_FUSE_MG, 0)
    if args.no_fuse or args.no_fold_prolong:
        ok.set_option(ok.OK_OPT_FUSE_PROLONG, 0)
    if args.issue_ahead:
        ok.set_option(ok.OK_OPT_ISSUE_AHEAD, 1)
    if args.trace_ranges:
        ok.set_option(ok.OK_OPT_TRACE_RANGES, 1)
    if args.gram_schmidt == "mgs":
        ok.set_option(ok.OK_OPT_GRAM_SCHMIDT, 1)
    if args.config == "sweep64":
        print(json.dumps(bench_sweep(args, torch, ok)), flush=True)
        return
    if args.config == "paper":
        print(json.dumps(bench_paper(args, torch, ok)), flush=True)
        return
    if args.config == "robustness":
        print(json.dumps(bench_robustness(args, torch, ok)), flush=True)
        return
    if args.config == "serve":
        print(json.dumps(bench_serve(args, torch, ok)), flush=True)
        return
    cfg = dict(CONFIGS[args.config])
    if args.kernel_probe > 0:
        print(json.dumps(kernel_probe(args, torch, ok, cfg)), flush=True)
        return
    print(json.dumps(bench_single(args, torch, ok, cfg)), flush=True)


if __name__ == "__main__":
    main()
