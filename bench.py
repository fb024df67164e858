"""Benchmark: timestep throughput of the Ohta-Kawasaki Newton-Krylov solve on
one MI355X.

A step is one timestep of the whole hot path (Newton residual, FGMRES with the
matching-Schur block preconditioner, Jacobian applies, updates) over the
configured synthetic field.  Prints ONE JSON line.

Default workload: 3D unit cube, Q1 hex on a uniform 128^3 mesh (2,146,689
nodes, 4,293,378 DOFs), eps=0.01, sigma=1000, m=0.1, theta=1, dt=2e-5,
u0 = m + 0.05*U(-1,1) seeded (seed 2), w0 = 0, FP64 throughout.
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


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def cpu_baseline(cfg, its_per_step, sample_its=4):
    """The FP64 CSR oracle on one host core: `sample_its` FGMRES iterations of
    the first Newton solve of timestep 1 (setup excluded, as on the GPU),
    scaled to a whole timestep by the FGMRES iterations per timestep."""
    from oracle.okref import Oracle
    from paper_1603_04570_amd.inputs import dofs, noise_state
    dim, n = cfg["dim"], cfg["n"]
    o = Oracle(dim, n, cfg["eps"], cfg["sigma"], cfg["m"], cfg["dt"], cfg["theta"],
               gmres_restart=sample_its, gmres_max_restarts=0)
    u, w = noise_state(dim, n, cfg["m"], cfg["seed"])
    t0 = time.perf_counter()
    F, _ = o.residual(u, w, u)
    x, its, st = o.fgmres(u, -F)
    dt_s = time.perf_counter() - t0
    per_it = dt_s / max(its, 1)
    step_s = per_it * its_per_step
    return {"value": dofs(dim, n) / step_s, "unit": "DOFs/s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle (serial FP64 CSR) on {dim}D {n}^{dim}: residual + {its} FGMRES "
                       f"iterations of the first Newton solve ({dt_s:.1f} s), scaled to the "
                       f"{its_per_step} FGMRES iterations of one timestep; host {cpu_model()}, "
                       f"nproc {os.cpu_count()}")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="3d128")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_1603_04570_amd import ok
    from paper_1603_04570_amd.inputs import CONFIGS, dofs, noise_state

    cfg = dict(CONFIGS[args.config])
    prec = args.precision or cfg["precision"]
    p = ok.default_params(dim=cfg["dim"], n=cfg["n"], eps=cfg["eps"], sigma=cfg["sigma"],
                          m=cfg["m"], dt=cfg["dt"], theta=cfg["theta"],
                          precision=ok.OK_MIXED if prec == "mixed" else ok.OK_FP64)
    dev = torch.device("cuda:0")
    P = ok.Problem(p, device=dev)
    u0, w0 = noise_state(cfg["dim"], cfg["n"], cfg["m"], cfg["seed"])
    u0d = torch.from_numpy(u0).to(dev)
    w0d = torch.from_numpy(w0).to(dev)
    u, w = u0d.clone(), w0d.clone()
    tuned = 0 if args.no_autotune else P.autotune()
    for _ in range(args.warmup):
        P.timestep(u, w, 1)
    u.copy_(u0d)
    w.copy_(w0d)
    if not args.no_profile:
        P.profile_enable(ok.OK_K_CHEB_MASS)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = P.timestep(u, w, args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    launches, kms, kbytes = P.profile_read() if not args.no_profile else (0, 0.0, 0.0)

    nd = dofs(cfg["dim"], cfg["n"])
    value = nd * args.steps / elapsed
    step_ms = np.array(stats.ms())
    its = stats.its()
    roofline = None
    if launches:
        avg_s = kms / launches * 1e-3
        per_launch = kbytes / launches
        ach = per_launch / avg_s / 1e9
        roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                    "kernel": "Chebyshev-Jacobi iteration on M (k_stencil, EpiChebStep)",
                    "bytes_per_launch": per_launch, "avg_us": round(avg_s * 1e6, 2),
                    "launches": launches}
    out = {
        "metric": "timestep DOFs/s",
        "value": value,
        "unit": "DOFs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {cfg['dim']}D Q1 {cfg['n']}^{cfg['dim']} "
                               f"eps={cfg['eps']} sigma={cfg['sigma']} m={cfg['m']} "
                               f"dt={cfg['dt']} theta={cfg['theta']} seed={cfg['seed']} "
                               f"precision={prec}",
                   "dofs": nd, "nodes": nd // 2, "global_batch": 1,
                   "parallelism": "none (1 GPU)"},
        "latency_ms": {"p50": float(np.percentile(step_ms, 50)),
                       "p99": float(np.percentile(step_ms, 99))},
        "newton_its": stats.per_step(),
        "fgmres_its": its,
        "roofline": roofline,
        "autotuned_shapes": tuned,
    }
    if not args.no_cpu_baseline:
        per_step = stats.fgmres_its_total / max(stats.steps_done, 1)
        out["cpu_baseline"] = cpu_baseline(cfg, int(round(per_step)))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
