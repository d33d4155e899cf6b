"""Benchmark: batched MPC QP solves per second on one MI355X.

A "step" is one control step of the RL-training workload: every agent's QP is
solved (stage setup, Riccati factor, 50 warm-started ADMM iterations, FP64 KKT
residual check) and every agent's plant is advanced by its own first stage
plus Gaussian noise, x0 <- A_0 x0 + B_0 u_0* + c_0 + w, w ~ N(0, 1e-2^2).
Default workload: 4096 humanoid agents (nx=48, nu=30, N=10), FP32.
All inputs are synthetic and resident in HBM before timing starts.

Prints ONE JSON line: throughput and latency, the iteration kernel's roofline
(algorithmic FP32 FLOPs per launch over its HIP-event time, against the FP32
vector peak, plus its recorded HBM traffic) and the FP64 CPU oracle's rate on
a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"alu_f32": 157.3e12, "alu_f64": 78.6e12, "hbm": 8.0e12}


def flops_iter_stage(nx, nu):
    """Matvec FLOPs of one ADMM iteration per stage: back chain A_cl' (nx^2),
    K' rt (nx nu), B' p' (nx nu), H^-1 (nu^2), B d (nx nu), forward chain
    A_cl (nx^2), K x (nx nu); 2 FLOP per multiply-add."""
    return 2 * (2 * nx * nx + 4 * nx * nu + nu * nu)


def flops_factor_stage(nx, nu):
    """FLOPs of one Riccati factor stage: P B, P A, B'(PB), B'(PA), K = -H^-1 G,
    H^-1, A'(PA), G'K, A_cl = A + B K, s = P c (2 FLOP per multiply-add; the
    Cholesky itself, nu^3/3, included)."""
    mac = (nx * nx * nu + nx ** 3 + nx * nu * nu + nu * nx * nx + nu * nu * nx + nu ** 3
           + nx ** 3 + nu * nx * nx + nx * nx * nu + nx * nx + nu ** 3 / 6)
    return 2 * mac


def sampled_errors(sol, ref, ids, shape, n_agents):
    """Worst norm-wise relative error over the sampled agents of u_0 and of the
    trajectory (x_1..N, u_0..N-1) against an oracle solution of those agents."""
    nx, nu = shape.nx, shape.nu
    x = sol["x"].cpu().numpy().reshape(n_agents, -1)[ids].astype(np.float64)[:, nx:]
    u = sol["u"].cpu().numpy().reshape(n_agents, -1)[ids].astype(np.float64)
    xo = ref["x"].reshape(len(ids), -1)[:, nx:]
    uo = ref["u"].reshape(len(ids), -1)
    tr, to = np.concatenate([x, u], 1), np.concatenate([xo, uo], 1)
    e_tr = np.abs(tr - to).max(1) / np.abs(to).max(1)
    e_u0 = np.abs(u[:, :nu] - uo[:, :nu]).max(1) / np.abs(uo[:, :nu]).max(1)
    return float(e_u0.max()), float(e_tr.max())


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--agents", type=int, default=4096)
    ap.add_argument("--horizon", type=int, default=10)
    ap.add_argument("--iters", type=int, default=50)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64", "fp32r", "fp32mfma"],
                    help="fp32r: factor products on the FP32 matrix cores with KKT-residual "
                         "refinement sweeps in the iterations (--refine-sweeps)")
    ap.add_argument("--refine-sweeps", type=int, default=3)
    ap.add_argument("--kernel", default="auto", choices=["auto", "generic", "fused", "persistent"],
                    help="persistent (with --uneven): one persistent iteration launch per shape "
                         "class over every horizon instead of one launch per horizon bucket")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="approximate wall time budget of the CPU-oracle baseline (0 = skip)")
    ap.add_argument("--check-agents", type=int, default=64,
                    help="agents whose first-step solution is compared with the FP64 oracle")
    ap.add_argument("--uneven", action="store_true",
                    help="time the uneven batch instead (8192 agents, N ~ U{5..20}, half humanoid, "
                         "half quadruped): autotuned launch groups, captured-graph steps "
                         "(prints its own JSON line)")
    ap.add_argument("--mixed", action="store_true",
                    help="time the mixed-precision sweep instead (16384 humanoid agents, N=16, "
                         "Q/R condition 1e4): FP32 vs BF16 / FP16 products with refinement, "
                         "step time and error vs the FP64 oracle per mode (prints its own JSON line)")
    ap.add_argument("--scaled", action="store_true",
                    help="time Alg. 1's scaling step and adaptive rho instead (16384 humanoid agents, "
                         "N=16, Q/R condition 1e6, FP32): plain vs Ruiz vs Ruiz + adaptive rho, step "
                         "time and the error of the fixed-iteration iterate against the converged "
                         "optimum (prints its own JSON line)")
    ap.add_argument("--scan", action="store_true",
                    help="parallel-in-time against serial Riccati factor on long horizons")
    ap.add_argument("--no-slip", action="store_true",
                    help="with --rti: the QP carries the feet's no-slip rows from the linearisation")
    ap.add_argument("--rti", action="store_true",
                    help="time the real-time iteration's control step on the articulated humanoid "
                         "(linearise, solve, torques, plant step)")
    ap.add_argument("--inner", action="store_true",
                    help="time the two inner solves side by side instead (exact-dynamics Riccati vs the "
                         "paper's KKT LDL^T with finite rho_eq; prints its own JSON line)")
    ap.add_argument("--serve", action="store_true",
                    help="run the served request loop instead: Poisson arrivals from independent "
                         "controllers of uneven shapes (prints its own JSON line)")
    ap.add_argument("--controllers", type=int, default=8192)
    ap.add_argument("--serve-precision", default="fp32", choices=("fp32", "bf16", "fp16", "fp32mfma"),
                    help="served loop precision (bf16/fp16: mixed precision with refinement; "
                         "fp32mfma: FP32 with the factor's products on the FP32 matrix cores)")
    ap.add_argument("--supersede", action="store_true",
                    help="served loop: a controller's waiting request is dropped when a newer one of "
                         "it arrives (solves/s and latency then count solved requests)")
    ap.add_argument("--max-batch", type=int, default=4096,
                    help="served loop: most requests per batch (with fewer than the controllers, a "
                         "batch forms while another runs)")
    ap.add_argument("--rate-hz", type=float, default=100.0, help="request rate per controller")
    ap.add_argument("--sim-seconds", type=float, default=60.0, help="length of the served trace")
    ap.add_argument("--max-inflight", type=int, default=3, help="batch slots of the server")
    ap.add_argument("--hbm-budget-gb", type=float, default=64.0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain device copy of 1 GiB (x5), the reference kernel for "
                         "scaling the FETCH_SIZE / WRITE_SIZE counters")
    ap.add_argument("--summarize-pmc", nargs=4, metavar=("FETCH_BENCH", "WRITE_BENCH",
                                                         "FETCH_COPY", "WRITE_COPY"),
                    help="turn four rocprofv3 --pmc counter_collection.csv files into the "
                         "traffic summary under profiles/ (no GPU needed)")
    return ap.parse_args()


TRAFFIC_MD = os.path.join(ROOT, "profiles", "traffic_k_admm_resident_humanoid4096.md")
COPY_BYTES = 1 << 30


def kernel_source_digest():
    import hashlib
    path = os.path.join(ROOT, "paper_2510_12717_amd", "csrc", "kernels_fused.hip")
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def _pmc_per_dispatch(path, name_part):
    """Mean counter value (summed over the counter's instances) per dispatch of the
    kernels whose name contains name_part."""
    import csv
    rows = list(csv.DictReader(open(path)))
    kcol = next(c for c in rows[0] if c.lower() in ("kernel_name", "kernel-name"))
    vcol = next(c for c in rows[0] if c.lower() in ("counter_value", "counter-value"))
    dcol = next(c for c in rows[0] if c.lower() in ("dispatch_id", "dispatch-id"))
    per = {}
    for r in rows:
        if name_part in r[kcol]:
            per[r[dcol]] = per.get(r[dcol], 0.0) + float(r[vcol])
    if not per:
        raise SystemExit(f"no dispatch of a kernel matching {name_part!r} in {path}")
    return sum(per.values()) / len(per), len(per)


def summarize_pmc(paths):
    """Traffic of the iteration kernel from FETCH_SIZE / WRITE_SIZE (KiB per dispatch),
    each scaled by what the same counter reads for a 1 GiB device copy."""
    fb, wb, fc, wc = paths
    kname = "k_admm_resident<48, 30, false>"
    f_k, n_f = _pmc_per_dispatch(fb, "k_admm_resident")
    w_k, n_w = _pmc_per_dispatch(wb, "k_admm_resident")
    f_c, _ = _pmc_per_dispatch(fc, "copy")
    w_c, _ = _pmc_per_dispatch(wc, "copy")
    scale_r = f_c * 1024.0 / COPY_BYTES
    scale_w = w_c * 1024.0 / COPY_BYTES
    traffic = f_k * 1024.0 / scale_r + w_k * 1024.0 / scale_w
    rec = {"kernel": kname, "source_digest": kernel_source_digest(),
           "fetch_kib_per_dispatch": f_k, "write_kib_per_dispatch": w_k,
           "dispatches": [n_f, n_w], "copy_fetch_kib": f_c, "copy_write_kib": w_c,
           "copy_bytes": COPY_BYTES, "read_scale": scale_r, "write_scale": scale_w,
           "traffic_bytes_per_launch": traffic}
    cmd = ("cd /tmp && timeout -s KILL 120 rocprofv3 --pmc {c} --output-format csv -d <out>/{d} "
           "-o run -- python3 <repo>/bench.py {a}")
    lines = ["# HBM traffic of the iteration kernel: 4096 humanoid agents (N=10, "
             "50 iterations, FP32)", "",
             "FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of `" + kname + "`, each divided by the "
             "ratio the same counter reads for a plain 1 GiB device copy (`bench.py --calibrate-copy`).",
             "Commands (four passes, one counter each; <out> is the run's output folder):", "", "```",
             cmd.format(c="FETCH_SIZE", d="pmc_FETCH_SIZE_bench", a="--steps 2 --warmup 1 --cpu-seconds 0 --check-agents 4"),
             cmd.format(c="FETCH_SIZE", d="pmc_FETCH_SIZE_copy", a="--calibrate-copy"),
             cmd.format(c="WRITE_SIZE", d="pmc_WRITE_SIZE_bench", a="--steps 2 --warmup 1 --cpu-seconds 0 --check-agents 4"),
             cmd.format(c="WRITE_SIZE", d="pmc_WRITE_SIZE_copy", a="--calibrate-copy"),
             "python bench.py --summarize-pmc <out>/pmc_{FETCH_SIZE,WRITE_SIZE}_bench/run_counter_collection.csv "
             "<out>/pmc_{FETCH_SIZE,WRITE_SIZE}_copy/run_counter_collection.csv", "```", "",
             "Algorithmic bytes per launch (operators loaded once, 4096 agents x (10 stages x 100 "
             "floats x 64 lanes + S_0, 2304 floats); vectors and the resident state in and out): "
             "1.13 GB read, 0.026 GB "
             "written.", "",
             "| quantity | value |", "|---|---|",
             f"| FETCH_SIZE per dispatch | {f_k:.0f} KiB |", f"| WRITE_SIZE per dispatch | {w_k:.0f} KiB |",
             f"| copy: FETCH_SIZE / bytes read | {scale_r:.3f} |",
             f"| copy: WRITE_SIZE / bytes written | {scale_w:.3f} |",
             f"| traffic per launch | {traffic / 1e9:.3f} GB |", "",
             "Machine-readable record (bench.py reports `traffic` from it while the kernel source "
             "digest matches):", "", "```json", json.dumps(rec), "```", ""]
    open(TRAFFIC_MD, "w").write("\n".join(lines))
    print(json.dumps(rec))


def recorded_traffic():
    """Traffic per launch from the committed counter summary, or None if the kernel
    source changed since the counters were taken."""
    try:
        text = open(TRAFFIC_MD).read()
        rec = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    if rec.get("source_digest") != kernel_source_digest():
        return None
    return rec["traffic_bytes_per_launch"]


def calibrate_copy():
    import torch
    n = COPY_BYTES // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": COPY_BYTES, "copy_bytes_written": COPY_BYTES, "reps": 5}))


def uneven(args):
    """Uneven batch: autotune the launch groups, capture one control step (warm
    solve + plant step) into a HIP graph, time replays."""
    import torch

    from paper_2510_12717_amd import mpc, synth

    torch.cuda.set_device(0)
    n = args.agents if args.agents != 4096 else 8192
    b = synth.uneven_batch(n, dtype=np.float32)
    prec = args.precision if args.precision in ("fp32", "fp32mfma") else "fp32"
    plan = mpc.Plan(b.shapes, precision=prec, iters=args.iters, kernel=args.kernel)
    prob = mpc.to_device(b, "fp32")
    t_tune = time.perf_counter()
    groups = plan.autotune(prob, reps=2)
    t_tune = time.perf_counter() - t_tune
    nx_tot = sum(s.nx for s in b.shapes)
    noise = torch.empty(nx_tot, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(99)
    plan.solve(prob)
    plan.capture(prob, warm_start=True, noise=noise, x0_next=prob["x0"])
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        noise.normal_(0.0, 1e-2, generator=gen)
        plan.replay(stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        noise.normal_(0.0, 1e-2, generator=gen)
        plan.replay(stream)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([a.elapsed_time(c) for a, c in ev])
    st = plan.get_solution()["status"]
    out = {"metric": "MPC QP solves/sec, uneven batch (captured step, autotuned groups)",
           "kernel": args.kernel, "precision": prec,
           "value": n * args.steps / wall, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
           "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{n} agents, N ~ U{{5..20}}, half humanoid (48, 30), half "
                                  "quadruped (36, 24), stance p ~ U[0.3, 0.9] per foot, "
                                  f"{args.iters} warm-started iterations", "agents": n,
                      "admm_iters": args.iters},
           "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
           "groups": [(g["family"], g["nx"], g["N"], g["n_agents"], g["threads"]) for g in groups],
           "autotune_s": t_tune, "status_ok": bool((st == 0).all().item())}
    print(json.dumps(out))


def mixed(args):
    """Mixed-precision sweep: one cold solve per timed step of 16384 humanoid agents
    (N = 16, Q/R condition 1e4) in each mode; errors of every 64th agent vs the
    FP64 oracle (u_0 and trajectory, norm-wise relative)."""
    import torch

    import oracle
    from paper_2510_12717_amd import mpc, synth

    torch.cuda.set_device(0)
    n = args.agents if args.agents != 4096 else 16384
    kappa = 1e4
    b = synth.conditioned_humanoid_batch(n, kappa=kappa, dtype=np.float32)
    prob = mpc.to_device(b, "fp32")
    ids = np.arange(0, n, 64)
    ref = oracle.solve_batch(synth.conditioned_humanoid_batch(agent_ids=ids, kappa=kappa), iters=args.iters)
    sh = b.shapes[0]
    modes = {}
    for prec, sweeps in (("fp32", 0), ("fp32mfma", 0), ("fp32r", 0), ("fp32r", 3), ("bf16", 0), ("bf16", 3),
                         ("fp16", 0), ("fp16", 3)):
        plan = mpc.Plan(b.shapes, precision=prec, iters=args.iters, max_refine_sweeps=sweeps)
        stream = torch.cuda.current_stream()
        for _ in range(max(args.warmup, 1)):
            plan.solve(prob, stream=stream)
        torch.cuda.synchronize()
        plan.set_timing(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan.solve(prob, stream=stream)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / args.steps * 1e3
        tm = plan.get_timing()
        fac_ms = tm["factor"][0] / max(tm["factor"][1], 1)
        # the factor's block products on the matrix cores: FP64 MFMA in the FP32 mode,
        # FP32 MFMA in fp32mfma / fp32r, BF16 / FP16 MFMA (FP32 accumulation) otherwise
        fac_flops = flops_factor_stage(sh.nx, sh.nu) * sh.N * n
        mdt = {"fp32": "f64", "fp32mfma": "f32", "fp32r": "f32"}.get(prec, prec)
        peak = {"f64": 78.6, "f32": 157.3}.get(mdt, 2500.0)
        u = plan.get_solution()["u"].cpu().numpy().reshape(n, sh.N * sh.nu)[ids].astype(np.float64)
        x = plan.get_solution()["x"].cpu().numpy().reshape(n, (sh.N + 1) * sh.nx)[ids].astype(np.float64)
        uo = ref["u"].reshape(len(ids), -1)
        xo = ref["x"].reshape(len(ids), -1)
        tr = np.concatenate([x[:, sh.nx:], u], 1)
        to = np.concatenate([xo[:, sh.nx:], uo], 1)
        e_u0 = np.abs(u[:, :sh.nu] - uo[:, :sh.nu]).max(1) / np.abs(uo[:, :sh.nu]).max(1)
        e_tr = np.abs(tr - to).max(1) / np.abs(to).max(1)
        key = prec if prec in ("fp32", "fp32mfma") else f"{prec}_sweeps{sweeps}"
        modes[key] = {"ms_per_step": ms, "solves_per_s": n / ms * 1e3,
                      "factor_ms": fac_ms,
                      "factor_roofline": {"bound": "mfma", "achieved": fac_flops / fac_ms / 1e9,
                                          "peak": peak, "unit": "TFLOP/s",
                                          "frac": fac_flops / fac_ms / 1e9 / peak,
                                          "mfma_dtype": mdt},
                      "err_u0_max": float(e_u0.max()), "err_traj_max": float(e_tr.max()),
                      "err_traj_p50": float(np.median(e_tr)), "kernel": plan.config()["kernel"]}
        plan.close()
    out = {"metric": "MPC QP solves/sec per precision mode and error vs FP64",
           "value": modes["fp32"]["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
           "steps": args.steps, "higher_is_better": True, "dtype": "mixed", "data": "synthetic",
           "config": {"workload": f"{n} humanoid agents, N=16, Q/R condition {kappa:g}, "
                                  f"{args.iters} cold ADMM iterations", "agents": n,
                      "checked_agents": int(len(ids))},
           "modes": modes}
    print(json.dumps(out))


def scaled(args):
    """Scaling step and adaptive rho on the conditioned sweep at kappa = 1e6: one cold
    solve of 16384 humanoid agents (N = 16) per timed step in each mode; for every
    1024th agent the error of the 50-iteration iterate against the problem's
    converged optimum (oracle, converge mode) and against the oracle's iterate of
    the same mode (u_0 and trajectory, norm-wise relative)."""
    import torch

    import oracle
    from oracle import scaling
    from paper_2510_12717_amd import mpc, synth

    torch.cuda.set_device(0)
    n = args.agents if args.agents != 4096 else 16384
    kappa = 1e6
    b = synth.conditioned_humanoid_batch(n, kappa=kappa, dtype=np.float32)
    prob = mpc.to_device(b, "fp32")
    ids = np.arange(0, n, 1024)
    sub = synth.conditioned_humanoid_batch(agent_ids=ids, kappa=kappa, dtype=np.float32)
    sh = b.shapes[0]
    opt = [oracle.solve(*[oracle.agent(sub, a)[k] for k in ("s", "A", "B", "c", "q", "r", "x_ref",
                                                           "x0", "tau_max", "mu", "stance")],
                        iters=0, tol=1e-9) for a in range(len(ids))]

    def err(u, x, o):
        uo, xo = np.ravel(o["u"]), np.ravel(o["x"])
        tr, to = np.concatenate([x[sh.nx:], u]), np.concatenate([xo[sh.nx:], uo])
        return (np.abs(u[:sh.nu] - uo[:sh.nu]).max() / np.abs(uo[:sh.nu]).max(),
                np.abs(tr - to).max() / np.abs(to).max())

    modes = {}
    for name, si, ri in (("plain", 0, 0), ("ruiz", 10, 0), ("ruiz_adaptive_rho", 10, 10),
                         ("adaptive_rho", 0, 10)):
        plan = mpc.Plan(b.shapes, precision="fp32", iters=args.iters, scaling_iters=si,
                        rho_interval=ri)
        stream = torch.cuda.current_stream()
        for _ in range(max(args.warmup, 1)):
            plan.solve(prob, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan.solve(prob, stream=stream)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / args.steps * 1e3
        sol = plan.get_solution()
        u = sol["u"].cpu().numpy().reshape(n, -1)[ids].astype(np.float64)
        x = sol["x"].cpu().numpy().reshape(n, -1)[ids].astype(np.float64)
        st = sol["status"].cpu().numpy()
        ref = [scaling.solve(oracle.agent(sub, a), iters=args.iters, ruiz_iters=si, rho_interval=ri)
               for a in range(len(ids))]
        e_opt = np.array([err(u[a], x[a], opt[a]) for a in range(len(ids))])
        e_ref = np.array([err(u[a], x[a], ref[a]) for a in range(len(ids))])
        o_opt = np.array([err(np.ravel(ref[a]["u"]), np.ravel(ref[a]["x"]), opt[a]) for a in range(len(ids))])
        modes[name] = {"ms_per_step": ms, "solves_per_s": n / ms * 1e3,
                       "status_ok": bool((st == 0).all()),
                       "gpu_vs_optimum": {"u0_median": float(np.median(e_opt[:, 0])),
                                          "traj_median": float(np.median(e_opt[:, 1])),
                                          "traj_max": float(e_opt[:, 1].max())},
                       "oracle_vs_optimum": {"traj_median": float(np.median(o_opt[:, 1])),
                                             "traj_max": float(o_opt[:, 1].max())},
                       "gpu_vs_oracle_same_mode": {"u0_max": float(e_ref[:, 0].max()),
                                                   "traj_max": float(e_ref[:, 1].max())}}
        plan.close()
    out = {"metric": "MPC QP solves/sec and fixed-iteration error vs the optimum, per scaling mode",
           "value": modes["ruiz_adaptive_rho"]["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
           "steps": args.steps, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{n} humanoid agents, N=16, Q/R condition {kappa:g}, "
                                  f"{args.iters} cold ADMM iterations", "agents": n,
                      "checked_agents": int(len(ids)), "ruiz_rounds": 10, "rho_interval": 10},
           "modes": modes}
    print(json.dumps(out))


def inner(args):
    """The two inner solves side by side on the N = 10 humanoid workload (4096
    agents, FP32, 50 cold iterations per timed solve): the exact-dynamics
    Riccati path (register-resident kernels) and the paper's form (dynamics as
    equality rows with rho_eq, quasi-definite KKT factored by LDL^T, generic
    kernels).  Per mode: time per solve, the largest dynamics residual of the
    returned iterates, and for every 256th agent the error of the 50-iteration
    iterate against the QP's converged optimum (oracle, converge mode) and
    against the oracle of the same mode."""
    import torch

    import oracle
    from oracle import kkt as okkt
    from paper_2510_12717_amd import mpc, synth

    torch.cuda.set_device(0)
    n = args.agents
    b = synth.humanoid_batch(n, dtype=np.float32)
    prob = mpc.to_device(b, "fp32")
    ids = np.arange(0, n, 256)
    sub = synth.humanoid_batch(agent_ids=ids, dtype=np.float32)
    sh = b.shapes[0]
    keys = ("s", "A", "B", "c", "q", "r", "x_ref", "x0", "tau_max", "mu", "stance")
    opt = [oracle.solve(*[oracle.agent(sub, a)[k] for k in keys], iters=0, tol=1e-10)
           for a in range(len(ids))]

    def err(u, x, o):
        uo, xo = np.ravel(o["u"]), np.ravel(o["x"])
        tr, to = np.concatenate([x[sh.nx:], u]), np.concatenate([xo[sh.nx:], uo])
        return (np.abs(u[:sh.nu] - uo[:sh.nu]).max() / np.abs(uo[:sh.nu]).max(),
                np.abs(tr - to).max() / np.abs(to).max())

    modes = {}
    for name, kw in (("riccati_exact_dynamics", {}), ("kkt_ldl_finite_rho_eq", {"inner_solve": 1})):
        plan = mpc.Plan(b.shapes, precision="fp32", iters=args.iters, **kw)
        stream = torch.cuda.current_stream()
        for _ in range(max(args.warmup, 1)):
            plan.solve(prob, stream=stream)
        torch.cuda.synchronize()
        plan.set_timing(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan.solve(prob, stream=stream)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / args.steps * 1e3
        tm = plan.get_timing()
        sol = plan.get_solution()
        u = sol["u"].cpu().numpy().reshape(n, -1)[ids].astype(np.float64)
        x = sol["x"].cpu().numpy().reshape(n, -1)[ids].astype(np.float64)
        res = sol["residuals"].cpu().numpy()
        st = sol["status"].cpu().numpy()
        if kw:
            ref = [okkt.solve(oracle.agent(sub, a), iters=args.iters) for a in range(len(ids))]
        else:
            ref = [oracle.solve(*[oracle.agent(sub, a)[k] for k in keys], iters=args.iters)
                   for a in range(len(ids))]
        e_opt = np.array([err(u[a], x[a], opt[a]) for a in range(len(ids))])
        e_ref = np.array([err(u[a], x[a], ref[a]) for a in range(len(ids))])
        modes[name] = {"ms_per_step": ms, "solves_per_s": n / ms * 1e3,
                       "kernel_ms": {k: v[0] / max(v[1], 1) for k, v in tm.items()},
                       "status_ok": bool((st == 0).all()),
                       "dynamics_residual_max": float(res[:, 2].max()),
                       "gpu_vs_optimum": {"u0_median": float(np.median(e_opt[:, 0])),
                                          "traj_median": float(np.median(e_opt[:, 1])),
                                          "traj_max": float(e_opt[:, 1].max())},
                       "gpu_vs_oracle_same_mode": {"u0_max": float(e_ref[:, 0].max()),
                                                   "traj_max": float(e_ref[:, 1].max())}}
        plan.close()
    out = {"metric": "MPC QP solves/sec and fixed-iteration error vs the optimum, per inner solve",
           "value": modes["kkt_ldl_finite_rho_eq"]["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
           "steps": args.steps, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{n} humanoid agents (nx=48, nu=30), N=10, {args.iters} cold ADMM "
                                  "iterations", "agents": n, "checked_agents": int(len(ids))},
           "modes": modes}
    print(json.dumps(out))


def serve(args):
    """Served loop: every controller (shapes as the uneven batch: N ~ U{5..20},
    half humanoid, half quadruped) sends Poisson requests at rate-hz for
    sim-seconds of wall time; its problem data sit in a device-resident pool.
    Latency = completion event time - arrival time, on the server's clock."""
    import ctypes
    import torch

    from paper_2510_12717_amd import mpc, synth

    torch.cuda.set_device(0)
    nc = args.controllers
    b = synth.uneven_batch(nc)
    prob = mpc.to_device(b, "fp32")
    reqs = mpc.agent_problems(prob, b)
    for r in reqs:
        r.warm_start = 1
    rec_p = np.frombuffer(reqs, dtype=np.dtype((np.void, ctypes.sizeof(mpc.ProblemBatch))))
    shapes = (mpc.Shape * nc)(*[mpc.Shape(*s.as_tuple()) for s in b.shapes])
    rec_s = np.frombuffer(shapes, dtype=np.dtype((np.void, ctypes.sizeof(mpc.Shape))))
    nu = np.array([s.nu for s in b.shapes])
    u0 = torch.zeros(int(nu.sum()), device="cuda")
    u0_ptr = (u0.data_ptr() + 4 * np.concatenate([[0], np.cumsum(nu)[:-1]])).astype(np.uint64)
    # arrivals: the superposition of nc independent Poisson processes of rate
    # rate_hz is one Poisson process of rate nc * rate_hz whose events pick a
    # controller uniformly; drawn in windows of 0.1 s as the trace advances
    rng = np.random.default_rng(11)
    total_rate = nc * args.rate_hz
    win = 0.1

    def window(t_lo):
        t_hi = min(t_lo + win, args.sim_seconds)
        k = rng.poisson(total_rate * (t_hi - t_lo))
        return np.sort(rng.uniform(t_lo, t_hi, k)), rng.integers(0, nc, k), t_hi

    srv = mpc.Server(precision=args.serve_precision, iters=args.iters,
                     hbm_budget_bytes=int(args.hbm_budget_gb * (1 << 30)), max_batch=args.max_batch,
                     max_inflight=args.max_inflight, supersede=args.supersede)
    # warm every controller once (cold first solves), outside the measurement
    srv.submit_many(np.arange(nc), rec_s, rec_p, u0_ptr, np.zeros(nc))
    srv.drain()
    srv.poll(cap=nc + 16)
    # tickets are consecutive integers: arrival times indexed by ticket
    tk_base = nc
    t_arr = np.full(int(total_rate * args.sim_seconds * 1.01) + 1024, np.nan)
    lat = []
    t0 = srv.clock()
    n, outstanding = 0, 0
    at, ac, t_next = window(0.0)
    i = 0
    sup_seen = srv.stats()["superseded"]
    next_report = 10.0
    while True:
        now = srv.clock() - t0
        while i == len(at) and t_next < args.sim_seconds and t_next <= now + win:
            at, ac, t_next = window(t_next)
            i = 0
        j = np.searchsorted(at, now, side="right")
        if j > i:
            idx = ac[i:j]
            tk = srv.submit_many(idx, rec_s[idx], rec_p[idx], u0_ptr[idx], t0 + at[i:j])
            if tk[-1] - tk_base >= len(t_arr):
                t_arr = np.concatenate([t_arr, np.full(len(t_arr) // 2 + j - i, np.nan)])
            t_arr[tk - tk_base] = t0 + at[i:j]
            outstanding += j - i
            n += j - i
            i = j
        tk, tm = srv.poll()
        if len(tk):
            lat.append(tm - t_arr[tk - tk_base])
            outstanding -= len(tk)
        if args.supersede:
            sup = srv.stats()["superseded"]
            outstanding -= sup - sup_seen
            sup_seen = sup
        if now >= next_report:
            print(f"serve: {now:.0f} s of {args.sim_seconds:g}, {n} requests, {outstanding} outstanding",
                  file=sys.stderr, flush=True)
            next_report += 10.0
        done_arriving = i == len(at) and t_next >= args.sim_seconds
        if done_arriving and not outstanding:
            break
        if done_arriving:
            srv.drain()
    lat = np.concatenate(lat) if lat else np.zeros(1)
    t_end = srv.clock() - t0
    st = srv.stats()
    lat = lat * 1e3
    n_sup = st["superseded"]
    out = {"metric": "served MPC QP solves/sec with p50/p95/p99 arrival-to-result latency",
           "value": (n - n_sup) / t_end, "unit": "solves/s", "n_gpus": 1, "higher_is_better": True,
           "dtype": {"fp32": "f32", "bf16": "bf16+f32", "fp16": "f16+f32", "fp32mfma": "f32"}[args.serve_precision],
           "data": "synthetic",
           "config": {"workload": f"{nc} controllers, Poisson {args.rate_hz:g} Hz each, "
                                  f"{args.sim_seconds:g} s, N ~ U{{5..20}}, half humanoid (48, 30), "
                                  "half quadruped (36, 24), warm-started", "controllers": nc,
                      "offered_rate": nc * args.rate_hz, "requests": int(n),
                      "admm_iters": args.iters, "hbm_budget_gb": args.hbm_budget_gb,
                      "max_batch": args.max_batch, "max_inflight": args.max_inflight,
                      "supersede": bool(args.supersede)},
           "superseded": int(n_sup), "superseded_per_s": n_sup / t_end,
           "latency_ms": {"p50": float(np.percentile(lat, 50)), "p95": float(np.percentile(lat, 95)),
                          "p99": float(np.percentile(lat, 99)), "max": float(lat.max())},
           "server": {k: st[k] for k in ("batches", "evictions", "resident_controllers",
                                         "resident_bytes")},
           "wall_s": t_end}
    print(json.dumps(out))


def rti(args):
    """The real-time iteration's control step on the N = 10 humanoid workload
    (4096 agents, --precision io) with the articulated humanoid tree holding
    its pose (balance costs, both feet in stance): linearise the
    dynamics about the current solution (mpc_linearize, written into the
    batch's A, B, c), solve the QP warm-started (mpc_solve), command joint
    torques from its first stage (mpc_rti_torque), step the plant on the
    linearised dynamics (mpc_advance_state).  Each part is timed with events on
    the one stream; the first linearisation is about seeded configurations."""
    import torch

    from paper_2510_12717_amd import mpc, synth

    torch.cuda.set_device(0)
    n, N = args.agents, args.horizon
    model = synth.articulated_model("humanoid", seed=3)
    robot = mpc.RobotModel(model)
    sh = synth.humanoid(N)
    prec = args.precision
    npd = np.float64 if prec == "fp64" else np.float32
    b = synth.make_batch([sh] * n, seed=0, stream_id=1, dtype=npd)
    prob = mpc.to_device(b, prec)
    plan = mpc.Plan(b.shapes, precision=prec, iters=args.iters, no_slip=1 if args.no_slip else 0,
                    kernel=args.kernel)
    st = synth.model_states(model, n * (N + 1), seed=5)
    X = torch.from_numpy(np.concatenate([st["q"], st["qd"]], 1).reshape(n, N + 1, sh.nx)
                         .astype(npd)).cuda()
    U = torch.from_numpy(np.ascontiguousarray(
        np.concatenate([st["tau"], st["F"]], 1).reshape(n, N + 1, sh.nu)[:, :N]
        .astype(npd))).cuda()
    # a balancing task: hold each agent's first configuration at rest (base
    # height 0.6 m, level, joints at zero), both feet in stance
    nq = sh.nx // 2
    hold = X[:, 0].clone()
    hold[:, 2] = 0.6
    hold[:, 3:nq] = 0.0
    hold[:, nq:] = 0.0
    prob["x_ref"].copy_(hold[:, None, :].expand(n, N + 1, sh.nx).reshape(-1))
    qw = torch.cat([torch.tensor([10.0, 10.0, 100.0, 100.0, 100.0, 100.0]), torch.full((nq - 6,), 10.0),
                    torch.ones(nq)]).to(X.dtype)
    rw = torch.cat([torch.full((sh.n_tau,), 1e-3), torch.full((sh.nu - sh.n_tau,), 1e-5)]).to(X.dtype)
    prob["q"].copy_(qw.repeat(n))
    prob["r"].copy_(rw.repeat(n))
    prob["stance"].fill_(1)
    prob["tau_max"].fill_(200.0)
    prob["mu"].fill_(0.8)
    prob["x0"].copy_(X[:, 0].reshape(-1))
    if args.no_slip:  # the feet's no-slip rows, re-linearised every step with A, B, c
        prob["J_foot"] = torch.empty(n * sh.n_feet * sh.foot_dim * sh.nx, dtype=X.dtype, device="cuda")
    sol = mpc.solution_buffers(b.shapes, prec)
    if args.no_slip:
        nzc = n * N * sh.n_feet * sh.foot_dim
        sol["zc"] = torch.empty(nzc, dtype=X.dtype, device="cuda")
        sol["yc"] = torch.empty(nzc, dtype=X.dtype, device="cuda")
    sol["x"], sol["u"] = X.view(-1), U.view(-1)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1234)
    noise = torch.empty((args.warmup + args.steps, n * sh.nx), dtype=X.dtype, device="cuda")
    noise.normal_(0.0, 1e-3, generator=gen)
    stream = torch.cuda.current_stream()
    dt, kp, kd = 0.02, 150.0, 5.0
    parts = ("linearize", "solve", "torque", "advance")
    acc = {k: 0.0 for k in parts}
    lin_status = torch.zeros(n, dtype=torch.int32, device="cuda")

    def step(i, warm, timed):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)] if timed else None
        if timed:
            ev[0].record(stream)
        _, _, _, ls = robot.linearize(X, U, dt, out=(prob["A"], prob["B"], prob["c"]),
                                      J_foot=prob.get("J_foot"), stream=stream)
        lin_status.bitwise_or_(ls)
        if timed:
            ev[1].record(stream)
        plan.solve(prob, warm_start=warm, stream=stream)
        plan.get_solution(stream=stream, out=sol)
        if timed:
            ev[2].record(stream)
        tau = robot.rti_torque(dt, kp, kd, X, U, prob["x0"].view(n, sh.nx), stream=stream)
        if timed:
            ev[3].record(stream)
        plan.advance_state(prob, noise[i], prob["x0"], stream=stream)
        if timed:
            ev[4].record(stream)
        return ev, tau

    bad_by_step = []
    for i in range(args.warmup):
        step(i, i > 0, False)
        bad_by_step.append(int((sol["status"] >= 2).sum()))
    torch.cuda.synchronize()
    evs = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev, tau = step(args.warmup + i, True, True)
        evs.append(ev)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps * 1e3
    for ev in evs:
        for k, name in enumerate(parts):
            acc[name] += ev[k].elapsed_time(ev[k + 1])
    status = sol["status"].cpu().numpy()
    out = {"mode": "rti", "workload": f"humanoid tree (6 + 18 coordinates, two 6D feet), {n} agents, N = {N}",
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall,
           "steps_per_s_per_agent": 1e3 / wall,
           "part_ms": {k: v / args.steps for k, v in acc.items()},
           "linearize_status_ok": bool(int(lin_status.abs().sum()) == 0),
           "linearize_status_counts": {str(k): int(v) for k, v in
                                       zip(*np.unique(lin_status.cpu().numpy(), return_counts=True))},
           "qp_status_ok": bool(np.isin(status, (0, 1)).all()),
           "qp_status_counts": {str(k): int(v) for k, v in zip(*np.unique(status, return_counts=True))},
           "qp_failed_after_warmup_steps": bad_by_step,
           "max_abs_x_finite_agents": float(X[torch.isfinite(X).flatten(1).all(1)].abs().max()),
           "torque_finite": bool(torch.isfinite(tau).all()),
           "iters": args.iters, "precision": prec, "no_slip_rows": bool(args.no_slip),
           "families": sorted({g["family"] for g in plan.groups()}),
           "dtype": ("f64" if prec == "fp64" else "f32 io, f64 dynamics and Riccati factor")}
    print(json.dumps(out))
    plan.close()
    robot.close()


def scan(args):
    """The parallel-in-time Riccati factor against the serial one on long
    horizons: FP32 plans of humanoid agents (generic kernels, 50 cold
    iterations), factor time per solve from the plan's phase timers and the
    whole solve, for a few batch sizes at N = 40 (about the longest horizon whose
    humanoid iterate fits the generic kernel's LDS) and N = 20."""
    import torch

    from paper_2510_12717_amd import mpc, synth

    torch.cuda.set_device(0)
    rows = []
    for n, N in ((4, 40), (16, 40), (64, 40), (256, 40), (1024, 40), (64, 20), (1024, 20)):
        b = synth.make_batch([synth.humanoid(N)] * n, seed=0, stream_id=1, dtype=np.float32)
        prob = mpc.to_device(b, "fp32")
        row = {"agents": n, "N": N}
        for name, kw in (("serial", {}), ("scan", {"riccati_scan": 1})):
            plan = mpc.Plan(b.shapes, precision="fp32", iters=args.iters, kernel="generic", **kw)
            for _ in range(2):
                plan.solve(prob)
            torch.cuda.synchronize()
            plan.set_timing(True)
            t0 = time.perf_counter()
            reps = 5
            for _ in range(reps):
                plan.solve(prob)
            torch.cuda.synchronize()
            tm = plan.get_timing()
            row[name] = {"solve_ms": (time.perf_counter() - t0) / reps * 1e3,
                         "factor_ms": tm["factor"][0] / max(tm["factor"][1], 1)}
            st = plan.get_solution()["status"]
            row[name]["status_ok"] = bool((st == 0).all().item())
            plan.close()
        rows.append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)
    print(json.dumps({"mode": "riccati_scan", "iters": args.iters, "rows": rows}))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU per process; --gpus must be 1 "
                                   "(agents are independent: a batch shards across GPUs with no exchange)"}))
        sys.exit(2)
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc)
        return
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.serve:
        serve(args)
        return
    if args.inner:
        inner(args)
        return
    if args.rti:
        rti(args)
        return
    if args.scan:
        scan(args)
        return
    if args.uneven:
        uneven(args)
        return
    if args.mixed:
        mixed(args)
        return
    if args.scaled:
        scaled(args)
        return
    import torch

    import oracle
    from paper_2510_12717_amd import mpc, synth

    torch.cuda.set_device(0)
    shape = synth.humanoid(args.horizon)
    batch = synth.make_batch([shape] * args.agents, seed=0, stream_id=1,
                             dtype=np.float64 if args.precision == "fp64" else np.float32)
    rkw = (dict(max_refine_sweeps=args.refine_sweeps, refine_tol=1e-6)
           if args.precision == "fp32r" else {})
    plan = mpc.Plan(batch.shapes, precision=args.precision, iters=args.iters, kernel=args.kernel, **rkw)
    prob = mpc.to_device(batch, args.precision)
    td = prob["A"].dtype
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1234)
    noise = torch.empty((args.warmup + args.steps, args.agents * shape.nx), dtype=td,
                        device="cuda")
    noise.normal_(0.0, 1e-2, generator=gen)
    x0_init = prob["x0"].clone()

    stream = torch.cuda.current_stream()

    def step(i, warm):
        plan.solve(prob, warm_start=warm, stream=stream)
        plan.advance_state(prob, noise[i], prob["x0"], stream=stream)

    # correctness spot check of the first (cold) step against the FP64 oracle
    plan.solve(prob, warm_start=False, stream=stream)
    sol = plan.get_solution(stream=stream)
    torch.cuda.synchronize()
    nchk = min(args.check_agents, args.agents)
    chk_ids = np.linspace(0, args.agents - 1, nchk).astype(int)
    sub = synth.make_batch([shape] * nchk, seed=0, stream_id=1, agent_ids=chk_ids)
    ref = oracle.solve_batch(sub, iters=args.iters)
    err_u0, err_traj = sampled_errors(sol, ref, chk_ids, shape, args.agents)
    status_ok = bool((sol["status"] == 0).all().item())

    # warmup (closed loop from the initial state)
    prob["x0"].copy_(x0_init)
    for i in range(args.warmup):
        step(i, warm=i > 0)
    torch.cuda.synchronize()

    plan.set_timing(True)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        step(args.warmup + i, warm=True)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    timing = plan.get_timing()
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    # status of every agent after the last timed step (a failed agent still counts as a
    # launched solve in `value`, so failures are reported beside it)
    n_bad = int((plan.get_solution(stream=stream)["status"] != 0).sum().item())

    # one more (untimed) warm step from the GPU's own resident iterate after the timed
    # loop, checked against the oracle started from that same iterate and x0
    plan.set_timing(False)
    prev = plan.get_solution(stream=stream)
    torch.cuda.synchronize()
    warm = {k: prev[k].cpu().numpy().astype(np.float64).reshape(args.agents, -1)[chk_ids].ravel()
            for k in ("u", "z", "y")}
    x0_chk = prob["x0"].cpu().numpy().astype(np.float64).reshape(args.agents, -1)[chk_ids].ravel()
    plan.solve(prob, warm_start=True, stream=stream)
    sol_w = plan.get_solution(stream=stream)
    torch.cuda.synchronize()
    ref_w = oracle.solve_batch(sub, iters=args.iters, warm=warm, x0=x0_chk)
    err_u0_w, err_traj_w = sampled_errors(sol_w, ref_w, chk_ids, shape, args.agents)
    solves = args.agents * args.steps
    value = solves / wall

    # dominant kernel: the ADMM-iteration launch (the factor is its own kernel)
    cfg = plan.config()
    admm_ms, admm_n = timing["admm"]
    fac_ms, fac_n = timing["factor"]
    avg_admm_s = admm_ms / max(admm_n, 1) * 1e-3
    fl_iter = flops_iter_stage(shape.nx, shape.nu) * shape.N * args.iters * args.agents
    peak = PEAK["alu_f64"] if args.precision == "fp64" else PEAK["alu_f32"]
    achieved = fl_iter / avg_admm_s
    kname = ("k_admm_resident<%d, %d, false>" % (shape.nx, shape.nu) if cfg["kernel"] == "fused"
             else "k_admm<%s>" % ("double" if args.precision == "fp64" else "float"))
    traffic = recorded_traffic() if cfg["kernel"] == "fused" else None
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12,
                "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
                "kernel": kname, "avg_launch_ms": avg_admm_s * 1e3,
                "flops_per_launch": fl_iter}

    # CPU baseline: the FP64 oracle, warm-started closed loop on a bounded sample
    cpu = None
    if args.cpu_seconds > 0:
        n_s = min(args.agents, 512)
        cb = synth.make_batch([shape] * n_s, seed=0, stream_id=1)
        threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
        t1 = time.perf_counter()
        steps_done, state, x0 = 0, None, cb.x0.copy()
        while True:
            o = oracle.solve_batch(cb, iters=args.iters, warm=state, x0=x0, n_threads=threads)
            state = {k: o[k] for k in ("u", "z", "y")}
            x0 = oracle.advance_batch(cb, x0, o["u"], synth.step_noise(cb, steps_done))
            steps_done += 1
            if time.perf_counter() - t1 >= args.cpu_seconds or steps_done >= 200:
                break
        cpu_wall = time.perf_counter() - t1
        cpu = {"value": n_s * steps_done / cpu_wall, "unit": "solves/s", "cores": int(o["threads"]),
               "kind": "oracle",
               "sample": f"{n_s} agents x {steps_done} warm-started control steps of the same "
                         f"workload (FP64 C oracle, OpenMP over agents)"}

    out = {
        "metric": "MPC QP solves/sec at 4096 agents N=10 + p99 latency; FP32/BF16 vs FP64 error",
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32", "data": "synthetic",
        "config": {"workload": f"{args.agents} humanoid agents (nx=48, nu=30), N={shape.N}, "
                               f"{args.iters} warm-started ADMM iterations per control step, "
                               "closed loop with plant noise",
                   "agents": args.agents, "N": shape.N, "nx": shape.nx, "nu": shape.nu,
                   "admm_iters": args.iters, "precision": args.precision,
                   "kernel": cfg["kernel"], "threads_per_agent": cfg["threads_per_agent"],
                   "lds_bytes": cfg["lds_bytes"], "parallelism": "agents (1 GPU)"},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "max": float(lat.max())},
        "kernel_ms": {"factor": fac_ms / max(fac_n, 1), "admm": admm_ms / max(admm_n, 1),
                      "residual": timing["residual"][0] / max(timing["residual"][1], 1)},
        "err_vs_fp64": {"u0": err_u0, "trajectory": err_traj, "agents_checked": int(nchk),
                        "status_ok": status_ok,
                        "after_timed_loop": {"u0": err_u0_w, "trajectory": err_traj_w,
                                             "steps_before": args.warmup + args.steps}},
        "agents_not_ok_after_timed_loop": n_bad,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
