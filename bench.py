#!/usr/bin/env python3
"""Throughput of the loss-gradient step of the transformer density operator
on one MI355X, BF16-MFMA path against the plain FP32 path.

One step = one call of tdo_loss_grad (gradient estimator of mode B) on the
dissipative Ising chain N = 32 (V = 2, g drawn from U[0.5, 2], gamma = 1),
transformer d = 64, 8 heads, 4 layers, MLP 256, B = 65536 samples: the
Lindbladian rows of every sample, the forward pass over every connected
configuration (two passes each), L_loc, the FP64 loss reduction, the backward
pass of every layer and the FP64 gradient reduction.  Inputs are synthetic
(seeded parameters at the N(0, 0.02) initialisation and i.i.d. uniform
configurations) and resident in HBM before the timed region.

Printed: one JSON line on stdout.  value = configurations per second of the
BF16 path, where a configuration is one evaluated log rho (a sample or one of
its nonzero Lindbladian row entries), each costing two transformer passes.
Progress goes to stderr.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "configs/sec fwd+bwd (loss grad), BF16-MFMA vs FP32 GPU at matched loss error"
PEAK_TFLOPS = {"bf16": 2500.0, "fp32": 157.3}  # MI355X dense MFMA
KERNELS = ("fwd_layer", "bwd_mlp", "bwd_attn")
# Source files whose change invalidates a recorded HBM-traffic measurement.
KERNEL_SOURCES = {
    "fwd_layer": ("net_fwd.hip", "net.h", "netapi.h"),
    "bwd_mlp": ("net_bwd_mlp.hip", "net.h", "netapi.h"),
    "bwd_attn": ("net_bwd_attn.hip", "net.h", "netapi.h"),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_flops_per_unit(kernel, n, d, m):
    """Algorithmic FLOPs of one configuration-pass through one layer.

    forward: QKV 6nd^2, W_O 2nd^2, scores and P.V 4n^2 d, MLP 4ndm;
    backward of the MLP: input gradient 4ndm + weight gradients 4ndm;
    backward of attention: input and weight gradients of QKV and W_O 16nd^2,
    dP, dV, dQ, dK 8n^2 d.  Recomputation is not counted."""
    if kernel == "fwd_layer":
        return 8 * n * d * d + 4 * n * n * d + 4 * n * d * m
    if kernel == "bwd_mlp":
        return 8 * n * d * m
    if kernel == "bwd_attn":
        return 16 * n * d * d + 8 * n * n * d
    raise ValueError(kernel)


def sources_digest(kernel):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2502_20723_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel, workload):
    """HBM bytes per launch from the committed counter summary, or None when
    there is none or the kernel's sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("sources_sha256") != sources_digest(kernel):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precs", default="fp32,bf16")
    ap.add_argument("--fp32-steps", type=int, default=3,
                    help="timed steps of the FP32 comparison leg (at most --steps; one step is about 17 s)")
    # 128 GiB of the 288 GB of HBM: fewer, larger chunks (each chunk pays the per-chunk
    # evaluation-list, loss and reduction launches and a launch tail per kernel)
    ap.add_argument("--workspace-gib", type=float, default=128.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true",
                    help="skip the loss check against the oracle (it runs in the oracle leg, with the CPU baseline)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched-workload and sampler measurements (BF16, reported beside the headline)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one elementwise copy of this many MiB (HBM counter calibration)")
    ap.add_argument("--lindblad-only", action="store_true",
                    help="measure only tdo_connected and tdo_local_lindbladian (HBM-bound) and print their line")
    ap.add_argument("--batched-only", action="store_true",
                    help="measure only the batched workload (64 uneven problems) and print its line")
    ap.add_argument("--sampler-only", action="store_true", help="measure only the sampler and print its line")
    ap.add_argument("--observables-only", action="store_true",
                    help="measure only the observables, purity and diagonal sampler and print their line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the samples shard "
              f"across GPUs with one all-reduce of the gradient, which this build does not run.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2502_20723_amd import synth, tdo

    name = "ising_n32"
    wl = synth.workload(name)
    arch, model, B = wl["arch"], wl["model"], wl["B"]
    n, d, m, L = model["n"], arch["d"], arch["mlp"], arch["layers"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    params_np = synth.params(arch, wl["seed"], "init")
    cfg_np = synth.configs(n, B, 3000)
    params = torch.from_numpy(params_np).to(dev)
    cfg = torch.from_numpy(cfg_np).to(dev)
    ctx = tdo.Ctx(0, int(args.workspace_gib * (1 << 30)))
    log(f"bench: {name} n={n} B={B} arch={arch} g={model['g']:.6f} P={tdo.num_params(arch)}")

    # configurations evaluated per step: every sample plus its nonzero off-diagonal row entries
    conn, _, ncon = ctx.connected(model, cfg)
    diag_present = (conn[:, 0, 0] == cfg[:, 0]) & (conn[:, 0, 1] == cfg[:, 1])
    E_step = int(ncon.sum().item()) + int((~diag_present).sum().item())
    del conn
    # configuration-passes per layer per step: two passes of every evaluated configuration.  Mode B's
    # second forward and backward over the B samples (the centring term, formed once F is known)
    # is implementation work and is not counted.
    units_step = 2 * E_step
    log(f"bench: {E_step} configurations per step (K_avg {E_step / B:.2f})")

    if args.copy_calibration_mib:
        nel = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.ones(nel, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        log(f"bench: calibration copy of {args.copy_calibration_mib} MiB done")
        del src, dst

    if args.lindblad_only or args.batched_only or args.sampler_only or args.observables_only:
        if args.observables_only:
            line = {"metric": "mixed-state observables, samples/s",
                    "observables": bench_observables(ctx, arch, params, n, synth),
                    "ising2d_4x8": bench_lattice2d(ctx, synth),
                    "sr": bench_sr(ctx, arch, params, n, synth)}
        elif args.lindblad_only:
            line = {"metric": "Lindbladian rows and L_loc, algorithmic HBM GB/s",
                    "lindblad": bench_lindblad(ctx, tdo, model, synth, args.steps)}
        elif args.batched_only:
            line = {"metric": "batched workload, configs/s", "batched_uneven": bench_batched(ctx, tdo, synth, args.steps)}
        else:
            line = {"metric": "Metropolis sampler, proposals/s", "sampler": bench_sampler(ctx, arch, params, n, synth)}
        print(json.dumps(line), flush=True)
        ctx.close()
        return

    results = {}
    stream = torch.cuda.current_stream()
    tuned = {}
    for prec in [p for p in args.precs.split(",") if p]:
        # the library's tile-shape tuner for this workload (untimed; the timed steps use its choice)
        fw, fg, mw = ctx.autotune(arch, params, model, cfg, prec, "B")
        tuned[prec] = {"fwd_waves_per_workgroup": fw, "fwd_workgroups_per_cu": fg, "bwd_mlp_waves_per_workgroup": mw}
        log(f"bench: {prec} tuned shapes {tuned[prec]}")
    for prec in [p for p in args.precs.split(",") if p]:
        steps = args.steps if prec == "bf16" else max(1, min(args.steps, args.fp32_steps))
        warmup = args.warmup if prec == "bf16" else min(args.warmup, 1)
        for i in range(warmup):
            t0 = time.time()
            loss, grad, _ = ctx.loss_grad(arch, params, model, cfg, None, prec, "B")
            torch.cuda.synchronize()
            log(f"bench: {prec} warmup step {i} {time.time() - t0:.2f} s loss {float(loss[0]):.6e}")
        torch.cuda.synchronize()
        ctx.profile(True)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for i in range(steps):
            loss, grad, _ = ctx.loss_grad(arch, params, model, cfg, None, prec, "B")
            if i == 0 or i == steps - 1:
                log(f"bench: {prec} step {i} queued")
        ev1.record(stream)
        torch.cuda.synchronize()
        total_ms = ev0.elapsed_time(ev1)
        kt = {k: ctx.profile_read(k) for k in KERNELS}
        ctx.profile(False)
        ms = total_ms / steps
        r = dict(ms_per_step=ms, steps=steps, tuned_shapes=tuned[prec], configs_per_s=E_step / (ms / 1e3),
                 loss=float(loss[0]),
                 grad_norm=float(torch.linalg.vector_norm(grad).item()), kernels={})
        for k, (kms, cnt) in kt.items():
            fl = kernel_flops_per_unit(k, n, d, m) * units_step * L * steps
            r["kernels"][k] = dict(total_ms=kms, launches=cnt, avg_launch_ms=kms / max(cnt, 1),
                                   share=kms / total_ms, tflops=fl / (kms / 1e3) / 1e12 if kms > 0 else 0.0,
                                   flops_per_launch=fl / max(cnt, 1))
        step_flops = sum(kernel_flops_per_unit(k, n, d, m) for k in KERNELS) * units_step * L
        r["step"] = dict(flops=step_flops, tflops=step_flops / (ms / 1e3) / 1e12,
                         frac_of_peak=step_flops / (ms / 1e3) / 1e12 / PEAK_TFLOPS[prec])
        results[prec] = r
        log(f"bench: {prec} {ms:.1f} ms/step, {r['configs_per_s'] / 1e6:.3f} M configs/s; kernels " +
            ", ".join(f"{k} {v['share'] * 100:.0f}% {v['tflops']:.0f} TF/s" for k, v in r["kernels"].items()))

    main_prec = "bf16" if "bf16" in results else next(iter(results))
    R = results[main_prec]
    dom = max(R["kernels"], key=lambda k: R["kernels"][k]["total_ms"])
    kd = R["kernels"][dom]
    achieved = kd["tflops"]
    roofline = dict(bound="mfma", kernel=dom, achieved=achieved, peak=PEAK_TFLOPS[main_prec], unit="TFLOP/s",
                    frac=achieved / PEAK_TFLOPS[main_prec], traffic=recorded_traffic(dom, name),
                    avg_launch_ms=kd["avg_launch_ms"], flops_per_launch=kd["flops_per_launch"],
                    flops_per_unit=kernel_flops_per_unit(dom, n, d, m),
                    unit_def="one configuration-pass through one layer",
                    whole_step_frac=R["step"]["frac_of_peak"], target_frac_n32=0.40)

    extras = None
    if not args.no_extras:
        extras = {"ising_n8": bench_small(ctx, tdo, synth, "ising_n8", args.steps),
                  "xyz_n16": bench_small(ctx, tdo, synth, "xyz_n16", args.steps),
                  "batched_uneven": bench_batched(ctx, tdo, synth, args.steps),
                  "batched_uneven_fp32": bench_batched(ctx, tdo, synth, 1, "fp32"),
                  "sampler": bench_sampler(ctx, arch, params, n, synth),
                  "observables": bench_observables(ctx, arch, params, n, synth),
                  "ising2d_4x8": bench_lattice2d(ctx, synth),
                  "sr": bench_sr(ctx, arch, params, n, synth),
                  "lindblad": bench_lindblad(ctx, tdo, model, synth, args.steps)}

    # the oracle leg (host): timed on a bounded sample, and (unless --no-check) the FP64 loss and
    # gradient of 16 sampled rows of the same batch, at the benchmark's weights and at "mid" weights
    # (where log rho varies across configurations, so that BF16 rounding shows), against which
    # the GPU's loss and gradient on those rows are compared (weights zero on the other rows)
    cpu, accuracy = None, None
    pick = np.sort(np.random.default_rng(7).choice(B, 16, replace=False))
    if not args.no_cpu_baseline:
        params_mid = synth.params(arch, wl["seed"], "mid")
        cpu, refs = cpu_baseline(arch, model, params_np, cfg_np,
                                 None if args.no_check else {"init": params_np, "mid": params_mid}, pick)
        if refs:
            w = torch.zeros(B, dtype=torch.float64, device=dev)
            w[torch.from_numpy(pick).to(dev)] = 1.0
            accuracy = {"rows": "16 uniformly drawn samples of the batch (ReLU kink units included)"}
            for scale, (F_ref, g_ref) in refs.items():
                p_dev = params if scale == "init" else torch.from_numpy(params_mid).to(dev)
                accuracy[scale] = {}
                for prec in results:
                    lg, gg, _ = ctx.loss_grad(arch, p_dev, model, cfg, w, prec, "B")
                    gerr = float(np.linalg.norm(gg.cpu().numpy() - g_ref) / np.linalg.norm(g_ref))
                    accuracy[scale][prec] = {"loss_rel_err": abs(float(lg[0]) - F_ref) / abs(F_ref),
                                             "grad_rel_l2_err": gerr}
            log(f"bench: errors vs FP64 oracle on 16 sampled rows: {accuracy}")

    out = {
        "metric": METRIC,
        "value": R["configs_per_s"],
        "unit": "configs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": R["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": main_prec,
        "data": "synthetic",
        "config": {"workload": f"{name}: dissipative Ising chain n=32 V=2 g={model['g']:.4f} gamma=1, "
                               f"d=64 heads=8 layers=4 mlp=256, B=65536, gradient mode B",
                   "B": B, "n": n, "configs_per_step": E_step, "parallelism": "single GPU"},
        "fp32_value": results.get("fp32", {}).get("configs_per_s"),
        "speedup_bf16_over_fp32": (results["bf16"]["configs_per_s"] / results["fp32"]["configs_per_s"]
                                   if "bf16" in results and "fp32" in results else None),
        "loss_rel_err_vs_oracle": ({p: v["loss_rel_err"] for p, v in accuracy["mid"].items()} if accuracy else None),
        "errors_vs_oracle": accuracy,
        "per_precision": results,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def evaluated_configs(ctx, model, cfg):
    """Configurations evaluated for these samples: each sample plus its nonzero
    off-diagonal Lindbladian entries."""
    conn, _, ncon = ctx.connected(model, cfg)
    diag = (conn[:, 0, 0] == cfg[:, 0]) & (conn[:, 0, 1] == cfg[:, 1])
    return int(ncon.sum().item()) + int((~diag).sum().item())


def bench_small(ctx, tdo, synth, name, steps):
    """A smaller workload (Ising n = 8 at width 32, B = 4096; XYZ n = 16 at width 64 with
    4 heads, B = 16384), FP32 and BF16: configurations per second of tdo_loss_grad (mode
    B, forward and backward) and of tdo_log_rho alone over the same evaluated
    configurations (each sample and its nonzero off-diagonal entries, gathered before
    timing), with the BF16 speed-ups."""
    import torch
    wl = synth.workload(name)
    arch, model, B = wl["arch"], wl["model"], wl["B"]
    params = torch.from_numpy(synth.params(arch, wl["seed"], "init")).cuda()
    cfg = torch.from_numpy(synth.configs(model["n"], B, 3000)).cuda()
    E = evaluated_configs(ctx, model, cfg)
    conn, _, ncon = ctx.connected(model, cfg)
    kmax = conn.shape[1]
    valid = torch.arange(kmax, device=cfg.device)[None, :] < ncon[:, None].long()
    ci, xi = conn.view(torch.int64), cfg.view(torch.int64)  # (index and compare as int64 bit patterns)
    offd = valid & ~((ci[:, :, 0] == xi[:, None, 0]) & (ci[:, :, 1] == xi[:, None, 1]))
    evalset = torch.cat([xi, ci[offd]], 0).contiguous().view(torch.uint64)
    del conn
    assert evalset.shape[0] == E
    res = {"n": model["n"], "arch": arch, "B": B, "configs_per_step": E}
    for prec in ("fp32", "bf16"):
        ctx.log_rho(arch, params, model["n"], evalset, prec)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(8):
            ctx.log_rho(arch, params, model["n"], evalset, prec)
        e1.record()
        torch.cuda.synchronize()
        res["forward_" + prec] = {"ms": e0.elapsed_time(e1) / 8, "configs_per_s": E / (e0.elapsed_time(e1) / 8 / 1e3)}
    res["forward_speedup_bf16_over_fp32"] = res["forward_bf16"]["configs_per_s"] / res["forward_fp32"]["configs_per_s"]
    for prec in ("fp32", "bf16"):
        ctx.loss_grad(arch, params, model, cfg, None, prec, "B")
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 4 * max(steps, 1)
        e0.record()
        for _ in range(reps):
            ctx.loss_grad(arch, params, model, cfg, None, prec, "B")
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[prec] = {"ms_per_step": ms, "configs_per_s": E / (ms / 1e3)}
    res["speedup_bf16_over_fp32"] = res["bf16"]["configs_per_s"] / res["fp32"]["configs_per_s"]
    log(f"bench: {name} B={B} ({E} configurations): loss+gradient fp32 {res['fp32']['configs_per_s'] / 1e6:.3f} M/s, "
        f"bf16 {res['bf16']['configs_per_s'] / 1e6:.3f} M/s ({res['speedup_bf16_over_fp32']:.1f}x); forward fp32 "
        f"{res['forward_fp32']['configs_per_s'] / 1e6:.2f} M/s, bf16 {res['forward_bf16']['configs_per_s'] / 1e6:.2f} M/s "
        f"({res['forward_speedup_bf16_over_fp32']:.1f}x)")
    return res


def bench_batched(ctx, tdo, synth, steps, prec="bf16"):
    """64 problems (n in [8, 40], half Ising half XYZ, own parameters), 2048 samples
    each, mode B, one tdo_loss_grad_batched call per step: eager call, recording
    call, then `steps` timed graph replays on a side stream."""
    import torch
    wl = synth.WORKLOADS["batched_uneven"]
    arch = wl["arch"]
    models = synth.uneven_problems(wl["problems"], wl["seed"])
    params = [torch.from_numpy(synth.params(arch, wl["seed"] + 7 * i, "init")).cuda() for i in range(len(models))]
    cfgs = [torch.from_numpy(synth.configs(m["n"], wl["B"], wl["seed"] + 11 * i)).cuda() for i, m in enumerate(models)]
    E = sum(evaluated_configs(ctx, m, c) for m, c in zip(models, cfgs))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        P = tdo.num_params(arch)
        out = (torch.empty(len(models), dtype=torch.float64, device="cuda"),
               [torch.empty(P, dtype=torch.float64, device="cuda") for _ in models])
        for _ in range(2):  # eager (sizes, autotunes), then recorded
            ctx.loss_grad_batched(arch, params, models, cfgs, None, prec, "B", out=out)
        s.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(steps):
            ctx.loss_grad_batched(arch, params, models, cfgs, None, prec, "B", out=out)
        e1.record(s)
        s.synchronize()
    ms = e0.elapsed_time(e1) / steps
    log(f"bench: batched workload {len(models)} problems, {E} configurations: {ms:.1f} ms/step, "
        f"{E / ms * 1e3 / 1e6:.3f} M configs/s ({prec}, graph replay)")
    return {"value": E / (ms / 1e3), "unit": "configs/s", "ms_per_step": ms, "configs_per_step": E,
            "problems": len(models), "B": wl["B"], "dtype": prec, "steps": steps}


def bench_sampler(ctx, arch, params, n, synth):
    """Metropolis sampling with the n = 32 network: 65536 chains, one sweep (2n
    proposals each) after one untimed sweep, BF16."""
    import torch
    C = 65536
    state = torch.from_numpy(synth.configs(n, C, 4000)).cuda()
    lr = ctx.log_rho(arch, params, n, state, "bf16")
    _, ctr = ctx.sample(arch, params, n, state, lr, 1, 0, 1, 0.5, "bf16")
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    ctx.sample(arch, params, n, state, lr, 1, ctr, 1, 0.5, "bf16")
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    props = C * 2 * n
    log(f"bench: sampler {C} chains x {2 * n} proposals in {ms:.1f} ms: {props / ms * 1e3 / 1e6:.2f} M proposals/s")
    return {"value": props / (ms / 1e3), "unit": "proposals/s", "chains": C, "sweeps": 1, "ms": ms, "dtype": "bf16"}


def bench_sr(ctx, arch, params, n, synth, B=256, iters=100):
    """Stochastic reconfiguration with the n = 32 network: the per-sample Jacobian of
    B = 256 samples (2B backward passes, in BF16 and in FP32; the FP32 one feeds
    the solve), then 100 conjugate-gradient
    iterations of (S + lambda I) x = g with S = J^T J applied as two passes over
    J (2B x P FP64).  Algorithmic HBM bytes per iteration: 2 x 2B x P x 8 (J read
    twice) plus the vectors."""
    import numpy as np
    import torch
    P = params.shape[0]
    # "mid" weights: at the "init" scale the centred log-derivatives are so small
    # that CG converges in two iterations
    params = torch.from_numpy(synth.params(arch, 1003, "mid")).cuda()
    cfg = torch.from_numpy(synth.configs(n, B, 7000)).cuda()
    g = torch.from_numpy(np.random.default_rng(7001).standard_normal(P)).cuda()

    def timed(fn):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        out = fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1), out

    ctx.jacobian(arch, params, n, cfg[:2], "bf16")
    ms_jb, Jb = timed(lambda: ctx.jacobian(arch, params, n, cfg, "bf16"))
    ctx.jacobian(arch, params, n, cfg[:2], "fp32")
    ms_j, J = timed(lambda: ctx.jacobian(arch, params, n, cfg, "fp32"))
    jb_err = float(((Jb - J).norm(dim=2) / J.norm(dim=(1, 2))[:, None]).max())
    del Jb
    ctx.sr_solve(J.clone(), g, 1e-3, 2)
    ms_s, (x, info) = timed(lambda: ctx.sr_solve(J, g, 1e-3, iters))
    res = float(info.cpu()[0])
    # the matrix-free form at the loss-gradient batch: no Jacobian stored; per CG iteration one
    # forward-mode pass (FP32) and one reverse-mode pass over all the samples
    Bf, it_f = 65536, 4
    cfg_f = torch.from_numpy(synth.configs(n, Bf, 7002)).cuda()
    tan = torch.from_numpy(np.random.default_rng(7003).standard_normal(P) * 0.1).cuda()
    ctx.log_rho_jvp(arch, params, n, cfg_f[:64], tan)
    ms_jvp, _ = timed(lambda: ctx.log_rho_jvp(arch, params, n, cfg_f, tan))
    mf = {"B": Bf, "jvp_ms": ms_jvp, "jvp_configs_per_s": Bf / (ms_jvp / 1e3)}
    for prec in ("fp32", "bf16"):
        ms_mf, (xm, infom) = timed(lambda: ctx.sr_solve_matfree(arch, params, n, cfg_f, g, 1e-3, it_f, None, prec))
        mf[prec] = {"cg_iters": it_f, "ms": ms_mf, "ms_per_iter": ms_mf / it_f, "residual": float(infom.cpu()[0])}
    log(f"bench: SR matrix-free B={Bf}: jvp {ms_jvp:.1f} ms, CG iteration fp32 {mf['fp32']['ms_per_iter']:.1f} ms, "
        f"bf16 {mf['bf16']['ms_per_iter']:.1f} ms")
    it_bytes = 2 * (2 * B) * P * 8 + 6 * P * 8
    gbs = iters * it_bytes / (ms_s / 1e3) / 1e9
    log(f"bench: SR n={n} B={B} P={P}: jacobian {ms_j:.1f} ms ({2 * B / (ms_j / 1e3):.0f} rows/s; bf16 "
        f"{ms_jb:.1f} ms, rows within {jb_err:.1e} of fp32), "
        f"{iters} CG iterations {ms_s:.1f} ms ({gbs:.0f} GB/s algorithmic), residual {res:.2e}")
    return {"B": B, "P": P, "jacobian_ms": ms_j, "jacobian_rows_per_s": 2 * B / (ms_j / 1e3),
            "jacobian_bf16_ms": ms_jb, "jacobian_bf16_max_row_rel_diff_vs_fp32": jb_err, "cg_iters": iters,
            "cg_ms": ms_s, "cg_GB/s": gbs, "cg_frac_of_8TB/s": gbs / 8000.0, "residual": res, "lambda": 1e-3,
            "matrix_free": mf}


def bench_lattice2d(ctx, synth, B=16384):
    """The 2D dissipative Ising model on a 4 x 8 periodic lattice (n = 32) with the
    benchmark network, BF16 loss and gradient (mode B) over B = 16384 samples: the
    same kernels as the chain with the lattice's bond sum in the diagonal entries."""
    import torch
    wl = synth.workload("ising2d_4x8")
    arch, model = wl["arch"], wl["model"]
    params = torch.from_numpy(synth.params(arch, wl["seed"], "init")).cuda()
    cfg = torch.from_numpy(synth.configs(model["n"], B, 3000)).cuda()
    E = evaluated_configs(ctx, model, cfg)
    ctx.loss_grad(arch, params, model, cfg, None, "bf16", "B")
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        ctx.loss_grad(arch, params, model, cfg, None, "bf16", "B")
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 3
    log(f"bench: ising2d_4x8 B={B} ({E} configurations): loss+gradient bf16 {E / ms * 1e3 / 1e6:.3f} M/s")
    return {"lattice": [4, 8], "n": model["n"], "B": B, "configs_per_step": E, "ms_per_step": ms,
            "configs_per_s": E / (ms / 1e3), "dtype": "bf16"}


def bench_observables(ctx, arch, params, n, synth):
    """Mixed-state observables with the n = 32 network, BF16: local estimators of
    the three magnetisation components and their sign-weighted means over 65536
    samples (n + 1 = 33 network rows each), the purity over 32768 pairs (3 rows
    each), and the diagonal chain (65536 chains, one sweep of n proposals).  Each
    is timed with HIP events after one untimed call.  FLOP/s counts the forward
    layers' algorithmic FLOPs (two configuration-passes per row)."""
    import numpy as np
    import torch
    B, Pp, C = 65536, 32768, 65536
    d, m, L = arch["d"], arch["mlp"], arch["layers"]
    row_flops = 2 * L * (8 * n * d * d + 4 * n * n * d + 4 * n * d * m)
    alpha = torch.from_numpy(np.ascontiguousarray(synth.configs(n, B, 6000)[:, 0])).cuda()
    pairs = torch.from_numpy(synth.configs(n, Pp, 6001)).cuda()
    pa, pb = pairs[:, 0].contiguous(), pairs[:, 1].contiguous()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    out = {}
    ms = timed(lambda: ctx.observables(arch, params, n, alpha, "bf16"))
    rows = B * (n + 1)
    out["local_estimators"] = {"value": B / (ms / 1e3), "unit": "samples/s", "samples": B, "rows": rows, "ms": ms,
                               "tflops": rows * row_flops / (ms / 1e3) / 1e12, "dtype": "bf16"}
    ms = timed(lambda: ctx.purity(arch, params, n, pa, pb, "bf16"))
    out["purity"] = {"value": Pp / (ms / 1e3), "unit": "pairs/s", "pairs": Pp, "rows": 3 * Pp, "ms": ms,
                     "tflops": 3 * Pp * row_flops / (ms / 1e3) / 1e12, "dtype": "bf16"}
    state = alpha.clone()
    slr = ctx.log_rho(arch, params, n, torch.stack([state, state], 1).contiguous(), "bf16")
    ctr = [0]

    def chain():
        _, ctr[0] = ctx.sample_diag(arch, params, n, state, slr, 3, ctr[0], 1, "bf16")

    ms = timed(chain)
    out["diag_sampler"] = {"value": C * n / (ms / 1e3), "unit": "proposals/s", "chains": C, "sweeps": 1, "ms": ms,
                           "dtype": "bf16"}
    log("bench: observables " + ", ".join(f"{k} {v['value'] / 1e6:.2f} M {v['unit']}" for k, v in out.items()))
    return out


def bench_lindblad(ctx, tdo, model, synth, steps, B=1 << 20):
    """tdo_connected and tdo_local_lindbladian on 2^20 samples of the n = 32 Ising
    chain (kmax = 3n + 1): time per call and algorithmic HBM bytes over it, against
    the 8 TB/s peak.  Algorithmic bytes per sample: rows 16 (read x) + 4 (count) +
    24 per entry (written y and coefficient; slots beyond the count are not written);
    L_loc 8 + 4 + 8 (log rho(x), count, result) + 16 per entry (coefficient and
    log rho(y) read).  The library is called directly on preallocated outputs (the
    binding's zero-filled output tensors would add fill kernels to the timing)."""
    import ctypes

    import torch
    n = model["n"]
    kmax = 3 * n + 1
    cfg = torch.from_numpy(synth.configs(n, B, 5000)).cuda()
    gen = torch.Generator(device="cuda").manual_seed(5001)
    lr_x = 0.1 * torch.randn((B, 2), generator=gen, device="cuda")
    lr_conn = 0.1 * torch.randn((B, kmax, 2), generator=gen, device="cuda")
    conn, mel, ncon = ctx.connected(model, cfg, kmax)
    out = ctx.local_lindbladian(lr_x, mel, ncon, lr_conn)
    torch.cuda.synchronize()
    entries = int(ncon.sum().item())
    res = {}
    L, P, st, mt = tdo.lib(), tdo._ptr, tdo._stream, tdo.model_t(model)

    def rows():
        tdo._check(L.tdo_connected(ctx.h, ctypes.byref(mt), P(cfg), B, kmax, P(conn), P(mel), P(ncon), st()))

    def lloc():
        tdo._check(L.tdo_local_lindbladian(ctx.h, B, P(lr_x), P(mel), P(ncon), kmax, P(lr_conn), P(out), st()))

    for name, call, nbytes in (("connected", rows, B * 20 + entries * 24),
                               ("local_lindbladian", lloc, B * 20 + entries * 16)):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(max(steps, 1)):
            call()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / max(steps, 1)
        gbs = nbytes / (ms / 1e3) / 1e9
        res[name] = {"ms": ms, "bytes": nbytes, "GB/s": gbs, "frac_of_8TB/s": gbs / 8000.0}
        log(f"bench: {name} B={B} ({entries} entries): {ms:.3f} ms, {gbs:.0f} GB/s algorithmic "
            f"({100 * gbs / 8000:.1f}% of 8 TB/s)")
    del conn, mel, ncon, out, lr_conn
    return {"B": B, "n": n, "kmax": kmax, "entries": entries, "kernels": res}


def cpu_baseline(arch, model, params_np, cfg_np, ref_params=None, pick=None):
    """The oracle leg: the FP64 oracle's loss and gradient (mode B) on a bounded
    prefix of the same samples, timed on the host and scaled to configurations per
    second; and, for each named parameter vector in ref_params, the oracle's loss and
    gradient on the rows in pick (untimed).  Returns (baseline dict, {name: (F, grad)})."""
    import numpy as np
    import torch

    from oracle import ansatz as oa
    from oracle import lindblad as ol
    from oracle import vmc

    A, M = oa.Arch(**arch), ol.Model(**model)
    th = params_np.astype(np.float64)

    def run(S):
        rows = ol.connected(M, cfg_np[:S])
        E = sum(1 + sum(1 for y in r[0] if not (y[0] == c[0] and y[1] == c[1])) for r, c in zip(rows, cfg_np[:S]))
        t0 = time.time()
        vmc.loss_grad(th, A, M, cfg_np[:S], None, mode="B")
        return E, time.time() - t0

    E, t = run(2)
    S = int(min(max(2, round(2 * 15.0 / max(t, 1e-3))), 512))
    E, t = run(S)
    log(f"bench: oracle {S} samples ({E} configurations) in {t:.1f} s")
    refs = {}
    for name, p in (ref_params or {}).items():
        F, g, _ = vmc.loss_grad(p.astype(np.float64), A, M, cfg_np[pick], None, mode="B")
        refs[name] = (F, g)
    cpu_model = ""
    try:
        cpu_model = next(l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return ({"value": E / t, "unit": "configs/s", "cores": torch.get_num_threads(), "kind": "oracle",
             "host_cores": os.cpu_count(), "host_cpu": cpu_model,
             "sample": f"first {S} of the 65536 samples ({E} configurations), FP64 loss and gradient (mode B); "
                       f"cores = the threads torch used"},
            refs)


if __name__ == "__main__":
    main()
