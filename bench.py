#!/usr/bin/env python3
"""Benchmark of the batched quadrotor environment step on one MI355X.

One bench step = one whole rollout of the headline workload: 65536
domain-randomised envs x 1000 env steps (observation, actor MLP, RK4,
reward, termination, in-kernel reset) in the autotuned fused kernel, inputs
resident in HBM.  value = env-steps/s.  Also reported: the plain five-kernel
per-step path on the same batch, the fused kernel launched once per step, the
roofline fraction of the dominant kernel (HIP events on the launch stream),
and the FP64 oracle timed on the host cores over a bounded sample.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
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

import workloads as wl  # noqa: E402

METRIC = "env-steps/s @65536 envs (fused vs plain) + fwd+bwd steps/s; err vs FP64 oracle"

# Algorithmic work per env step of the forward path: actor MACs
# (146*64 + 64*64 + 64*4 = 13696, i.e. 27392 FLOP) plus ~1.1 kFLOP for
# observation, action map, four dynamics evaluations, RK4 combination,
# renormalisation and reward.
FLOP_PER_ENV_STEP = 28_500
# Algorithmic HBM bytes of one env step of the plain five-kernel path: the
# observation kernel reads p, q, v, w (52 B), head, counters and the ring
# (524 B) and writes the observation (584 B); the three dense layers read
# their inputs and write their outputs (584+256, 256+256, 256+16 B); the
# dynamics kernel reads parameters, state, action and counters (128 B) and
# writes a ring slot, counters, state, reward and done (97 B).
PLAIN_BYTES_PER_ENV_STEP = 1160 + 840 + 512 + 272 + 225
PEAK_FP32_MFMA = 157.3e12      # MI355X dense fp32 matrix FLOP/s
PEAK_BF16_MFMA = 2.5e15        # dense bf16 matrix FLOP/s
PEAK_FP32_VALU = 78.6e12       # fp32 vector FLOP/s without packed instructions
PEAK_FP64 = 78.6e12            # fp64 vector and matrix FLOP/s
PEAK_HBM = 8.0e12
ACTOR_GEMM_FLOP = 27_392      # the forward actor's three GEMMs, per env step
# Dynamics-only env step: four right-hand sides (about 103 FLOP each: rotor
# thrusts, force and torques, quaternion rate, acceleration, Euler, motor
# lag), the RK4 combinations (221), renormalisation (12), action map (8) and
# reward (35).
DYN_FLOP_PER_ENV_STEP = 700
# Algorithmic work per env step of forward + backward (no recompute counted):
# the forward (28.5 kFLOP), the actor's input VJP and weight gradient (27392
# FLOP each) and the dynamics VJP (about 2.4 kFLOP).  Of it, the actor's
# three GEMMs (3 x 27392) run on matrix cores; the rest is scalar fp32.
FLOP_FWD_BWD_ENV_STEP = 28_500 + 2 * 27_392 + 2_400
ACTOR_GEMM_FLOP_FWD_BWD = 3 * 27_392


TRAFFIC_PROFILES = {
    "k_fused<MFMA>": os.path.join(ROOT, "profiles", "k_fused_mfma_fwd65536_dr_hbm_traffic.md"),
    "k_fused4<MFMA>": os.path.join(ROOT, "profiles", "k_fused4_mfma_fwd65536_dr_hbm_traffic.md"),
}


def measured_traffic(kernel, n_envs, steps_per_launch):
    """HBM bytes per launch from the committed counter summary of `kernel`,
    or None when there is none, the kernel sources changed since the counters
    were taken, or the launch shape differs."""
    import hashlib
    path = TRAFFIC_PROFILES.get(kernel)
    if path is None or not os.path.exists(path):
        return None
    fields = {}
    for line in open(path).read().splitlines():
        line = line.strip()
        for key in ("traffic_bytes_per_launch", "launch_shape", "sources", "sources_sha256"):
            if line.startswith(key + ": "):
                fields[key] = line.split(": ", 1)[1]
    if not {"traffic_bytes_per_launch", "launch_shape", "sources", "sources_sha256"} <= set(fields):
        return None
    h = hashlib.sha256()
    for f in fields["sources"].split():
        with open(os.path.join(ROOT, "paper_2311_13081_amd", "csrc", os.path.basename(f)), "rb") as fh:
            h.update(fh.read())
    if fields["sources_sha256"] != h.hexdigest():
        return None
    if fields["launch_shape"] != f"{n_envs} envs x {steps_per_launch} steps":
        return None
    return float(fields["traffic_bytes_per_launch"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="fwd65536_dr")
    ap.add_argument("--plain-steps", type=int, default=100,
                    help="env steps per timed plain-path rollout")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the plain / per-step comparison legs")
    ap.add_argument("--cpu-seconds", type=float, default=25.0)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (3 times): the "
                         "reference for scaling HBM traffic counters")
    ap.add_argument("--only-fwd-bwd", action="store_true",
                    help="run only the forward+backward legs and print them (for profiling "
                         "the backward kernels)")
    ap.add_argument("--fwd-bwd-legs", default=None,
                    help="comma-separated forward+backward legs to run (default: all)")
    ap.add_argument("--variant", default="auto", choices=["auto", "mfma4", "mfma", "valu", "split"],
                    help="auto = run the autotuner; otherwise a fixed fused kernel, one launch "
                         "per rollout (used for profiling so only timed launches appear)")
    return ap.parse_args()


def time_rollouts(torch, sim, actor, T, K, W, record=False):
    """W warm-up rollouts, then K timed rollouts bracketed by synchronisation;
    HIP events on the launch stream give the device time.  record=True also
    writes the per-step rewards [T][N] and done flags [T][N] (buffers
    allocated before the timed region)."""
    out = sim.rollout(actor, T, rewards=record, dones=record) if record else None
    for _ in range(W):
        sim.rollout(actor, T, rewards=record, dones=record, out=out)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(K):
        sim.rollout(actor, T, rewards=record, dones=record, out=out)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dev_ms = ev0.elapsed_time(ev1)
    _, launches = sim.last_rollout_timing()
    return wall, dev_ms, launches


def cpu_baseline(cfg, W, seconds):
    """FP64 oracle on a bounded sample of the same workload (env ids spread
    over the batch), all host threads."""
    import oracle
    oracle.build(force=False)
    nthreads = min(os.cpu_count() or 1, 64)
    N = cfg["n_envs"]
    # rate probe large enough that thread start-up does not dominate it
    probe_ids = np.linspace(0, N - 1, min(N, nthreads * 32)).astype(np.uint32)
    b = oracle.Batch.init(cfg, len(probe_ids), ids=probe_ids)
    t0 = time.perf_counter()
    b.rollout(W, 40, nthreads=nthreads)
    rate = len(probe_ids) * 40 / max(time.perf_counter() - t0, 1e-6)
    n = int(max(nthreads, min(N, rate * seconds / 200)))
    steps = int(max(20, min(1000, rate * seconds / n)))
    ids = np.linspace(0, N - 1, n).astype(np.uint32)
    b = oracle.Batch.init(cfg, n, ids=ids)
    t0 = time.perf_counter()
    b.rollout(W, steps, nthreads=nthreads)
    dt = time.perf_counter() - t0
    # one thread, on a tenth of the time budget
    probe_ids = probe_ids[:64]
    n1 = len(probe_ids)
    steps1 = int(max(20, min(1000, n * steps / dt / nthreads * seconds / 10 / n1)))
    b1 = oracle.Batch.init(cfg, n1, ids=probe_ids)
    t1 = time.perf_counter()
    b1.rollout(W, steps1, nthreads=1)
    dt1 = time.perf_counter() - t1
    return {"value": n * steps / dt, "unit": "env-steps/s", "cores": nthreads, "kind": "oracle",
            "sample": f"{n} of {N} envs x {steps} steps (same config, seeds, env ids), "
                      f"{dt:.1f} s",
            "single_thread": {"value": n1 * steps1 / dt1,
                              "sample": f"{n1} envs x {steps1} steps, {dt1:.1f} s"}}


# Error norm per state component group (p, q, v, w, rotor speeds): the
# difference relative to the larger of the reference's magnitude and the
# group's floor (1 m, 1, 1 m/s, 1 rad/s, 1000 RPM).
_FLOORS = np.array([1.0] * 3 + [1.0] * 4 + [1.0] * 3 + [1.0] * 3 + [1000.0] * 4)


def oracle_step_error(torch, pkg, cfg, W, variant, warm_steps=250, n_sample=2048):
    """The headline kernel's one-step error against the FP64 oracle on a
    sample of envs of the headline batch, from the GPU's own state after
    `warm_steps` steps (a mix of episode ages, some just reset)."""
    import oracle
    N = cfg["n_envs"]
    sim = pkg.QuadSim(cfg)
    sim.set_variant(*variant)
    a = sim.actor_tensor(W)
    sim.rollout(a, warm_steps, rewards=False, dones=False)
    st = {k: v.cpu().numpy() for k, v in sim.get_state().items()}
    th = sim.get_params().cpu().numpy()
    r, d = sim.step(actor=a)
    s1 = sim.get_state()["state"].cpu().numpy()
    r = r.cpu().numpy()
    d = d.cpu().numpy()
    sim.close()
    ids = np.linspace(0, N - 1, n_sample).astype(np.uint32)
    ref = oracle.Batch(cfg, n_sample, ids=ids)
    ref.set_soa(st["state"][:, ids], st["hist"][:, :, ids], t_ep=st["t_ep"][ids],
                ep=st["episode"][ids], theta_soa=th[:, ids])
    out = ref.rollout(W, 1, nthreads=min(os.cpu_count() or 1, 64))
    same = d[ids] == out["dones"][0]
    err = np.abs(s1[:, ids].T - ref.s) / np.maximum(np.abs(ref.s), _FLOORS)
    rerr = np.abs(r[ids] - out["rewards"][0]) / np.maximum(np.abs(out["rewards"][0]), 1.0)
    return {"one_step_state_max": float(err[same].max()), "one_step_reward_max":
            float(rerr[same].max()), "done_flags_equal": int(same.sum()), "envs": n_sample,
            "after_steps": warm_steps, "bar": 1e-5}


def _traj_err(S_gpu, S_ref):
    """Worst R16 error over envs and components at every step; S_gpu
    [T+1][17][n] (GPU layout), S_ref [T+1][n][17] (oracle layout)."""
    g = np.swapaxes(np.asarray(S_gpu, np.float64), 1, 2)
    e = np.abs(g - S_ref) / np.maximum(np.abs(S_ref), _FLOORS)
    return np.where(np.isnan(e), np.inf, e).max(axis=(1, 2))


def oracle_trajectory_error(torch, pkg, W, variant, T=64, trials=8):
    """The 64-step trajectory figures of the 64-env forward workload (nominal
    body, seeded Xavier policy, no termination): the worst error over steps
    0..T against the FP64 oracle of the headline kernel and of the FP64 path,
    beside the FP64 oracle's own envelope (its trajectory from start states
    perturbed by one float32 rounding, worst of `trials` draws)."""
    import oracle
    cfg = wl.workload_config("fwd64")
    n = cfg["n_envs"]
    ref = oracle.Batch.init(cfg, n)
    base = ref.copy().rollout(W, T, record=True)["states"]
    rng = np.random.default_rng(0)
    env = np.zeros(T + 1)
    for _ in range(trials):
        b = ref.copy()
        b.s = b.s * (1 + 2.0 ** -24 * rng.choice([-1.0, 1.0], size=b.s.shape))
        env = np.maximum(env, _traj_err(np.swapaxes(b.rollout(W, T, record=True)["states"], 1, 2),
                                        base))
    out = {}
    for label, flags in (("fp32_headline_kernel", 0), ("fp64_path", wl.F_FP64)):
        c = dict(cfg)
        c["flags"] = cfg["flags"] | flags
        sim = pkg.QuadSim(c)
        if not flags:
            sim.set_variant(*variant)
        S = sim.rollout(sim.actor_tensor(W), T, rewards=False, dones=False,
                        states=True)["states"].cpu().numpy()
        sim.close()
        out[label] = _traj_err(S, base)
    e32, e64 = out["fp32_headline_kernel"], out["fp64_path"]
    return {"workload": f"fwd64: {n} nominal envs, seeded Xavier policy, {T} steps",
            "bar": 1e-4,
            "fp32_headline_kernel_max": float(e32.max()),
            "fp32_headline_kernel_step1": float(e32[1]),
            "fp64_oracle_envelope_max": float(env.max()),
            "fp32_over_envelope": float(e32.max() / env.max()),
            "fp64_path_max": float(e64.max()),
            "fp32_meets_bar": bool(e32.max() < 1e-4),
            "fp64_path_meets_bar": bool(e64.max() < 1e-4)}


def fwd_bwd(torch, pkg, name, K, W, warmup=1, bf16=False):
    """Forward rollout with tape + discrete adjoint on a differentiable
    workload; returns env-steps/s of the pair (N x H per fwd+bwd).  bf16:
    the actor on bf16 matrix cores (SIM_F_ACTOR_BF16)."""
    cfg = wl.workload_config(name)
    cfg["ckpt_every"] = K
    if bf16:
        cfg["flags"] |= wl.F_ACTOR_BF16
    H = wl.workload_steps(name)
    N = cfg["n_envs"]
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    sim = pkg.QuadSim(cfg)
    torch.cuda.synchronize()
    handle_bytes = free0 - torch.cuda.mem_get_info()[0]
    sim.set_variant(pkg.SIM_V_FUSED_MFMA4)   # the kernel taped rollouts use
    a = sim.actor_tensor(W)
    snap = {k: v.clone() for k, v in sim.get_state().items()}
    if name.startswith("sysid"):
        # ground truth with the randomised parameters theta*, then a perturbed
        # body theta* (1 + delta), delta ~ U(-0.1, 0.1) (seed 3); loss = MSE
        # over position, attitude, velocity and angular velocity
        theta_star = sim.get_params().clone()
        truth = sim.rollout(a, H, rewards=False, dones=False, states=True)["states"].clone()
        g = torch.Generator(device="cpu").manual_seed(3)
        delta = (torch.rand(theta_star.shape, generator=g) * 0.2 - 0.1).to(theta_star.device)
        theta = theta_star * (1 + delta)
    else:
        truth = None
        theta = sim.get_params().clone()

    # the loss's cotangent d MSE / dS = 2 (S - truth) / count on the first 13
    # state components: the backward is linear in its cotangents, so it gets
    # S - truth (one pass into a buffer whose rotor rows stay zero) and the
    # two small gradients are scaled afterwards
    dS = torch.zeros((H + 1, 17, N), dtype=torch.float32, device="cuda") if truth is not None else None
    dR0 = torch.zeros((H, N), dtype=torch.float32, device="cuda") if truth is not None else None
    scale = 2.0 / ((H + 1) * 13 * N)

    def one():
        sim.set_state(**snap)
        S, R = pkg.rollout(sim, a, theta, H)
        if truth is not None:
            torch.sub(S[:, :13], truth[:, :13], out=dS[:, :13])
            ga, gp = sim.backward(a, d_rewards=dR0, d_states=dS)
            ga.mul_(scale)
            gp.mul_(scale)
        else:
            ga, gp = sim.backward(a)
        return ga, gp

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        one()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    sim.close()
    rate = N * H / dt
    if bf16:
        # actor GEMMs on bf16 matrix cores, the scalar rest on fp32 vector ALUs
        t_roof = (ACTOR_GEMM_FLOP_FWD_BWD / PEAK_BF16_MFMA
                  + (FLOP_FWD_BWD_ENV_STEP - ACTOR_GEMM_FLOP_FWD_BWD) / PEAK_FP32_VALU)
        roof = {"bound": "bf16 mfma + fp32 valu", "roof_env_steps_per_s": 1.0 / t_roof,
                "frac": rate * t_roof}
    else:
        ach = rate * FLOP_FWD_BWD_ENV_STEP / 1e12
        roof = {"bound": "mfma", "achieved": ach, "peak": PEAK_FP32_MFMA / 1e12,
                "unit": "TFLOP/s", "frac": ach * 1e12 / PEAK_FP32_MFMA}
    roof["flop_per_env_step"] = FLOP_FWD_BWD_ENV_STEP
    K = cfg["ckpt_every"]
    # checkpoints of (state, history, counters): 147 floats per env; the
    # backward's record: 171 floats per env and step (x, a, both layers'
    # pre-activations, the 18 observed state features, 4 ReLU mask words)
    # plus the action tape: the 128-float history at the start of the
    # recorded span and 4 floats per step
    mem = {"device_bytes_of_handle": handle_bytes,
           "tape_bytes": (H // K + 1) * 147 * N * 4,
           "records_of_whole_horizon_bytes": (H * (171 + 4) + 128) * N * 4}
    return {"env_steps_per_s": rate, "ms_per_fwd_bwd": dt * 1e3, "n_envs": N,
            "horizon": H, "ckpt_every": K, "actor": "bf16" if bf16 else "f32",
            "roofline": roof, "memory": mem}


def fwd_bwd_legs(torch, pkg, W, only=None):
    """The differentiable workloads: the policy gradient on 1024 nominal envs
    over 64 steps, the same on 65536 randomised envs (the hover-biased
    policy, which keeps every body's rates bounded over the horizon),
    and system identification on 16384 randomised envs over 256 steps (fp32
    and bf16 actor), checkpoints every 16 steps.  grad65536_dr_rec64 is the
    65536-env policy gradient with one 64-step segment: the taped forward
    records the whole horizon (3 GB in HBM) and the backward recomputes
    nothing.  only: names of the legs to run (all when None)."""
    legs = {"grad1024": ("grad1024", 16, W, False),
            "grad65536_dr": ("grad65536_dr", 16, wl.sysid_actor(0), False),
            "grad65536_dr_rec64": ("grad65536_dr", 64, wl.sysid_actor(0), False),
            "sysid16384": ("sysid16384", 16, wl.sysid_actor(0), False),
            "sysid16384_bf16": ("sysid16384", 16, wl.sysid_actor(0), True)}
    return {k: fwd_bwd(torch, pkg, name, K, actor, bf16=bf16)
            for k, (name, K, actor, bf16) in legs.items() if only is None or k in only}


def fixed_episodes(torch, pkg, actor):
    """4096 nominal envs x 1000 steps with every episode truncated at 500
    steps: the plain five-kernel step launched from the host, the same
    graph-captured, the fused kernel launched once per step, and the
    persistent fused kernel (autotuned, graph-replayed)."""
    cfg = wl.workload_config("fwd4096")
    T = wl.workload_steps("fwd4096")
    N = cfg["n_envs"]
    res = {"n_envs": N, "rollout_steps": T}
    names = {1: "plain", 2: "fused_valu", 3: "fused_mfma", 4: "fused_mfma4", 5: "fused_split"}
    for label, variant, spl, use_graph in (
            ("plain_eager", pkg.SIM_V_PLAIN, 0, False), ("plain_graph", pkg.SIM_V_PLAIN, 0, True),
            ("fused_per_step_launch", pkg.SIM_V_FUSED_MFMA, 1, True),
            ("fused_per_step_launch", pkg.SIM_V_FUSED_MFMA4, 1, True),
            ("fused_per_step_launch", pkg.SIM_V_FUSED_SPLIT, 1, True),
            ("persistent", None, 0, True)):
        sim = pkg.QuadSim(cfg)
        if variant is None:
            sim.autotune(actor, T)
        else:
            sim.set_variant(variant, spl, use_graph)
        w, _, _ = time_rollouts(torch, sim, actor, T, 2, 1)
        v, s, g = sim.get_variant()
        r = {"env_steps_per_s": N * T * 2 / w, "ms_per_env_step": w * 1e3 / (2 * T),
             "variant": names[v], "steps_per_launch": s}
        sim.close()
        # the per-step launch leg keeps the fastest fused kernel
        if label not in res or r["env_steps_per_s"] > res[label]["env_steps_per_s"]:
            res[label] = r
    return res


def dynamics_only(torch, pkg, n_envs, T, reps=3):
    """Dynamics-only rollouts (no actor): a constant action per env, the
    nominal body's hover command (the reward's action baseline), over T steps
    with randomised bodies, termination and reset; rewards and dones written
    each step."""
    cfg = wl.workload_config("fwd65536_dr")
    cfg["n_envs"] = n_envs
    sim = pkg.QuadSim(cfg)
    a = torch.full((4, n_envs), cfg["C_rab"], dtype=torch.float32, device="cuda")
    sim.rollout_actions(a, T)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        sim.rollout_actions(a, T)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    kernel_ms, _ = sim.last_rollout_timing()
    sim.close()
    rate = n_envs * T / (kernel_ms * 1e-3)
    return {"env_steps_per_s": n_envs * T / dt, "n_envs": n_envs, "rollout_steps": T,
            "ms_per_rollout": dt * 1e3, "kernel_ms": kernel_ms,
            "roofline": {"bound": "valu", "achieved": rate * DYN_FLOP_PER_ENV_STEP / 1e12,
                         "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s",
                         "frac": rate * DYN_FLOP_PER_ENV_STEP / PEAK_FP32_VALU,
                         "waves": (n_envs + 63) // 64, "simds": 1024}}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the environment batch is one GPU's share and "
              "the library has no multi-GPU path; run it with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2311_13081_amd as pkg

    name = args.workload
    cfg = wl.workload_config(name)
    T = wl.workload_steps(name)
    N = cfg["n_envs"]
    W = wl.xavier_actor(0)
    if args.copy_probe_mib:
        n = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.only_fwd_bwd:
        only = args.fwd_bwd_legs.split(",") if args.fwd_bwd_legs else None
        print(json.dumps({"fwd_bwd": fwd_bwd_legs(torch, pkg, W, only)}), flush=True)
        return
    sim = pkg.QuadSim(cfg)
    actor = sim.actor_tensor(W)
    if args.variant == "auto":
        sim.autotune(actor, T)
    else:
        sim.set_variant({"mfma4": pkg.SIM_V_FUSED_MFMA4, "mfma": pkg.SIM_V_FUSED_MFMA,
                         "valu": pkg.SIM_V_FUSED_VALU, "split": pkg.SIM_V_FUSED_SPLIT}[args.variant],
                        0, True)
    v, spl, graph = sim.get_variant()
    wall, dev_ms, launches = time_rollouts(torch, sim, actor, T, args.steps, args.warmup)
    env_steps = N * T * args.steps
    value = env_steps / wall
    ms_per_step = wall * 1e3 / args.steps
    kernel_ms = dev_ms / (args.steps * launches)
    flop_per_launch = FLOP_PER_ENV_STEP * N * (T / launches)
    achieved = flop_per_launch / (kernel_ms * 1e-3)
    vname = {1: "plain", 2: "fused_valu", 3: "fused_mfma", 4: "fused_mfma4", 5: "fused_split"}[v]
    kname = {1: "plain (5 kernels)", 2: "k_fused<VALU>", 3: "k_fused<MFMA>",
             4: "k_fused4<MFMA>", 5: "k_split<MFMA>"}[v]
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "env-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": name, "n_envs": N, "rollout_steps": T, "dr": bool(cfg["dr_enable"]),
                   "terminate_autoreset": True, "variant": vname, "steps_per_launch": spl,
                   # a graph is captured and replayed only for multi-launch rollouts
                   "hipgraph": bool(graph) and launches > 1,
                   "launch": ("hipGraph replay of %d launches" % launches if graph and launches > 1
                              else "%d launch(es) from the host" % launches),
                   "launches_per_step": launches},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_FP32_MFMA / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_MFMA,
                     "traffic": measured_traffic(kname, N, T // launches),
                     "kernel": kname,
                     "kernel_ms": kernel_ms, "flop_per_env_step": FLOP_PER_ENV_STEP},
    }
    if not args.no_extras:
        extras = {}
        # plain five-kernel step, graph-captured and eager, on the same batch
        for label, use_graph in (("plain_graph", True), ("plain_eager", False)):
            s2 = pkg.QuadSim(cfg)
            s2.set_variant(pkg.SIM_V_PLAIN, 0, use_graph)
            w2, d2, _ = time_rollouts(torch, s2, actor, args.plain_steps, 2, 1)
            rate = N * args.plain_steps * 2 / w2
            gbs = rate * PLAIN_BYTES_PER_ENV_STEP / 1e9
            extras[label] = {"env_steps_per_s": rate,
                             "ms_per_env_step": w2 * 1e3 / (2 * args.plain_steps),
                             "roofline": {"bound": "hbm", "achieved": gbs,
                                          "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                                          "frac": gbs * 1e9 / PEAK_HBM,
                                          "bytes_per_env_step": PLAIN_BYTES_PER_ENV_STEP}}
            s2.close()
        # fused kernel launched once per env step
        s3 = pkg.QuadSim(cfg)
        s3.set_variant(pkg.SIM_V_FUSED_MFMA, 1, True)
        w3, _, _ = time_rollouts(torch, s3, actor, args.plain_steps, 2, 1)
        extras["fused_per_step_launch"] = {"env_steps_per_s": N * args.plain_steps * 2 / w3,
                                           "ms_per_env_step": w3 * 1e3 / (2 * args.plain_steps)}
        s3.close()
        extras["fused_vs_plain_speedup"] = value / extras["plain_graph"]["env_steps_per_s"]
        # against the best any unfused path with these intermediates could do:
        # the plain step's algorithmic bytes moved at the HBM peak
        extras["fused_vs_plain_hbm_roof"] = value / (PEAK_HBM / PLAIN_BYTES_PER_ENV_STEP)
        # the same kernel as a hipGraph-captured rollout of 100-step launches
        # (ten kernel nodes replayed per rollout)
        sim.set_variant(v, 100, True)
        wg, dg, lg = time_rollouts(torch, sim, actor, T, 2, 1)
        extras["headline_graph_100_steps_per_launch"] = {
            "env_steps_per_s": N * T * 2 / wg, "kernel_ms": dg / (2 * lg),
            "launches_per_rollout": lg, "hipgraph": lg > 1}
        # the headline kernel and shape with per-step rewards and done flags
        # written to HBM (5 B per env step)
        sim.set_variant(v, spl, graph)
        w4, d4, l4 = time_rollouts(torch, sim, actor, T, 2, 1, record=True)
        extras["headline_recorded"] = {"env_steps_per_s": N * T * 2 / w4,
                                       "kernel_ms": d4 / (2 * l4)}
        # the same workload with the bf16 actor option (a precision trade,
        # not the headline arithmetic)
        cfg_b = dict(cfg)
        cfg_b["flags"] = cfg["flags"] | wl.F_ACTOR_BF16
        s5 = pkg.QuadSim(cfg_b)
        s5.autotune(actor, T)
        w5, d5, l5 = time_rollouts(torch, s5, actor, T, 2, 1)
        t_roof = ACTOR_GEMM_FLOP / PEAK_BF16_MFMA + (FLOP_PER_ENV_STEP - ACTOR_GEMM_FLOP) / PEAK_FP32_VALU
        extras["headline_bf16_actor"] = {
            "env_steps_per_s": N * T * 2 / w5, "kernel_ms": d5 / (2 * l5),
            "roofline": {"bound": "bf16 mfma + fp32 valu", "roof_env_steps_per_s": 1.0 / t_roof,
                         "frac": N * T * 2 / w5 * t_roof}}
        s5.close()
        # the headline workload with the training extras (per-episode
        # disturbance and actor observation noise), and the FP64 path
        for label, flags, steps in (("headline_training_extras", wl.F_DISTURB | wl.F_OBS_NOISE, T),
                                    ("headline_fp64_100_steps", wl.F_FP64, 100)):
            cfg_x = wl.training_extras(cfg) if flags != wl.F_FP64 else dict(cfg)
            cfg_x["flags"] = cfg["flags"] | flags
            s6 = pkg.QuadSim(cfg_x)
            if flags != wl.F_FP64:
                s6.set_variant(v, spl, graph)
            w6, d6, l6 = time_rollouts(torch, s6, actor, steps, 2, 1)
            extras[label] = {"env_steps_per_s": N * steps * 2 / w6, "kernel_ms": d6 / (2 * l6),
                             "rollout_steps": steps}
            if flags == wl.F_FP64:
                ach = FLOP_PER_ENV_STEP * N * steps / (d6 / (2 * l6) * 1e-3)
                extras[label]["roofline"] = {
                    "bound": "fp64 mfma", "achieved": ach / 1e12, "peak": PEAK_FP64 / 1e12,
                    "unit": "TFLOP/s", "frac": ach / PEAK_FP64}
            s6.close()
        res["comparison"] = extras
        res["fixed_episodes_4096"] = fixed_episodes(torch, pkg, actor)
    sim.close()
    if not args.no_extras:
        res["fwd_bwd"] = fwd_bwd_legs(torch, pkg, W)
        res["dynamics_only"] = {"n8192_T2000": dynamics_only(torch, pkg, 8192, 2000),
                                "n65536_T1000": dynamics_only(torch, pkg, 65536, 1000)}
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(cfg, W, args.cpu_seconds)
        res["err_vs_oracle"] = oracle_step_error(torch, pkg, cfg, W, (v, spl, graph))
        res["err_vs_oracle"]["trajectory_64"] = oracle_trajectory_error(torch, pkg, W,
                                                                        (v, spl, graph))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
