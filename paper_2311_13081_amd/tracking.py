"""Trajectory tracking in simulation with a trained position controller, by the
set-point shift of Sec. IV: the policy observes its position and velocity
relative to a moving set point (clipped to the errors seen in training) and
so follows it, as in the tracking experiment of Sec. VI, which flies the
figure-eight Lissajous curve p(t) = (cos(2 pi t / T), sin(4 pi t / T) / 2,
const) with cycle times T of 15, 5.5 and 3.5 s (Table III, real flights).

Every step runs in the library: the set point is handed over with
sim_set_target and the policy evaluated inside the fused step kernel.
"""
from __future__ import annotations

import math

import torch

from .sim import QuadSim


def lissajous(t: float, period: float, z: float = 0.0):
    """Set point (position, velocity) of the figure eight at time t."""
    w = 2.0 * math.pi / period
    p = (math.cos(w * t), 0.5 * math.sin(2.0 * w * t), z)
    v = (-w * math.sin(w * t), w * math.cos(2.0 * w * t), 0.0)
    return p, v


def track(sim: QuadSim, flat: torch.Tensor, period: float, cycles: int = 2,
          pos_clip: float = 0.2, vel_clip: float = 1.0):
    """Flies `cycles` cycles of the figure eight with every env of `sim`
    (started at rest at the curve's start point, level, rotors at the hover
    speed) and returns per-env RMS position errors over the last cycle: (e
    over x, y, z; e_xy), tensors [N].  The handle's termination and reset
    flags should be off (the curve leaves the training box)."""
    dev = sim.device
    N = sim.N
    dt = float(sim.cfg["dt"])
    st = sim.get_state()
    s = st["state"].clone()
    p0, _ = lissajous(0.0, period)
    s[0:3] = torch.tensor(p0, device=dev).unsqueeze(1)
    s[3] = 1.0
    s[4:13] = 0.0
    th = sim.get_params()
    # hover speed of each body: c2 w^2 + c1 w + c0 = m g / 4
    need = th[0] * float(sim.cfg["g"]) / 4 - th[4]
    wh = 2 * need / (th[5] + torch.sqrt(th[5] ** 2 + 4 * th[6] * need))
    s[13:17] = wh.unsqueeze(0)
    ah = 2 * (wh - float(sim.cfg["rpm_min"])) / (float(sim.cfg["rpm_max"]) -
                                                float(sim.cfg["rpm_min"])) - 1
    hist = ah.reshape(1, 1, N).expand(32, 4, N).contiguous()
    sim.set_state(state=s, hist=hist, t_ep=torch.zeros(N, dtype=torch.int32, device=dev))
    steps = int(round(cycles * period / dt))
    last = int(round(period / dt))
    err2 = torch.zeros(N, device=dev)
    err2_xy = torch.zeros(N, device=dev)
    tgt = torch.empty(6, N, device=dev)
    for k in range(steps):
        p_sp, v_sp = lissajous(k * dt, period)
        tgt[0:3] = torch.tensor(p_sp, device=dev).unsqueeze(1)
        tgt[3:6] = torch.tensor(v_sp, device=dev).unsqueeze(1)
        sim.set_target(tgt, pos_clip, vel_clip)
        sim.step(actor=flat)
        if k >= steps - last:
            p_ref, _ = lissajous((k + 1) * dt, period)
            p = sim.get_state(parts=("state",))["state"][0:3]
            d = p - torch.tensor(p_ref, device=dev).unsqueeze(1)
            err2 += (d ** 2).sum(0)
            err2_xy += (d[0:2] ** 2).sum(0)
    sim.set_target(None)
    return torch.sqrt(err2 / last), torch.sqrt(err2_xy / last)


def tracking_table(flat: torch.Tensor, env_cfg: dict, n_envs: int = 64,
                   periods=(15.0, 5.5, 3.5), cycles: int = 2, pos_clip: float = 0.2,
                   vel_clip: float = 1.0):
    """The sim analogue of Table III: for each cycle time the mean, median and
    minimum over envs (different disturbance and noise draws) of the RMS
    tracking error e and e_xy over the last cycle, and the fraction of envs
    whose error stays finite and below 1 m."""
    import workloads as wl
    cfg = dict(env_cfg, n_envs=n_envs, max_episode_steps=0)
    cfg["flags"] = int(cfg["flags"]) & ~(wl.F_TERMINATE | wl.F_AUTORESET)
    rows = {}
    for T in periods:
        sim = QuadSim(cfg)
        e, exy = track(sim, flat, T, cycles, pos_clip, vel_clip)
        sim.close()
        ok = torch.isfinite(e) & (e < 1.0)
        ef = torch.where(ok, e, torch.full_like(e, float("inf")))
        exyf = torch.where(ok, exy, torch.full_like(exy, float("inf")))
        rows[f"{T:g}s"] = dict(
            e_mean=float(ef[ok].mean()) if ok.any() else float("inf"),
            e_median=float(ef.median()), e_min=float(ef.min()),
            e_xy_mean=float(exyf[ok].mean()) if ok.any() else float("inf"),
            e_xy_median=float(exyf.median()), ok_frac=float(ok.float().mean()))
    return rows
