"""Seeded synthetic inputs shared by the oracle checks, the GPU tests and the
benchmark.

This module holds no arithmetic of the simulated method: it only fixes
constants, draws actor weights and draws synthetic states.  Both the FP64
oracle (``oracle/``) and the GPU library (``paper_2311_13081_amd``) receive
what is built here; neither imports the other.

Body and workloads follow "Learning to Fly in Seconds" (Eschmann, Albani,
Loianno): a 27 g Crazyflie-class quadrotor with a 0.15 s motor time constant
(Sec. IV), 100 Hz simulation (Sec. V, Simulation), action history of 32 steps
so the actor sees 18 + 4*32 = 146 inputs (Sec. IV).  The paper's parameter
sheet is not part of the paper; every constant it would supply is a stated
reading below (thrust curve, yaw moment, RPM range, reward constants, reset
ranges).
"""
from __future__ import annotations

import math

import numpy as np

NSTATE = 17
NHIST = 32
NACT = 4
NOBS = 18 + 4 * NHIST
NHID = 64
NPARAM = 8
NACTOR = NHID * NOBS + NHID + NHID * NHID + NHID + NACT * NHID + NACT  # 13828

F_TERMINATE = 1
F_AUTORESET = 2
F_RENORM_Q = 4
F_FP64 = 8
F_ACTOR_BF16 = 16
F_DISTURB = 32
F_OBS_NOISE = 64

PARAM_NAMES = ("m", "Jxx", "Jyy", "Jzz", "c0", "c1", "c2", "Tm")

# Reward action offset C_rab: the normalised hover action of the nominal body,
# rounded (rotors near 14475.8 RPM out of 0..21702 RPM, c2 = 3.16e-10 N/RPM^2
# carrying 0.027 kg * 9.81 m/s^2).
HOVER_ACTION_NOMINAL = 0.334053


def crazyflie_config(**overrides) -> dict:
    """Nominal body, limits, reset ranges and reward constants.

    Parameter order: m, Jxx, Jyy, Jzz, c0, c1, c2, Tm (thrust T = c0 + c1 w +
    c2 w^2 with w in RPM, T_m the motor time constant).
    """
    cfg = dict(
        dt=0.01,
        g=9.81,
        arm=0.028,           # per-axis rotor offset [m]
        k_m=6.0e-3,          # yaw moment per newton of rotor thrust [m]
        rpm_min=0.0,
        rpm_max=21702.0,
        nominal=[0.027, 3.85e-6, 3.85e-6, 5.9675e-6, 0.0, 0.0, 3.16e-10, 0.15],
        dr_lo=[0.8, 0.8, 0.8, 0.8, 0.8, 0.8, 0.8, 0.5],
        dr_hi=[1.2, 1.2, 1.2, 1.2, 1.2, 1.2, 1.2, 1.5],
        pos_limit=0.6,
        vel_limit=2.0,
        init_pos=0.2,
        init_angle=math.pi / 2,
        init_vel=1.0,
        init_angvel=1.0,
        C_rp=1.0,
        C_rq=1.0,
        C_rv=0.1,
        C_rw=0.01,
        C_ra=0.01,
        C_rab=HOVER_ACTION_NOMINAL,
        C_rs=1.0,
        max_episode_steps=500,
        flags=F_RENORM_Q,
        dr_enable=0,
        seed=1,
        dr_seed=2,
        n_envs=64,
        max_tape_horizon=0,
        ckpt_every=16,
        # training extras (active only under F_DISTURB / F_OBS_NOISE)
        dist_force=0.0,
        dist_torque=0.0,
        obs_noise=(0.0, 0.0, 0.0, 0.0),
    )
    for k, v in overrides.items():
        if k not in cfg:
            raise KeyError(f"unknown config key {k!r}")
        cfg[k] = v
    return cfg


def training_extras(cfg: dict) -> dict:
    """The training MDP of the paper's asymmetric actor-critic setup on top of
    cfg: per-episode force/torque disturbances and actor observation noise.
    The paper's magnitudes are in its missing parameter sheet; these readings
    are small next to the vehicle's own authority: a force bound of 5 % of the
    nominal weight per axis (0.0132 N), a torque bound of 1 % of the maximal
    roll torque arm * T_max (4.2e-5 N m), and noise std 1 mm, 0.01 (rotation
    entries), 2 cm/s and 0.05 rad/s."""
    out = dict(cfg)
    m = cfg["nominal"][0]
    t_max = cfg["nominal"][6] * cfg["rpm_max"] ** 2
    out["flags"] = cfg["flags"] | F_DISTURB | F_OBS_NOISE
    out["dist_force"] = 0.05 * m * cfg["g"]
    out["dist_torque"] = 0.01 * cfg["arm"] * t_max
    out["obs_noise"] = (0.001, 0.01, 0.02, 0.05)
    return out


# The workloads: a small parity case, the plain-vs-fused comparison, the large
# randomised batch, the differentiable rollout, the system-ID rollout, and the
# policy gradient at the large batch's size (65536 randomised envs).
WORKLOADS = {
    "fwd64": dict(n_envs=64, steps=500, flags=F_RENORM_Q, dr_enable=0, max_episode_steps=500),
    "fwd4096": dict(n_envs=4096, steps=1000, flags=F_RENORM_Q | F_AUTORESET, dr_enable=0,
                    max_episode_steps=500),
    "fwd65536_dr": dict(n_envs=65536, steps=1000,
                        flags=F_RENORM_Q | F_TERMINATE | F_AUTORESET, dr_enable=1,
                        max_episode_steps=500),
    "grad1024": dict(n_envs=1024, steps=64, flags=F_RENORM_Q, dr_enable=0, max_episode_steps=0),
    "sysid16384": dict(n_envs=16384, steps=256, flags=F_RENORM_Q, dr_enable=1,
                       max_episode_steps=0, ckpt_every=16),
    "grad65536_dr": dict(n_envs=65536, steps=64, flags=F_RENORM_Q, dr_enable=1,
                         max_episode_steps=0, ckpt_every=16),
}

# workloads whose rollouts are differentiated (a tape of the whole horizon)
DIFFERENTIABLE = ("grad1024", "sysid16384", "grad65536_dr")


def workload_config(name: str, **overrides) -> dict:
    w = dict(WORKLOADS[name])
    steps = w.pop("steps")
    w.update(overrides)
    cfg = crazyflie_config(**w)
    if name in DIFFERENTIABLE and "max_tape_horizon" not in overrides:
        cfg["max_tape_horizon"] = steps
    return cfg


def workload_steps(name: str) -> int:
    return WORKLOADS[name]["steps"]


def xavier_actor(seed: int = 0) -> np.ndarray:
    """Flat float32 actor parameters [W1 | b1 | W2 | b2 | W3 | b3] with
    torch.nn.Linear layouts ([out][in] weights).  Xavier-uniform weights with
    bound sqrt(6 / (fan_in + fan_out)), zero biases, numpy PCG64 seed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for fan_out, fan_in in ((NHID, NOBS), (NHID, NHID), (NACT, NHID)):
        bound = math.sqrt(6.0 / (fan_in + fan_out))
        parts.append(rng.uniform(-bound, bound, size=fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    w = np.concatenate(parts).astype(np.float32)
    assert w.size == NACTOR
    return w


def sysid_actor(seed: int = 0, scale: float = 0.1) -> np.ndarray:
    """Policy of the system-identification workload: the Xavier draw of
    xavier_actor(seed) scaled by `scale`, with the output bias set so a zero
    hidden state commands the nominal hover action (atanh(C_rab)).  The
    unscaled Xavier policy spins a third of the bodies past the stability
    limit of RK4 at dt = 0.01 s within 256 steps (their states overflow);
    this one keeps 256-step rollouts finite while still feeding the state
    back through all three layers."""
    w = xavier_actor(seed).astype(np.float64)
    n_w = NACTOR - NACT
    w[:n_w] *= scale
    w[n_w:] = math.atanh(HOVER_ACTION_NOMINAL)
    return w.astype(np.float32)


def random_actor(seed: int, scale: float = 1.0) -> np.ndarray:
    """Xavier weights with non-zero biases (so bias paths are exercised)."""
    w = xavier_actor(seed).astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    n1 = NHID * NOBS
    n2 = NHID * NHID
    n3 = NACT * NHID
    o = 0
    for n_w, n_b in ((n1, NHID), (n2, NHID), (n3, NACT)):
        o += n_w
        w[o:o + n_b] = rng.uniform(-0.1, 0.1, size=n_b)
        o += n_b
    return (w * scale).astype(np.float32)


def random_states(n: int, seed: int, rpm_max: float = 21702.0):
    """Synthetic float32 states inside the training envelope, SoA [17][n], and
    histories [32][4][n] in (-1, 1).  Quaternions are random unit vectors
    (rounded to float32); rotor speeds span the RPM range."""
    rng = np.random.Generator(np.random.PCG64(seed))
    s = np.empty((NSTATE, n), np.float64)
    s[0:3] = rng.uniform(-0.6, 0.6, size=(3, n))
    q = rng.normal(size=(4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    q[:, q[0] < 0] *= -1.0
    s[3:7] = q
    s[7:10] = rng.uniform(-2.0, 2.0, size=(3, n))
    s[10:13] = rng.uniform(-8.0, 8.0, size=(3, n))
    s[13:17] = rng.uniform(0.1 * rpm_max, 0.95 * rpm_max, size=(4, n))
    h = rng.uniform(-1.0, 1.0, size=(NHIST, NACT, n))
    return s.astype(np.float32), h.astype(np.float32)


def random_actions(n: int, seed: int) -> np.ndarray:
    """Normalised actions [4][n] in (-1, 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-1.0, 1.0, size=(NACT, n)).astype(np.float32)
