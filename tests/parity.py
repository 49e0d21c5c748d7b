"""Error norms used by the GPU-vs-oracle parity tests.

Per-step norm: e = max over envs and components of |gpu - ref| / max(|ref|,
floor), floors per group (1 m, 1, 1 m/s, 1 rad/s, 1000 RPM): a relative error
for large values and an absolute one near zero.  Reward: |dr| / max(|r|, 1).
"""
import numpy as np

FLOOR = np.array([1.0] * 3 + [1.0] * 4 + [1.0] * 3 + [1.0] * 3 + [1000.0] * 4)

STEP_TOL = 1e-5        # one step from identical inputs
TRAJ_TOL = 1e-4        # 64-step closed-loop trajectory


def state_err(gpu_soa, ref_aos):
    """gpu: [17][n] (or [..., 17, n]); ref: [n][17] (or [..., n, 17])."""
    g = np.asarray(gpu_soa, np.float64)
    r = np.asarray(ref_aos, np.float64)
    g = np.swapaxes(g, -1, -2)
    e = np.abs(g - r) / np.maximum(np.abs(r), FLOOR)
    e = np.where(np.isnan(e), np.inf, e)
    return e


def max_state_err(gpu_soa, ref_aos):
    return float(state_err(gpu_soa, ref_aos).max())


def reward_err(gpu, ref):
    g = np.asarray(gpu, np.float64)
    r = np.asarray(ref, np.float64)
    return float((np.abs(g - r) / np.maximum(np.abs(r), 1.0)).max())


def box_margin(s_aos, pos_limit, vel_limit):
    """Smallest relative distance of any box coordinate to its threshold."""
    s = np.asarray(s_aos, np.float64)
    mp = np.abs(np.abs(s[..., 0:3]) - pos_limit) / pos_limit
    mv = np.abs(np.abs(s[..., 7:10]) - vel_limit) / vel_limit
    return np.minimum(mp.min(-1), mv.min(-1))


def oracle_envelope(orc, cfg, W, T, n, ids=None, trials=8, seed=0):
    """Sensitivity of the closed loop itself: the FP64 oracle run from its own
    start states perturbed by one float32 rounding (each component times
    1 +- 2^-24, random signs), against the unperturbed FP64 run.  Returns the
    worst error over trials at every t (shape [T+1]).  No float32 path can
    beat this envelope by much, since rounding the start state to float32 is
    already such a perturbation."""
    ref = orc.Batch.init(cfg, n, ids=ids)
    base = ref.copy().rollout(W, T, record=True)["states"]
    rng = np.random.default_rng(seed)
    env = np.zeros(T + 1)
    for _ in range(trials):
        b = ref.copy()
        b.s = b.s * (1 + 2.0 ** -24 * rng.choice([-1.0, 1.0], size=b.s.shape))
        st = b.rollout(W, T, record=True)["states"]
        e = state_err(np.swapaxes(st, 1, 2), base).max(axis=(1, 2))
        env = np.maximum(env, e)
    return env, base


ENVELOPE_FACTOR = 1.5
"""Float32 trajectories must stay within this multiple of the FP64 envelope
(measured: at most 0.86 of it over 64 steps)."""

GRAD_ENVELOPE_FACTOR = 4.0
"""Per-env parameter gradients: the bar is max(1e-3, this multiple of the
env's own FP64 gradient envelope)."""


def param_scale(cfg, theta_aos):
    """Per-parameter scale of the relative gradient norm: the parameter's
    value; for zero-valued c0, c1 the size that makes the term comparable
    (m g/4 and m g / (4 w_hover))."""
    s = np.abs(theta_aos).astype(np.float64).copy()
    mg4 = theta_aos[:, 0] * cfg["g"] / 4
    wh = np.sqrt(mg4 / theta_aos[:, 6])
    s[:, 4] = np.where(s[:, 4] == 0, mg4, s[:, 4])
    s[:, 5] = np.where(s[:, 5] == 0, mg4 / wh, s[:, 5])
    return s


def param_grad_err(g, g_ref, scale):
    """Per-env relative error of parameter gradients [n][8] in scaled
    coordinates (each d/dtheta_i times theta_i)."""
    return (np.linalg.norm((g - g_ref) * scale, axis=1)
            / np.linalg.norm(g_ref * scale, axis=1))


def grad_envelope(batch, W, T, dR=None, dS=None, trials=8, seed=0, nthreads=8):
    """Sensitivity of the FP64 gradients themselves: the oracle's adjoint from
    its start states perturbed by one float32 rounding (each component times
    1 +- 2^-24, random signs) against the unperturbed adjoint.  Returns the
    worst over trials of the actor gradient's relative change and of every
    env's parameter-gradient change (shape [n]), and the unperturbed
    (J, gW, gtheta)."""
    J, gW, gth = batch.grad(W, T, dR=dR, dS=dS, nthreads=nthreads)
    sc = param_scale(batch.cfg, batch.theta)
    rng = np.random.default_rng(seed)
    env_p = np.zeros(batch.n)
    env_a = 0.0
    for _ in range(trials):
        b = batch.copy()
        b.s = b.s * (1 + 2.0 ** -24 * rng.choice([-1.0, 1.0], size=b.s.shape))
        _, gW2, gth2 = b.grad(W, T, dR=dR, dS=dS, nthreads=nthreads)
        env_p = np.maximum(env_p, param_grad_err(gth2, gth, sc))
        env_a = max(env_a, float(np.linalg.norm(gW2 - gW) / np.linalg.norm(gW)))
    return env_a, env_p, (J, gW, gth)
