"""Closed-loop sensitivity of the fwd64 workload, from the FP64 oracle alone.

Under the seeded Xavier actor the bodies spin up to hundreds of rad/s within
64 steps, and a single float32-sized perturbation of the start state (each
component times 1 +- 2^-24) grows past 1e-4 in the per-step error norm.  This
is why the GPU trajectory bar is stated relative to this envelope: even an
exact-arithmetic integrator fed float32 start states could not stay within
1e-4 of the FP64 trajectory for 64 steps."""
import numpy as np

import workloads as wl
from parity import grad_envelope, oracle_envelope


def test_float32_sized_perturbation_grows_past_1e4_within_64_steps(oracle_lib):
    cfg = wl.workload_config("fwd64")
    W = wl.xavier_actor(0)
    env, base = oracle_envelope(oracle_lib, cfg, W, 64, 64)
    assert env[1] < 1e-5                   # one step: inside the per-step bar
    assert env.max() > 1e-4                # 64 steps: beyond the 1e-4 bar
    w = np.linalg.norm(base[64, :, 10:13], axis=1)
    assert np.median(w) > 100.0            # the bodies spin fast by then


def test_envelope_is_deterministic(oracle_lib):
    cfg = wl.workload_config("fwd64")
    W = wl.xavier_actor(0)
    a, _ = oracle_envelope(oracle_lib, cfg, W, 16, 16)
    b, _ = oracle_envelope(oracle_lib, cfg, W, 16, 16)
    assert np.array_equal(a, b)


def test_sysid_actor_keeps_long_rollouts_finite(oracle_lib):
    """The sys-ID workload rolls out 256 steps without termination.  The
    plain Xavier policy drives part of the batch past the RK4 stability limit
    (states overflow), the scaled, hover-biased policy does not."""
    cfg = wl.workload_config("sysid16384", n_envs=48)
    b = oracle_lib.Batch.init(cfg, 48)
    S = b.copy().rollout(wl.sysid_actor(0), 256, record=True, nthreads=4)["states"]
    assert np.isfinite(S).all()
    assert np.abs(S[:, :, 10:13]).max() < 50.0
    S2 = b.copy().rollout(wl.xavier_actor(0), 256, record=True, nthreads=4)["states"]
    assert not np.isfinite(S2[-1]).all()


def test_grad1024_fp64_gradient_envelope(oracle_lib):
    """Per-env sensitivity of the FP64 parameter gradients of the grad1024
    configuration (1024 nominal envs, horizon 64, seeded Xavier policy, loss
    = sum of rewards): a float32-sized perturbation of the start state moves
    most envs' gradients by a few 1e-6, but a few fast-spinning envs' by
    more than the 1e-3 bar.  This is the allowance the GPU gradient test
    applies to those envs (4 x the env's envelope); the actor gradient, a
    sum over all envs, stays stable."""
    cfg = wl.crazyflie_config(n_envs=1024, flags=wl.F_RENORM_Q, dr_enable=0, max_episode_steps=0,
                              max_tape_horizon=64, ckpt_every=16)
    ob = oracle_lib.Batch.init(cfg, 1024)
    s32, h32 = (x.astype(np.float32) for x in ob.soa())
    b = oracle_lib.Batch(cfg, 1024)
    b.set_soa(s32, h32, theta_soa=ob.theta.T.astype(np.float32))
    env_a, env_p, (J, gW, gth) = grad_envelope(b, wl.xavier_actor(0), 64, nthreads=8)
    assert np.isfinite(J) and np.all(np.isfinite(gth))
    assert np.median(env_p) < 2e-5
    assert np.quantile(env_p, 0.99) < 5e-4
    assert env_p.max() > 1e-3               # some envs are ill-conditioned
    assert env_a < 1e-4
