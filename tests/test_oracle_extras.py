"""Pins for the oracle's training extras (Sec. IV, asymmetric actor-critic
paragraph): the per-episode force/torque disturbance, the actor's observation
noise and the 28-value critic observation.

Closed forms: a constant force on a body with no thrust and no rotation gives
a constant acceleration f/m - g e_z, so position is quadratic in time and RK4
reproduces it to rounding; a torque along a principal axis of a body that
rotates about that axis only gives a constant angular acceleration tau/J
(the gyroscopic term w x Jw vanishes), so the rate is linear in time.
Distributions: bounds, moments and Kolmogorov-Smirnov tests of the draws.
The adjoint with both extras on is pinned by central differences of the
oracle's own loss.
"""
import numpy as np
import pytest
from scipy import stats

import workloads as wl


def extras_cfg(**kw):
    return wl.training_extras(wl.crazyflie_config(**kw))


def still_body(cfg):
    th = np.array(cfg["nominal"], np.float64)
    x = np.zeros(17)
    x[3] = 1.0
    return th, x


def test_force_disturbance_gives_exact_parabola(oracle_lib):
    cfg = wl.crazyflie_config()
    th, x = still_body(cfg)
    x[0:3] = (0.1, -0.2, 0.3)
    x[7:10] = (0.5, 0.0, -0.25)
    d = np.array([0.004, -0.011, 0.007, 0.0, 0.0, 0.0])
    u = np.zeros(4)
    acc = d[:3] / th[0] - np.array([0.0, 0.0, cfg["g"]])
    y = x.copy()
    for n in range(1, 51):
        y = oracle_lib.rk4(cfg, th, y, u, dist=d)
        t = n * cfg["dt"]
        assert np.allclose(y[0:3], x[0:3] + x[7:10] * t + 0.5 * acc * t * t, rtol=0, atol=1e-13)
        assert np.allclose(y[7:10], x[7:10] + acc * t, rtol=0, atol=1e-13)
    # the derivative itself: the force enters as f/m
    dx0 = oracle_lib.dynamics(cfg, th, x, u)
    dx1 = oracle_lib.dynamics(cfg, th, x, u, dist=d)
    assert np.allclose(dx1[7:10] - dx0[7:10], d[:3] / th[0], rtol=1e-14, atol=0)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_torque_disturbance_gives_linear_rate(oracle_lib, axis):
    cfg = wl.crazyflie_config()
    th, x = still_body(cfg)
    tau = 3e-5
    d = np.zeros(6)
    d[3 + axis] = tau
    y = x.copy()
    for n in range(1, 41):
        y = oracle_lib.rk4(cfg, th, y, np.zeros(4), dist=d)
        t = n * cfg["dt"]
        w = np.zeros(3)
        w[axis] = tau * t / th[1 + axis]
        assert np.allclose(y[10:13], w, rtol=1e-12, atol=1e-15)


def test_disturbance_draws(oracle_lib):
    cfg = extras_cfg()
    F, Tq = cfg["dist_force"], cfg["dist_torque"]
    D = np.array([oracle_lib.disturbance(cfg, e, ep) for e in range(400) for ep in range(10)])
    assert np.all(np.abs(D[:, :3]) <= F) and np.all(np.abs(D[:, 3:]) <= Tq)
    U = np.concatenate([(D[:, :3] / F + 1) / 2, (D[:, 3:] / Tq + 1) / 2], axis=1)
    for k in range(6):
        assert stats.kstest(U[:, k], "uniform").pvalue > 1e-3
    c = np.corrcoef(U.T)
    assert np.abs(c - np.eye(6)).max() < 0.06
    # keyed by the episode: a new draw per episode, fixed within it
    assert not np.allclose(oracle_lib.disturbance(cfg, 3, 0), oracle_lib.disturbance(cfg, 3, 1))
    assert np.array_equal(oracle_lib.disturbance(cfg, 3, 2), oracle_lib.disturbance(cfg, 3, 2))
    # off without the flag
    off = dict(cfg, flags=wl.F_RENORM_Q)
    assert not oracle_lib.disturbance(off, 3, 2).any()


def test_noise_draws_are_standard_normal(oracle_lib):
    cfg = extras_cfg()
    Z = np.array([oracle_lib.normals18(cfg, e, 0, t) for e in range(100) for t in range(60)])
    z = Z.ravel()
    assert abs(z.mean()) < 0.02 and abs(z.std() - 1) < 0.02
    assert stats.kstest(z, "norm").pvalue > 1e-3
    c = np.corrcoef(Z.T)
    assert np.abs(c - np.eye(18)).max() < 0.08
    # each step of an episode gets its own draw
    assert not np.allclose(oracle_lib.normals18(cfg, 1, 0, 5), oracle_lib.normals18(cfg, 1, 0, 6))


def test_noisy_observation_structure(oracle_lib):
    cfg = extras_cfg()
    b = oracle_lib.Batch.init(cfg, 3)
    s, H = b.s[1], b.H[1]
    o = oracle_lib.observe(s, H)
    on = oracle_lib.observe_noisy(cfg, 1, 4, 17, s, H)
    z = oracle_lib.normals18(cfg, 1, 4, 17)
    sig = np.repeat(cfg["obs_noise"], [3, 9, 3, 3])
    assert np.allclose(on[:18] - o[:18], sig * z, rtol=0, atol=1e-15)
    assert np.array_equal(on[18:], o[18:])
    off = dict(cfg, flags=wl.F_RENORM_Q)
    assert np.array_equal(oracle_lib.observe_noisy(off, 1, 4, 17, s, H), o)


def test_critic_observation_layout(oracle_lib):
    cfg = extras_cfg()
    b = oracle_lib.Batch.init(cfg, 2)
    s = b.s[1]
    oc = oracle_lib.critic_obs(cfg, 1, 6, s)
    R = oracle_lib.rotmat(s[3:7])
    expect = np.concatenate([s[0:3], R.ravel(), s[7:10], s[10:13], s[13:17],
                             oracle_lib.disturbance(cfg, 1, 6)])
    assert oc.shape == (28,) and np.array_equal(oc, expect)


def test_rollout_uses_episode_disturbance_and_noise(oracle_lib):
    """Batched steps equal a hand-driven loop of observe_noisy + actor + rk4
    with the episode's disturbance, across a truncation reset."""
    cfg = extras_cfg(max_episode_steps=5, flags=wl.F_RENORM_Q | wl.F_AUTORESET)
    cfg = wl.training_extras(cfg)
    W = wl.random_actor(2).astype(np.float64)
    b = oracle_lib.Batch.init(cfg, 2)
    ref = b.copy()
    out = b.rollout(W, 8, record=True)
    s, H = ref.s[1].copy(), ref.H[1].copy()
    th = ref.theta[1]
    t_ep, ep = 0, 0
    for t in range(8):
        o = oracle_lib.observe_noisy(cfg, 1, ep, t_ep, s, H)
        a = oracle_lib.actor(W, o)
        u = cfg["rpm_min"] + 0.5 * (a + 1) * (cfg["rpm_max"] - cfg["rpm_min"])
        s = oracle_lib.rk4(cfg, th, s, u, dist=oracle_lib.disturbance(cfg, 1, ep))
        s[3:7] /= np.linalg.norm(s[3:7])
        H = np.concatenate([H[1:], a[None]])
        t_ep += 1
        if t_ep >= 5:
            assert out["dones"][t, 1] == 2
            break
        assert np.allclose(out["states"][t + 1, 1], s, rtol=0, atol=1e-12)
    assert ep == 0 and b.ep[1] == 1


def test_adjoint_with_extras_matches_central_fd(oracle_lib):
    cfg = extras_cfg(max_episode_steps=0, dr_enable=1)
    # stronger disturbance so its terms in the parameter gradient matter
    cfg["dist_force"] *= 10
    cfg["dist_torque"] *= 10
    n, T = 3, 12
    b = oracle_lib.Batch.init(cfg, n)
    b.t_ep[:] = [0, 7, 30]
    b.ep[:] = [0, 2, 5]
    W = wl.random_actor(4).astype(np.float64)
    rng = np.random.default_rng(1)
    dR = rng.uniform(0.5, 1.5, size=(T, n))
    dS = rng.normal(size=(T + 1, n, 17)) * 1e-2
    dS[:, :, 13:17] *= 1e-4
    _, gW, gth = b.grad(W, T, dR=dR, dS=dS)
    for i in range(n):
        fd = np.zeros(8)
        sc = np.abs(b.theta[i]).copy()
        sc[4] = b.theta[i, 0] * cfg["g"] / 4
        sc[5] = sc[4] / 14000.0
        for k in range(8):
            h = 1e-6 * sc[k]
            bp, bm = b.copy(), b.copy()
            bp.theta[i, k] += h
            bm.theta[i, k] -= h
            fd[k] = (bp.grad(W, T, dR=dR, dS=dS, want_grad=False)[0] -
                     bm.grad(W, T, dR=dR, dS=dS, want_grad=False)[0]) / (2 * h)
        err = np.linalg.norm((gth[i] - fd) * sc) / np.linalg.norm(fd * sc)
        assert err < 1e-6, (i, err)
