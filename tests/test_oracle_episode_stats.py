"""Episode accumulators of the FP64 oracle: the return of the running episode
and the return and length of the last finished one (Sec. V, Training:
episode length and return measure training progress).  Pinned by a closed
form at hover, by the split of one rollout into shorter calls, and by the
bookkeeping identity that every reward belongs to exactly one episode."""
import numpy as np
import pytest

import workloads as wl


def test_hover_episode_return_closed_form(oracle_lib):
    """Level, still, at the origin, rotors at the hover speed, commanding the
    hover action, with the reward's action baseline C_rab set to that action:
    every penalty term is zero, so each step earns exactly C_rs.  A truncated
    episode of k steps returns k C_rs and has length k, and the running
    return restarts at zero with the reset."""
    k = 7
    cfg = wl.crazyflie_config(n_envs=1, flags=wl.F_RENORM_Q | wl.F_AUTORESET,
                              max_episode_steps=k, dr_enable=0)
    th = np.array(cfg["nominal"], np.float64)
    wh = oracle_lib.hover_rpm(cfg, th)
    ah = 2.0 * (wh - cfg["rpm_min"]) / (cfg["rpm_max"] - cfg["rpm_min"]) - 1.0
    cfg["C_rab"] = ah
    b = oracle_lib.Batch(cfg, 1)
    b.theta[0] = th
    b.s[0] = np.array([0, 0, 0, 1, 0, 0, 0, 0, 0, 0, 0, 0, 0] + [wh] * 4, np.float64)
    b.H[0] = ah
    out = b.rollout(None, k, actions=np.full((k, 1, 4), ah), record=True)
    assert not out["dones"][:-1].any() and out["dones"][-1, 0] == 2
    assert np.allclose(out["rewards"][:, 0], cfg["C_rs"], rtol=1e-12, atol=0)
    assert b.len_last[0] == k
    assert b.ret_last[0] == pytest.approx(k * cfg["C_rs"], rel=1e-12)
    assert b.ret_cur[0] == 0.0
    assert b.t_ep[0] == 0 and b.ep[0] == 1


def _cfg(n):
    return wl.crazyflie_config(n_envs=n, dr_enable=1, max_episode_steps=20,
                               flags=wl.F_RENORM_Q | wl.F_TERMINATE | wl.F_AUTORESET)


def test_accumulators_carry_across_calls(oracle_lib):
    """One 60-step rollout and the same 60 steps in calls of 7, 13 and 40
    steps, or of one step each, leave identical accumulators."""
    n, W = 64, wl.xavier_actor(0)
    runs = []
    for split in ([60], [7, 13, 40], [1] * 60):
        b = oracle_lib.Batch.init(_cfg(n), n)
        for T in split:
            b.rollout(W, T)
        runs.append((b.ret_cur.copy(), b.ret_last.copy(), b.len_last.copy(), b.ep.copy()))
    assert runs[0][3].max() >= 3          # several episodes ended
    for other in runs[1:]:
        for a, c in zip(runs[0], other):
            assert np.array_equal(a, c)


def test_every_reward_belongs_to_one_episode(oracle_lib):
    """Stepping one step at a time and collecting the last finished episode's
    return and length whenever an episode ends: the collected returns plus
    the running return add up to all rewards received, the lengths plus the
    running episode's step count to the number of steps, and each collected
    length is the number of steps since the previous end."""
    n, T, W = 48, 80, wl.xavier_actor(0)
    b = oracle_lib.Batch.init(_cfg(n), n)
    total = np.zeros(n)
    closed = np.zeros(n)
    lens = np.zeros(n, np.int64)
    since = np.zeros(n, np.int64)
    for _ in range(T):
        out = b.rollout(W, 1)
        total += out["rewards"][0]
        since += 1
        d = out["dones"][0] != 0
        closed[d] += b.ret_last[d]
        lens[d] += b.len_last[d]
        assert np.array_equal(b.len_last[d], since[d])
        since[d] = 0
    assert (b.ep >= 2).any()
    assert np.allclose(closed + b.ret_cur, total, rtol=1e-12, atol=1e-12)
    assert np.array_equal(lens + b.t_ep, np.full(n, T))


def test_batch_equals_single_env_runs(oracle_lib):
    n, W = 16, wl.xavier_actor(0)
    ids = np.arange(n, dtype=np.uint32)
    b = oracle_lib.Batch.init(_cfg(n), n)
    b.rollout(W, 50)
    for i in range(n):
        s = oracle_lib.Batch.init(_cfg(1), 1, ids=ids[i:i + 1])
        s.rollout(W, 50)
        assert s.ret_cur[0] == b.ret_cur[i] and s.ret_last[0] == b.ret_last[i]
        assert s.len_last[0] == b.len_last[i]
