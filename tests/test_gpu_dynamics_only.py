"""Dynamics-only rollouts (policy replaced by given actions) against the
oracle and against stepping one action at a time."""
import numpy as np
import pytest

import workloads as wl
from parity import STEP_TOL, max_state_err, state_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pkg():
    import paper_2311_13081_amd as p
    p.load()
    return p


def np_(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def test_hover_holds_for_long_rollouts(pkg, oracle_lib):
    """Level, still bodies at the hover speed commanding the hover action stay
    put for 2000 steps (constant-action mode)."""
    n = 8192
    cfg = wl.crazyflie_config(n_envs=n, max_episode_steps=0)
    sim = pkg.QuadSim(cfg)
    wh = oracle_lib.hover_rpm(cfg, np.array(cfg["nominal"]))
    ah = 2 * wh / cfg["rpm_max"] - 1
    s = np.zeros((17, n), np.float32)
    s[0:3] = np.random.default_rng(0).uniform(-0.3, 0.3, size=(3, n))
    s[3] = 1.0
    s[13:17] = wh
    sim.set_state(state=s)
    a = torch.full((4, n), ah, dtype=torch.float32, device="cuda")
    out = sim.rollout_actions(a, 2000)
    sf = np_(sim.get_state()["state"])
    err = np.abs(sf - s).max(axis=1)
    print("hover drift after 2000 steps per component", err)
    assert err[0:3].max() < 1e-3 and err[13:17].max() < 0.05
    assert not np_(out["dones"]).any()
    sim.close()


def test_per_step_actions_match_oracle_and_single_steps(pkg, oracle_lib):
    n, T = 700, 12
    flags = wl.F_RENORM_Q | wl.F_TERMINATE | wl.F_AUTORESET
    cfg = wl.crazyflie_config(n_envs=n, dr_enable=1, flags=flags, max_episode_steps=7)
    A = np.stack([wl.random_actions(n, seed=100 + t) for t in range(T)])   # [T][4][N]
    sim = pkg.QuadSim(cfg)
    st0 = {k: v.clone() for k, v in sim.get_state().items()}
    out = sim.rollout_actions(torch.as_tensor(A).cuda(), T, states=True)
    st = {k: np_(v) for k, v in sim.get_state().items()}
    # the oracle from the same seeded start
    ref = oracle_lib.Batch.init(cfg, n)
    ro = ref.rollout(None, T, actions=np.transpose(A, (0, 2, 1)).astype(np.float64), record=True)
    d = np_(out["dones"])
    assert np.array_equal(d, ro["dones"])          # truncation at 7 resets everyone
    assert (d == 2).sum() == n
    e = state_err(np_(out["states"]), ro["states"]).max(axis=(1, 2))
    assert e[1] < STEP_TOL and e.max() < 1e-4
    assert np.array_equal(st["episode"], ref.ep) and np.array_equal(st["t_ep"], ref.t_ep)
    # history: the actions since the reset (given float32 values, exact), the
    # hover fill of the reset body before that (float32 arithmetic against
    # double: the initial-history tolerance)
    hg = np.transpose(st["hist"], (2, 0, 1))
    print("history max abs error", np.abs(hg - ref.H).max())
    assert np.allclose(hg, ref.H, rtol=2e-6, atol=2e-7)
    te = st["t_ep"]
    assert te.min() >= 1 and te.max() < T
    for e_ in range(n):
        k = int(te[e_])
        assert np.array_equal(hg[e_, 32 - k:], A[T - k:, :, e_])
    # the same as T single steps with external actions, bitwise for the history
    sim.set_state(**st0)
    for t in range(T):
        sim.step(actions=torch.as_tensor(A[t]).cuda())
    st1 = {k: np_(v) for k, v in sim.get_state().items()}
    assert np.array_equal(st1["hist"], st["hist"])
    assert np.array_equal(st1["episode"], st["episode"])
    assert max_state_err(st1["state"], st["state"].T) < 1e-6
    sim.close()


def test_constant_actions_short_rollout_keeps_old_history(pkg):
    """T < 32 without reset: the older history slots survive, shifted."""
    n, T = 256, 5
    cfg = wl.crazyflie_config(n_envs=n, max_episode_steps=0)
    sim = pkg.QuadSim(cfg)
    _, h = wl.random_states(n, seed=3)
    sim.set_state(hist=h)
    a = torch.as_tensor(wl.random_actions(n, seed=4)).cuda()
    sim.rollout_actions(a, T)
    hg = np_(sim.get_state()["hist"])
    assert np.array_equal(hg[:32 - T], h[T:])
    for s in range(32 - T, 32):
        assert np.array_equal(hg[s], np_(a))
    sim.close()


@pytest.mark.parametrize("max_steps", [1, 3, 9])
def test_short_episodes_long_launch_equals_single_steps(pkg, max_steps):
    """Episodes of 1, 3 or 9 steps inside one 96-step launch (envs reset
    again before the drawn-ahead start states are refilled) against 96
    one-step launches of the same kernel, which draw in place: bitwise."""
    n, T = 999, 96
    flags = wl.F_RENORM_Q | wl.F_TERMINATE | wl.F_AUTORESET
    cfg = wl.crazyflie_config(n_envs=n, dr_enable=1, flags=flags, max_episode_steps=max_steps)
    A = torch.as_tensor(np.stack([wl.random_actions(n, seed=300 + t) for t in range(T)])).cuda()
    sim = pkg.QuadSim(cfg)
    st0 = {k: v.clone() for k, v in sim.get_state().items()}
    out = sim.rollout_actions(A, T)
    one = {k: np_(v) for k, v in sim.get_state().items()}
    one.update({k: np_(v) for k, v in out.items()})
    assert (one["dones"] != 0).sum() >= n * (T // max_steps) // 2
    sim.set_state(**st0)
    r, d = [], []
    for t in range(T):
        o = sim.rollout_actions(A[t:t + 1], 1)   # per-step form, as above
        r.append(np_(o["rewards"])[0])
        d.append(np_(o["dones"])[0])
    many = {k: np_(v) for k, v in sim.get_state().items()}
    many.update(rewards=np.stack(r), dones=np.stack(d))
    for k in one:
        assert np.array_equal(one[k], many[k], equal_nan=True), (max_steps, k)
    sim.close()
