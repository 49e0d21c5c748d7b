"""Training extras on the GPU (per-episode disturbance, actor observation
noise, critic observation) against the FP64 oracle, through the C ABI.

The extras draw from the same counter RNG on both sides (the kernels in
float, the oracle in double), so the comparisons keep the fp32 step bar of
1e-5, the strict 1e-4 trajectory bar for the double-precision path, bit-exact
episode bookkeeping, and the 1e-3 gradient bar.
"""
import numpy as np
import pytest

import workloads as wl
from parity import STEP_TOL, TRAJ_TOL, max_state_err, reward_err, state_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

VARIANTS = {"plain": 1, "valu": 2, "mfma": 3, "mfma4": 4, "split": 5}


@pytest.fixture(scope="module")
def pkg():
    import paper_2311_13081_amd as p
    p.load()
    return p


def np_(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def extras(**kw):
    return wl.training_extras(wl.crazyflie_config(**kw))


def counters(n, seed=1):
    rng = np.random.default_rng(seed)
    return (rng.integers(0, 400, n).astype(np.int32), rng.integers(0, 40, n).astype(np.int32))


@pytest.mark.parametrize("variant", list(VARIANTS))
def test_one_step_with_extras(pkg, oracle_lib, variant):
    n = 1000
    cfg = extras(n_envs=n, dr_enable=1, max_episode_steps=0)
    sim = pkg.QuadSim(cfg)
    sim.set_variant(VARIANTS[variant])
    W = wl.random_actor(3)
    s, h = wl.random_states(n, seed=21)
    t_ep, ep = counters(n)
    sim.set_state(state=s, hist=h, t_ep=t_ep, episode=ep)
    th = np_(sim.get_params())
    r, _ = sim.step(actor=sim.actor_tensor(W))
    st = sim.get_state()
    ref = oracle_lib.Batch(cfg, n)
    ref.set_soa(s, h, t_ep=t_ep, ep=ep, theta_soa=th)
    out = ref.rollout(W, 1)
    assert max_state_err(np_(st["state"]), ref.s) < STEP_TOL
    assert reward_err(np_(r), out["rewards"][0]) < STEP_TOL
    # the extras matter at this size: without them the step differs
    plain = oracle_lib.Batch(dict(cfg, flags=wl.F_RENORM_Q), n)
    plain.set_soa(s, h, t_ep=t_ep, ep=ep, theta_soa=th)
    plain.rollout(W, 1)
    assert max_state_err(plain.s.T, ref.s) > 10 * STEP_TOL
    sim.close()


def test_observe_matches_oracle_and_feeds_the_actor(pkg, oracle_lib):
    n = 700
    cfg = extras(n_envs=n, dr_enable=1, max_episode_steps=0)
    sim = pkg.QuadSim(cfg)
    s, h = wl.random_states(n, seed=22)
    t_ep, ep = counters(n, seed=2)
    sim.set_state(state=s, hist=h, t_ep=t_ep, episode=ep)
    o = sim.observe()
    ao, co = np_(o["actor"]), np_(o["critic"])
    H = np.transpose(h, (2, 0, 1)).astype(np.float64)
    ao_ref = np.array([oracle_lib.observe_noisy(cfg, e, int(ep[e]), int(t_ep[e]),
                                                s[:, e].astype(np.float64), H[e])
                       for e in range(n)])
    co_ref = np.array([oracle_lib.critic_obs(cfg, e, int(ep[e]), s[:, e].astype(np.float64))
                       for e in range(n)])
    assert np.abs(ao.T - ao_ref).max() < 2e-6
    assert np.abs(co.T[:, :22] - co_ref[:, :22]).max() < 2e-6 * np.abs(co_ref[:, :22]).max()
    assert np.allclose(co.T[:, 22:], co_ref[:, 22:], rtol=1e-6, atol=1e-12)
    # the next policy step sees exactly this observation
    W = wl.random_actor(4)
    sim.step(actor=sim.actor_tensor(W))
    a_gpu = np_(sim.get_state()["hist"])[31].T
    a_ref = np.array([oracle_lib.actor(W, x) for x in ao.T.astype(np.float64)])
    assert np.abs(a_gpu - a_ref).max() < 2e-5
    sim.close()


def test_fp64_trajectory_with_extras_and_resets(pkg, oracle_lib):
    """Double-precision path: strict 1e-4 bar over 200 steps with truncation
    resets (new disturbance per episode), flags and counters bit-exact."""
    n, T = 256, 200
    cfg = extras(n_envs=n, dr_enable=1, max_episode_steps=60,
                 flags=wl.F_RENORM_Q | wl.F_AUTORESET | wl.F_FP64)
    cfg = wl.training_extras(cfg)
    sim = pkg.QuadSim(cfg)
    W = wl.sysid_actor(0)
    out = sim.rollout(sim.actor_tensor(W), T, states=True)
    ref = oracle_lib.Batch.init(cfg, n)
    ro = ref.rollout(W, T, record=True, nthreads=8)
    assert np.array_equal(np_(out["dones"]), ro["dones"])
    st = sim.get_state()
    assert np.array_equal(np_(st["episode"]), ref.ep)
    e = state_err(np_(out["states"]), ro["states"]).max()
    print("fp64 with extras, 200-step max error", e)
    assert e < TRAJ_TOL
    sim.close()


@pytest.mark.parametrize("variant", ["mfma", "mfma4", "split"])
def test_fp32_episodes_with_extras(pkg, oracle_lib, variant):
    """Fused kernels over 150 steps with resets: per-step parity from the
    GPU's own snapshots (the fp32 bar), done flags bit-exact."""
    n, T = 512, 150
    cfg = extras(n_envs=n, dr_enable=1, max_episode_steps=50,
                 flags=wl.F_RENORM_Q | wl.F_AUTORESET)
    cfg = wl.training_extras(cfg)
    sim = pkg.QuadSim(cfg)
    sim.set_variant(VARIANTS[variant])
    W = wl.sysid_actor(0)
    a = sim.actor_tensor(W)
    worst = 0.0
    for t in range(T):
        st = {k: np_(v) for k, v in sim.get_state().items()}
        r, d = sim.step(actor=a)
        ref = oracle_lib.Batch(cfg, n)
        ref.set_soa(st["state"], st["hist"], t_ep=st["t_ep"], ep=st["episode"],
                    theta_soa=np_(sim.get_params()))
        out = ref.rollout(W, 1)
        assert np.array_equal(np_(d), out["dones"][0])
        worst = max(worst, max_state_err(np_(sim.get_state()["state"]), ref.s))
    print(f"{variant} with extras: worst one-step error over {T} steps {worst:.2e}")
    assert worst < STEP_TOL
    assert np_(sim.get_state()["episode"]).min() == 3
    sim.close()


def test_backward_with_extras(pkg, oracle_lib):
    n, T, K = 96, 24, 8
    cfg = extras(n_envs=n, dr_enable=1, max_episode_steps=0, max_tape_horizon=T, ckpt_every=K)
    cfg["dist_force"] *= 10
    cfg["dist_torque"] *= 10
    ob = oracle_lib.Batch.init(cfg, n)
    s32, h32 = (x.astype(np.float32) for x in ob.soa())
    t_ep, ep = counters(n, seed=3)
    sim = pkg.QuadSim(cfg)
    sim.set_state(state=s32, hist=h32, t_ep=t_ep, episode=ep)
    th = np_(sim.get_params())
    W = wl.random_actor(5)
    a = sim.actor_tensor(W)
    sim.rollout(a, T, rewards=True, dones=False, record_tape=True)
    ga, gp = sim.backward(a)
    ga, gp = np_(ga).astype(np.float64), np_(gp).astype(np.float64).T
    ref = oracle_lib.Batch(cfg, n)
    ref.set_soa(s32, h32, t_ep=t_ep, ep=ep, theta_soa=th)
    _, gW, gth = ref.grad(W, T, nthreads=8)
    ea = np.linalg.norm(ga - gW) / np.linalg.norm(gW)
    sc = np.abs(th.T).astype(np.float64)
    sc[:, 4] = th[0] * cfg["g"] / 4
    sc[:, 5] = sc[:, 4] / 14000.0
    epar = np.linalg.norm((gp - gth) * sc, axis=1) / np.linalg.norm(gth * sc, axis=1)
    print(f"extras backward: actor rel err {ea:.2e}, params max {epar.max():.2e}")
    assert ea < 1e-3 and epar.max() < 1e-3
    sim.close()


def test_dynamics_only_with_disturbance(pkg, oracle_lib):
    """12 steps: random actions from random states spin the bodies, and over
    longer horizons float32 rounding grows as in the closed loop."""
    n, T = 400, 12
    cfg = extras(n_envs=n, dr_enable=1, max_episode_steps=0)
    sim = pkg.QuadSim(cfg)
    t_ep, ep = counters(n, seed=4)
    s, h = wl.random_states(n, seed=23)
    sim.set_state(state=s, hist=h, t_ep=t_ep, episode=ep)
    th = np_(sim.get_params())
    A = np.stack([wl.random_actions(n, seed=300 + t) for t in range(T)])
    out = sim.rollout_actions(torch.as_tensor(A).cuda(), T, states=True)
    ref = oracle_lib.Batch(cfg, n)
    ref.set_soa(s, h, t_ep=t_ep, ep=ep, theta_soa=th)
    ro = ref.rollout(None, T, actions=np.transpose(A, (0, 2, 1)).astype(np.float64), record=True)
    e = state_err(np_(out["states"]), ro["states"]).max(axis=(1, 2))
    assert e[1] < STEP_TOL and e.max() < 1e-4
    sim.close()
