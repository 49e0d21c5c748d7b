"""Set-point shift of the actor's observation (Sec. IV: a position controller
follows any set point through its observed position and velocity errors,
clipped to the trained range) against the FP64 oracle, through the C ABI.

The oracle side is written from the definition: observe the state with p and
v replaced by the clipped errors (and the step's noise), evaluate the actor
on it, and advance the true state one step with that action.
Bar: 1e-5 per step (tests/parity.py)."""
import numpy as np
import pytest

import workloads as wl
from parity import STEP_TOL, max_state_err, reward_err

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


def oracle_step(orc, cfg, s, h, t_ep, ep, th, W, target, pc, vc, ids=None):
    """One step of every env from float32 inputs: the actor sees the shifted,
    clipped position and velocity (with its observation noise when on)."""
    n = s.shape[1]
    acts = np.zeros((1, n, 4))
    for i in range(n):
        x = s[:, i].astype(np.float64).copy()
        x[0:3] = np.clip(x[0:3] - target[0:3, i], -pc, pc)
        x[7:10] = np.clip(x[7:10] - target[3:6, i], -vc, vc)
        H = h[:, :, i].astype(np.float64)                       # [32][4]
        env = i if ids is None else int(ids[i])
        if cfg["flags"] & wl.F_OBS_NOISE:
            o = orc.observe_noisy(cfg, env, int(ep[i]), int(t_ep[i]), x, H)
        else:
            o = orc.observe(x, H)
        acts[0, i] = orc.actor(W, o)
    b = orc.Batch(cfg, n)
    b.set_soa(s, h, t_ep=t_ep, ep=ep, theta_soa=th)
    out = b.rollout(None, 1, actions=acts)
    return b, out, acts[0]


@pytest.mark.parametrize("extras", [False, True])
@pytest.mark.parametrize("variant", list(VARIANTS))
def test_setpoint_one_step(pkg, oracle_lib, variant, extras):
    n, pc, vc = 300, 0.2, 1.0
    cfg = wl.crazyflie_config(n_envs=n, dr_enable=1, flags=wl.F_RENORM_Q, max_episode_steps=0)
    if extras:
        cfg = wl.training_extras(cfg)
    sim = pkg.QuadSim(cfg)
    sim.set_variant(VARIANTS[variant], 0, True)
    W = wl.random_actor(3)
    s, h = wl.random_states(n, seed=12)
    rng = np.random.default_rng(13)
    target = np.concatenate([rng.uniform(-0.5, 0.5, (3, n)), rng.uniform(-1.5, 1.5, (3, n))])
    target = target.astype(np.float32)
    t_ep = rng.integers(0, 100, n).astype(np.int32)
    ep = rng.integers(0, 5, n).astype(np.int32)
    sim.set_state(state=s, hist=h, t_ep=t_ep, episode=ep)
    sim.set_target(torch.as_tensor(target), pc, vc)
    th = np_(sim.get_params())
    r, _ = sim.step(actor=sim.actor_tensor(W))
    ref, out, acts = oracle_step(oracle_lib, cfg, s, h, t_ep, ep, th, W,
                                 target.astype(np.float64), pc, vc)
    st = sim.get_state()
    assert max_state_err(np_(st["state"]), ref.s) < STEP_TOL
    assert reward_err(np_(r), out["rewards"][0]) < STEP_TOL
    # the applied action is the newest history slot
    assert np.allclose(np_(st["hist"])[31].T, acts, rtol=0, atol=2e-6)
    sim.close()


def test_setpoint_observation_and_clear(pkg, oracle_lib):
    """sim_observe's actor observation carries the shift (the critic's stays
    absolute); removing the set point restores the plain step bit for bit."""
    n = 200
    cfg = wl.crazyflie_config(n_envs=n, dr_enable=1, flags=wl.F_RENORM_Q, max_episode_steps=0)
    sim = pkg.QuadSim(cfg)
    s, h = wl.random_states(n, seed=3)
    sim.set_state(state=s, hist=h)
    target = np.tile(np.array([[0.3], [-0.1], [0.05], [0.5], [0.0], [-2.0]], np.float32), (1, n))
    sim.set_target(torch.as_tensor(target), 0.2, 1.0)
    o = sim.observe()
    oa, oc = np_(o["actor"]), np_(o["critic"])
    exp_p = np.clip(s[0:3] - target[0:3], -0.2, 0.2)
    exp_v = np.clip(s[7:10] - target[3:6], -1.0, 1.0)
    assert np.allclose(oa[0:3], exp_p, rtol=0, atol=1e-7)
    assert np.allclose(oa[12:15], exp_v, rtol=0, atol=1e-7)
    assert np.array_equal(oc[0:3], s[0:3]) and np.array_equal(oc[12:15], s[7:10])
    sim.set_target(None)
    a = sim.actor_tensor(wl.random_actor(3))
    snap = {k: v.clone() for k, v in sim.get_state().items()}
    sim.rollout(a, 20, rewards=False, dones=False)
    x1 = np_(sim.get_state()["state"])
    other = pkg.QuadSim(cfg)
    other.set_state(**snap)
    other.rollout(a, 20, rewards=False, dones=False)
    assert np.array_equal(x1, np_(other.get_state()["state"]))
    sim.close()
    other.close()


def test_setpoint_refused_for_taped_rollouts(pkg):
    from paper_2311_13081_amd import SimError
    n = 64
    cfg = wl.crazyflie_config(n_envs=n, flags=wl.F_RENORM_Q, max_episode_steps=0,
                              max_tape_horizon=8, ckpt_every=4)
    sim = pkg.QuadSim(cfg)
    sim.set_target(torch.zeros(6, n), 0.2, 1.0)
    a = sim.actor_tensor(wl.random_actor(3))
    with pytest.raises(SimError) as ei:
        sim.rollout(a, 8, record_tape=True)
    assert ei.value.code == -4
    sim.set_target(None)
    sim.rollout(a, 8, record_tape=True)
    sim.close()


def test_tracking_runs(pkg):
    """The tracking loop flies a short figure eight with the hover-biased
    policy and reports finite errors per env (mechanics only: this policy is
    not trained to track)."""
    from paper_2311_13081_amd.tracking import track
    cfg = wl.crazyflie_config(n_envs=16, flags=wl.F_RENORM_Q, max_episode_steps=0)
    sim = pkg.QuadSim(cfg)
    e, exy = track(sim, sim.actor_tensor(wl.sysid_actor(0)), period=1.0, cycles=2)
    assert e.shape == (16,) and bool(torch.isfinite(e).all()) and bool((exy <= e + 1e-6).all())
    sim.close()
