"""Episode accumulators of every forward kernel (running return, last finished
episode's return and length; Sec. V, Training) against the FP64 oracle's,
through the C ABI (sim_get_state / sim_set_state).

Bars: lengths bit-exact; returns |gpu - ref| / max(|ref|, 1) <= 1e-4 (sums of
rewards that each meet the 1e-5 per-step bar)."""
import numpy as np
import pytest

import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

VARIANTS = {"plain": 1, "valu": 2, "mfma": 3, "mfma4": 4, "split": 5}
RET_TOL = 1e-4


@pytest.fixture(scope="module")
def pkg():
    import paper_2311_13081_amd as p
    p.load()
    return p


def np_(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(g, r):
    g = np.asarray(g, np.float64)
    r = np.asarray(r, np.float64)
    return float((np.abs(g - r) / np.maximum(np.abs(r), 1.0)).max())


def truncation_cfg(n, flags=0):
    # fixed 7-step episodes (no early termination), so every env closes its
    # episodes at the same steps on both sides
    return wl.crazyflie_config(n_envs=n, dr_enable=1, max_episode_steps=7,
                               flags=wl.F_RENORM_Q | wl.F_AUTORESET | flags)


@pytest.mark.parametrize("variant", list(VARIANTS))
def test_episode_stats_match_oracle(pkg, oracle_lib, variant):
    """777 randomised envs, 40 steps of the Xavier policy in 7-step episodes
    (5 closed, 5 steps into the sixth): accumulators equal the oracle's."""
    n, T = 777, 40
    cfg = truncation_cfg(n)
    sim = pkg.QuadSim(cfg)
    sim.set_variant(VARIANTS[variant], 0, True)
    W = wl.xavier_actor(0)
    sim.rollout(sim.actor_tensor(W), T, rewards=False, dones=False)
    st = sim.get_state()
    ref = oracle_lib.Batch.init(cfg, n)
    ref.rollout(W, T, nthreads=8)
    ret, ln = np_(st["returns"]), np_(st["last_len"])
    print(f"{variant}: running return err {rel(ret[0], ref.ret_cur):.2e}, last return err "
          f"{rel(ret[1], ref.ret_last):.2e}")
    assert np.array_equal(ln, ref.len_last) and np.all(ln == 7)
    assert np.array_equal(np_(st["t_ep"]), ref.t_ep)
    assert rel(ret[0], ref.ret_cur) < RET_TOL
    assert rel(ret[1], ref.ret_last) < RET_TOL
    sim.close()


@pytest.mark.parametrize("variant", list(VARIANTS))
def test_episode_stats_equal_recorded_outputs(pkg, variant):
    """With termination, uneven episodes: the accumulators are the sums of the
    rollout's own recorded rewards split at its recorded done flags (summed
    here in double precision), in one persistent launch and in 13-step graph
    launches alike (bitwise)."""
    n, T = 2048, 300
    cfg = wl.crazyflie_config(n_envs=n, dr_enable=1, max_episode_steps=100,
                              flags=wl.F_RENORM_Q | wl.F_TERMINATE | wl.F_AUTORESET)
    W = wl.xavier_actor(0)
    res = []
    for spl in (0, 13):
        sim = pkg.QuadSim(cfg)
        sim.set_variant(VARIANTS[variant], spl, True)
        out = sim.rollout(sim.actor_tensor(W), T)
        st = sim.get_state()
        res.append({k: np_(v) for k, v in list(out.items()) + list(st.items())})
        sim.close()
    for k in ("returns", "last_len"):
        assert np.array_equal(res[0][k], res[1][k]), k
    r, d = res[0]["rewards"].astype(np.float64), res[0]["dones"]
    cur, last = np.zeros(n), np.zeros(n)
    length, last_len = np.zeros(n, np.int64), np.zeros(n, np.int64)
    for t in range(T):
        cur += r[t]
        length += 1
        fin = d[t] != 0
        last[fin], last_len[fin] = cur[fin], length[fin]
        cur[fin], length[fin] = 0.0, 0
    assert (d & 1).any() and (d != 0).sum(axis=0).min() >= 2
    assert np.array_equal(res[0]["last_len"], last_len)
    assert np.array_equal(res[0]["t_ep"], length)
    assert rel(res[0]["returns"][0], cur) < 1e-5
    assert rel(res[0]["returns"][1], last) < 1e-5


def test_episode_stats_fp64_path(pkg, oracle_lib):
    n, T = 300, 40
    cfg = truncation_cfg(n, wl.F_FP64)
    sim = pkg.QuadSim(cfg)
    W = wl.xavier_actor(0)
    sim.rollout(sim.actor_tensor(W), T, rewards=False, dones=False)
    st = sim.get_state()
    ref = oracle_lib.Batch.init(cfg, n)
    ref.rollout(W, T, nthreads=8)
    ret = np_(st["returns"])
    assert np.array_equal(np_(st["last_len"]), ref.len_last)
    # float32 rounding of the returned double sums
    assert rel(ret[0], ref.ret_cur) < 1e-6 and rel(ret[1], ref.ret_last) < 1e-6
    sim.close()


def test_episode_stats_dynamics_only(pkg, oracle_lib):
    """Given actions (the dynamics-only rollout) accumulate like policy steps."""
    n, T = 500, 30
    cfg = truncation_cfg(n)
    sim = pkg.QuadSim(cfg)
    a = wl.random_actions(n, seed=4)
    sim.rollout_actions(torch.as_tensor(a).cuda(), T, rewards=False, dones=False)
    st = sim.get_state()
    ref = oracle_lib.Batch.init(cfg, n)
    ref.rollout(None, T, actions=np.broadcast_to(a.T[None], (T, n, 4)).astype(np.float64))
    ret = np_(st["returns"])
    assert np.array_equal(np_(st["last_len"]), ref.len_last)
    assert rel(ret[0], ref.ret_cur) < RET_TOL and rel(ret[1], ref.ret_last) < RET_TOL
    sim.close()


def test_episode_stats_snapshot_and_reset(pkg):
    """set_state restores the accumulators; reset zeroes them."""
    n = 256
    cfg = truncation_cfg(n)
    sim = pkg.QuadSim(cfg)
    a = sim.actor_tensor(wl.xavier_actor(0))
    sim.rollout(a, 10, rewards=False, dones=False)
    snap = {k: v.clone() for k, v in sim.get_state().items()}
    assert np_(snap["last_len"]).min() == 7 and np.abs(np_(snap["returns"])).max() > 0
    sim.rollout(a, 5, rewards=False, dones=False)
    sim.set_state(**snap)
    again = sim.get_state()
    for k in ("returns", "last_len"):
        assert np.array_equal(np_(again[k]), np_(snap[k]))
    sim.reset()
    z = sim.get_state()
    assert not np_(z["returns"]).any() and not np_(z["last_len"]).any()
    sim.close()
