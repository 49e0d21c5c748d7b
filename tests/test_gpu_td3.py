"""The TD3 training loop's use of the environment, on a short run: the replay
buffer holds post-step states (before the restart of finished envs), every
stored reward equals the FP64 oracle's reward of its transition under the
reward constants in force at the end (the buffer is re-scored after each
curriculum round; without re-scoring the early transitions keep their old
rewards), the curriculum reaches the env, and the evaluation rollouts (the
policy inside the fused step kernel) report episode lengths in range.

Bar: rewards |dr| / max(|r|, 1) <= 1e-5."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def td3():
    import paper_2311_13081_amd as p
    p.load()
    from paper_2311_13081_amd import td3 as t
    return t


def _short(t, recalc):
    cfg = t.TD3Config(total_steps=2500, n_envs=4, warmup=500, curriculum_every=1000,
                      eval_every=1000, eval_envs=64, eval_steps=100, recalc_rewards=recalc,
                      C_factor=dict(C_rp=1.5, C_ra=2.0), C_target=dict(C_rp=10.0, C_ra=1.0))
    return cfg, t.train(cfg)


def _oracle_rewards(oracle_lib, env_cfg, C, replay, ids):
    c = dict(env_cfg, **C)
    s = replay.s_next.cpu().numpy()
    a = replay.a.cpu().numpy()
    return np.array([oracle_lib.reward(c, s[:, i].astype(np.float64), a[i].astype(np.float64))
                     for i in ids])


def test_td3_short_run_mechanics(td3, oracle_lib):
    cfg, out = _short(td3, True)
    rec, buf = out["records"], out["replay"]
    print("td3 short run", rec)
    assert [r["step"] for r in rec] == [1000, 2000, 2500]
    assert [r["stage"] for r in rec] == [0, 1, 2]
    assert out["C"]["C_rp"] == pytest.approx(2.25) and out["C"]["C_ra"] == pytest.approx(0.04)
    for r in rec:
        assert 1 <= r["eval_len_mean"] <= 100 and np.isfinite(r["eval_ret_mean"])
        assert r["train_episodes"] > 0
    assert buf.size == 2500
    ids = np.arange(0, 2500, 7)
    ref = _oracle_rewards(oracle_lib, out["env_cfg"], out["C"], buf, ids)
    r = buf.r.cpu().numpy()[ids].astype(np.float64)
    err = float((np.abs(r - ref) / np.maximum(np.abs(ref), 1.0)).max())
    print(f"stored rewards vs oracle under the final constants: {err:.2e}")
    assert err < 1e-5
    # terminal flags: terminated transitions left the box or went non-finite
    s = buf.s_next.cpu().numpy()
    term = buf.term.cpu().numpy()[:2500] != 0
    out_box = (np.abs(s[0:3]) > np.float32(0.6)).any(axis=0) | \
        (np.abs(s[7:10]) > np.float32(2.0)).any(axis=0) | \
        ~np.isfinite(s).all(axis=0)
    assert np.array_equal(term, out_box[:2500])


def test_td3_without_recalculation_keeps_old_rewards(td3, oracle_lib):
    cfg, out = _short(td3, False)
    buf = out["replay"]
    ids = np.arange(0, 2500, 7)
    ref = _oracle_rewards(oracle_lib, out["env_cfg"], out["C"], buf, ids)
    r = buf.r.cpu().numpy()[ids].astype(np.float64)
    err = np.abs(r - ref) / np.maximum(np.abs(ref), 1.0)
    late = ids >= 2000   # added under the final constants
    assert err[late].max() < 1e-5
    assert (err[~late] > 1e-4).mean() > 0.5


def test_graph_updates_match_eager_updates(td3):
    """The learner's update replayed from the captured graphs (critic only;
    critic, actor and targets) against the same update run eagerly, from the
    same networks, replay contents and random streams: eight updates in
    turn, every replay checked against the eager result, with the other
    learner's eager work between the replays."""
    import copy
    import dataclasses
    t = td3
    dev = torch.device("cuda")
    torch.manual_seed(0)
    cfg = t.TD3Config(total_steps=4096)
    buf = t.Replay(4096, dev)
    g = torch.Generator(device=dev).manual_seed(1)
    n = 4096
    buf.add(torch.randn(n, 146, device=dev, generator=g), torch.randn(n, 28, device=dev, generator=g),
            torch.rand(n, 4, device=dev, generator=g) * 2 - 1, torch.randn(n, device=dev, generator=g),
            torch.randn(n, 146, device=dev, generator=g), torch.randn(n, 28, device=dev, generator=g),
            (torch.rand(n, device=dev, generator=g) < 0.05).float(),
            torch.randn(17, n, device=dev, generator=g))
    nets = (t.Actor().to(dev), t.Critics(cfg.critic_hidden).to(dev))
    learners, gens = [], []
    for graph in (False, True):
        a, c = copy.deepcopy(nets[0]), copy.deepcopy(nets[1])
        at, ct = copy.deepcopy(a), copy.deepcopy(c)
        for p in list(at.parameters()) + list(ct.parameters()):
            p.requires_grad_(False)
        learners.append(t.Learner(dataclasses.replace(cfg, graph_updates=graph), a, c, at, ct,
                                  buf, dev))
        gens.append(torch.Generator(device=dev).manual_seed(7))
    worst = 0.0
    for u in range(1, 9):
        do_actor = u % cfg.policy_delay == 0
        for lr, gen in zip(learners, gens):
            lr.update(gen, do_actor)
        torch.cuda.synchronize()
        pe = [p.detach() for p in learners[0].online + learners[0].target]
        pg = [p.detach() for p in learners[1].online + learners[1].target]
        for x, y in zip(pe, pg):
            d = float((x - y).abs().max()) / max(float(x.abs().max()), 1e-30)
            worst = max(worst, d)
            assert d <= 1e-6, (u, d)
    assert learners[1].graphs is not None
    print(f"graph vs eager updates: worst relative parameter difference {worst:.1e}")


def test_graph_training_loop_matches_eager_loop(td3):
    """A short run with the environment step and the learner replayed from
    captured graphs (re-captured after each curriculum round) against the
    same run with every step eager: the same replay contents, evaluation
    records and final policy, bit for bit."""
    import dataclasses
    t = td3
    base = t.TD3Config(total_steps=2500, n_envs=4, warmup=500, curriculum_every=1000,
                       eval_every=1000, eval_envs=64, eval_steps=100,
                       C_factor=dict(C_rp=1.5, C_ra=2.0), C_target=dict(C_rp=10.0, C_ra=1.0))
    outs = [t.train(dataclasses.replace(base, graph_updates=g, graph_env=g)) for g in (False, True)]
    (e, g) = outs
    for k in ("oa", "oc", "noa", "noc", "a", "r", "term", "s_next"):
        x, y = getattr(e["replay"], k), getattr(g["replay"], k)
        assert torch.equal(x, y), k
    assert torch.equal(e["actor"].flat(), g["actor"].flat())
    strip = lambda recs: [{kk: v for kk, v in r.items() if kk != "wall_s"} for r in recs]
    assert strip(e["records"]) == strip(g["records"])
    print("graph loop vs eager loop: replay, records and policy identical;",
          "wall", [r["wall_s"] for r in e["records"]][-1], "vs", [r["wall_s"] for r in g["records"]][-1])
