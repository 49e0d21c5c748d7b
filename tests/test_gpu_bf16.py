"""bf16 actor option (SIM_F_ACTOR_BF16) against the FP64 oracle.

The option trades precision for speed, so it is held to three checks:
  1. the kernel computes what the bf16 arithmetic defines: a CPU emulation
     (weights and every layer input rounded to bf16 with round-to-nearest-
     even, products and sums in FP64, activations from the oracle's FP64
     observation) agrees with the GPU's applied actions to fp32 accumulation
     noise, except where an input sits next to a bf16 rounding tie and the
     two sides round it to neighbouring values (one bf16 ulp, 2^-8 relative,
     of one term);
  2. the rest of the step is the fp32 step: the oracle driven by the action
     the GPU applied matches the GPU's next state at the fp32 step tolerance;
  3. the error against the FP64 oracle -- actions, and gradients through a
     bf16 rollout next to the fp32 ones -- is reported (and bounded loosely:
     same descent direction, errors of the order bf16 rounding predicts).
"""
import numpy as np
import pytest

import workloads as wl
from parity import STEP_TOL, max_state_err, state_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U_BF16 = 2.0 ** -8


@pytest.fixture(scope="module")
def pkg():
    import paper_2311_13081_amd as p
    p.load()
    return p


def np_(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def unpack(W):
    W = np.asarray(W, np.float64)
    o = 0
    out = []
    for shape in ((64, 146), (64,), (64, 64), (64,), (4, 64), (4,)):
        n = int(np.prod(shape))
        out.append(W[o:o + n].reshape(shape))
        o += n
    return out


def bf16_round(x):
    """Round to the nearest bf16 value (ties to even), via float32."""
    b = np.asarray(x, np.float64).astype(np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_actor(W, o):
    """The bf16 actor's arithmetic: rounded weights and inputs, exact sums."""
    W1, b1, W2, b2, W3, b3 = (bf16_round(w) if i % 2 == 0 else w
                              for i, w in enumerate(unpack(W)))
    h1 = np.maximum(W1 @ bf16_round(o) + b1, 0.0)
    h2 = np.maximum(W2 @ bf16_round(h1) + b2, 0.0)
    return np.tanh(W3 @ bf16_round(h2) + b3)


def test_bf16_config_rules(pkg):
    from paper_2311_13081_amd import SimError
    cfg = wl.crazyflie_config(n_envs=64, flags=wl.F_RENORM_Q | wl.F_ACTOR_BF16 | wl.F_FP64)
    with pytest.raises(SimError) as ei:
        pkg.QuadSim(cfg)
    assert ei.value.code == -1
    cfg = wl.crazyflie_config(n_envs=64, flags=wl.F_RENORM_Q | wl.F_ACTOR_BF16)
    sim = pkg.QuadSim(cfg)
    assert sim.get_variant()[0] == pkg.SIM_V_FUSED_MFMA4
    for v in (pkg.SIM_V_FUSED_VALU, pkg.SIM_V_PLAIN, pkg.SIM_V_FUSED_SPLIT):
        with pytest.raises(SimError) as ei:
            sim.set_variant(v)
        assert ei.value.code == -5
    sim.set_variant(pkg.SIM_V_FUSED_MFMA)
    assert sim.get_variant()[0] == pkg.SIM_V_FUSED_MFMA
    sim.close()


@pytest.mark.parametrize("variant", ["mfma4", "mfma"])
def test_bf16_one_step_matches_bf16_arithmetic(pkg, oracle_lib, variant):
    """Both matrix-core kernels (quarter-lane: 16x16x32 bf16 products; one
    env per lane: 4-block 16x16x4 and 16x16x32 bf16 products, fp32 4x4x1 on
    rounded inputs for layer 3) against the emulated bf16 arithmetic."""
    n = 1000
    cfg = wl.crazyflie_config(n_envs=n, dr_enable=1, max_episode_steps=0,
                              flags=wl.F_RENORM_Q | wl.F_ACTOR_BF16)
    sim = pkg.QuadSim(cfg)
    sim.set_variant({"mfma4": pkg.SIM_V_FUSED_MFMA4, "mfma": pkg.SIM_V_FUSED_MFMA}[variant])
    W = wl.random_actor(3)
    s, h = wl.random_states(n, seed=77)
    sim.set_state(state=s, hist=h)
    th = np_(sim.get_params())
    sim.step(actor=sim.actor_tensor(W))
    st = {k: np_(v) for k, v in sim.get_state().items()}
    a_gpu = st["hist"][31].T.astype(np.float64)          # newest slot = applied action
    obs = [oracle_lib.observe(s[:, e].astype(np.float64),
                              np.transpose(h, (2, 0, 1))[e].astype(np.float64))
           for e in range(n)]
    a_emu = np.array([bf16_actor(W, o) for o in obs])
    a_ref = np.array([oracle_lib.actor(W, o) for o in obs])
    d_emu = np.abs(a_gpu - a_emu).max(axis=1)
    d_ref = np.abs(a_gpu - a_ref).max(axis=1)
    q = lambda d: {p_: float(np.quantile(d, p_)) for p_ in (0.5, 0.9, 0.99, 1.0)}
    print(f"bf16 vs emulated bf16 arithmetic, per-env max |da| quantiles {q(d_emu)}")
    print(f"bf16 vs FP64 oracle, per-env max |da| quantiles {q(d_ref)}")
    # 1. agreement with the bf16 arithmetic: most envs to accumulation noise,
    #    the rest within a few tie flips (each <= 2^-8 |w x| <~ 1e-3 at the
    #    output)
    assert np.quantile(d_emu, 0.99) < 1e-6
    assert d_emu.max() < 1e-2
    # 3. against FP64: of the order of bf16 rounding, and really rounded
    assert d_ref.max() < 0.1 and np.quantile(d_ref, 0.5) > 1e-4
    # 2. the dynamics after the actor: fp32 step tolerance
    ref = oracle_lib.Batch(cfg, n)
    ref.set_soa(s, h, theta_soa=th)
    ref.rollout(None, 1, actions=a_gpu[None].astype(np.float32).astype(np.float64))
    assert max_state_err(st["state"], ref.s) < STEP_TOL
    sim.close()


def test_bf16_taped_equals_untaped_and_resumes(pkg):
    """Taped and untaped bf16 rollouts run the same code: bitwise equal."""
    n, T = 200, 24
    cfg = wl.crazyflie_config(n_envs=n, flags=wl.F_RENORM_Q | wl.F_ACTOR_BF16, max_episode_steps=0,
                              max_tape_horizon=T, ckpt_every=8)
    sim = pkg.QuadSim(cfg)
    a = sim.actor_tensor(wl.random_actor(5))
    snap = {k: v.clone() for k, v in sim.get_state().items()}
    S1 = np_(sim.rollout(a, T, states=True, record_tape=True)["states"])
    sim.set_state(**snap)
    S2 = np_(sim.rollout(a, T, states=True)["states"])
    assert np.array_equal(S1, S2)
    sim.close()


def grads(pkg, orc, flags, W, n=128, T=32, K=8):
    cfg = wl.crazyflie_config(n_envs=n, flags=flags, dr_enable=1, max_episode_steps=0,
                              max_tape_horizon=T, ckpt_every=K)
    ob = orc.Batch.init(cfg, n)
    s32, h32 = (x.astype(np.float32) for x in ob.soa())
    sim = pkg.QuadSim(cfg)
    sim.set_state(state=s32, hist=h32)
    th = np_(sim.get_params())
    a = sim.actor_tensor(W)
    sim.rollout(a, T, rewards=True, dones=False, record_tape=True)
    ga, gp = sim.backward(a)
    ga, gp = np_(ga).astype(np.float64), np_(gp).astype(np.float64).T
    sim.close()
    ref = orc.Batch(cfg, n)
    ref.set_soa(s32, h32, theta_soa=th)
    _, gW, gth = ref.grad(W, T, nthreads=8)
    ea = np.linalg.norm(ga - gW) / np.linalg.norm(gW)
    ep = np.linalg.norm(gp - gth, axis=1) / np.linalg.norm(gth, axis=1)
    cos = float(ga @ gW / (np.linalg.norm(ga) * np.linalg.norm(gW)))
    return ea, ep, cos


def test_bf16_gradients_reported_against_fp64(pkg, oracle_lib):
    W = wl.sysid_actor(0)
    res = {}
    for name, flags in (("fp32", wl.F_RENORM_Q), ("bf16", wl.F_RENORM_Q | wl.F_ACTOR_BF16)):
        ea, ep, cos = grads(pkg, oracle_lib, flags, W)
        res[name] = (ea, float(np.median(ep)), float(ep.max()), cos)
        print(f"{name} actor: d(sum r) gradient rel err {ea:.3e} (cosine {cos:.6f}); "
              f"params rel err median {np.median(ep):.3e} max {ep.max():.3e}")
    assert res["fp32"][0] < 1e-3
    assert res["bf16"][3] > 0.99      # same descent direction
    assert res["bf16"][0] > res["fp32"][0]


def test_bf16_one_lane_rollout_tracks_quarter_lane(pkg):
    """Long rollouts of the two bf16 kernels (different summation orders of
    the same bf16 products) with resets: done flags mostly equal, states close
    while episodes agree."""
    n, T = 512, 60
    flags = wl.F_RENORM_Q | wl.F_ACTOR_BF16 | wl.F_TERMINATE | wl.F_AUTORESET
    cfg = wl.crazyflie_config(n_envs=n, dr_enable=1, flags=flags, max_episode_steps=25)
    W = wl.random_actor(11)
    res = {}
    for v in ("mfma4", "mfma"):
        sim = pkg.QuadSim(cfg)
        sim.set_variant({"mfma4": pkg.SIM_V_FUSED_MFMA4, "mfma": pkg.SIM_V_FUSED_MFMA}[v])
        out = sim.rollout(sim.actor_tensor(W), T, rewards=True, dones=True, states=True)
        res[v] = {k: np_(x) for k, x in out.items()}
        sim.close()
    same = (res["mfma4"]["dones"] == res["mfma"]["dones"]).mean()
    assert same > 0.99, same
    # R16 norm (relative, with per-group floors) over the first steps, on the
    # envs whose done flags agree there
    ok = (res["mfma4"]["dones"][:5] == res["mfma"]["dones"][:5]).all(axis=0)
    assert ok.mean() > 0.98
    d = state_err(res["mfma"]["states"][1:6][:, :, ok],
                  np.transpose(res["mfma4"]["states"][1:6][:, :, ok], (0, 2, 1))).max()
    print("one-lane vs quarter-lane bf16, steps 1..5, R16 norm", d)
    assert d < 1e-4, d
