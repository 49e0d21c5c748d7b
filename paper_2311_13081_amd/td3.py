"""TD3 with the reward curriculum, trained on the batched quadrotor
environment in simulation: the training paradigm of Sec. IV and V (an
asymmetric actor-critic with TD3, Fujimoto et al. 2018; penalty weights of
the reward multiplied by fixed factors every 100 000 steps until they reach
their targets; the exploration noise decayed on the same schedule; every
reward in the replay buffer recomputed after each change of the reward).

The learner (networks, replay buffer, optimiser) is plain torch: it consumes
the environment.  Every environment step, observation, reward, reset and
re-scoring of stored transitions runs in the library's kernels through the C
ABI; the evaluation rollouts run the policy inside the fused step kernel
with the actor's weights in the library's flat layout.

    python -m paper_2311_13081_amd.td3 --steps 300000 --out curve.jsonl
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from dataclasses import asdict, dataclass, field

import torch
import torch.nn as nn

from .sim import QuadSim

REWARD_KEYS = QuadSim.REWARD_KEYS


@dataclass
class TD3Config:
    total_steps: int = 300_000     # environment interactions, all training envs together
    n_envs: int = 1                # training envs stepped together
    updates_per_env_step: float = 1.0
    warmup: int = 10_000           # uniform random actions before the first update
    batch: int = 256
    gamma: float = 0.99
    tau: float = 0.005
    lr_actor: float = 1e-4
    lr_critic: float = 1e-3
    policy_delay: int = 2
    target_noise: float = 0.2
    target_noise_clip: float = 0.5
    critic_hidden: int = 64
    # curriculum: every `curriculum_every` steps the penalty weights and the
    # exploration noise are multiplied by their factors, clamped at targets
    curriculum_every: int = 100_000
    C_factor: dict = field(default_factory=lambda: dict(C_rp=1.2, C_ra=1.4))
    C_target: dict = field(default_factory=lambda: dict(C_rp=2.0, C_ra=0.05))
    expl_noise: float = 0.5
    expl_factor: float = 0.8
    expl_target: float = 0.1
    recalc_rewards: bool = True
    # the learner's update replayed from two captured HIP graphs (critic
    # only; critic, actor and targets), and the environment step with its
    # bookkeeping from two more (the policy's action; the step, replay
    # insert, restarts and next observation); the same arithmetic as the
    # eager loop, whose random draws stay outside the graphs
    graph_updates: bool = True
    graph_env: bool = True
    eval_every: int = 10_000
    eval_envs: int = 256
    eval_steps: int = 500
    seed: int = 0


def curriculum(cfg: TD3Config, C_init: dict, step: int):
    """Reward constants and exploration noise in force at env step `step`:
    after k = step // curriculum_every rounds each scheduled constant is
    C_init * factor^k, clamped at its target (from below or above, whichever
    side the target lies on); the noise likewise."""
    k = step // cfg.curriculum_every
    C = dict(C_init)
    for name, f in cfg.C_factor.items():
        v = C_init[name] * f ** k
        tgt = cfg.C_target[name]
        C[name] = min(v, tgt) if f >= 1 else max(v, tgt)
    s = cfg.expl_noise * cfg.expl_factor ** k
    sigma = max(s, cfg.expl_target) if cfg.expl_factor <= 1 else min(s, cfg.expl_target)
    return C, sigma, k


class Actor(nn.Module):
    """146-64-64-4, ReLU, ReLU, tanh: the policy the step kernel evaluates."""

    def __init__(self):
        super().__init__()
        self.l1, self.l2, self.l3 = nn.Linear(146, 64), nn.Linear(64, 64), nn.Linear(64, 4)

    def forward(self, o):
        return torch.tanh(self.l3(torch.relu(self.l2(torch.relu(self.l1(o))))))

    def flat(self, out=None):
        """[W1 | b1 | W2 | b2 | W3 | b3] (torch Linear layouts), the flat
        actor vector of the C ABI."""
        parts = [self.l1.weight, self.l1.bias, self.l2.weight, self.l2.bias, self.l3.weight,
                 self.l3.bias]
        v = torch.cat([p.detach().reshape(-1) for p in parts])
        if out is None:
            return v.contiguous()
        out.copy_(v)
        return out


def critic_obs_scale(env_cfg: dict):
    """Affine map of the 28-value critic observation {p, R, v, w, rotor speeds,
    f_r, tau_r} to order-one inputs: rotor speeds to the action scale [-1, 1],
    the disturbance force and torque by their bounds; the rest as it is."""
    scale = torch.ones(28)
    shift = torch.zeros(28)
    span = float(env_cfg["rpm_max"]) - float(env_cfg["rpm_min"])
    scale[18:22] = 2.0 / span
    shift[18:22] = -1.0 - 2.0 * float(env_cfg["rpm_min"]) / span
    fb, tb = float(env_cfg.get("dist_force", 0.0)), float(env_cfg.get("dist_torque", 0.0))
    scale[22:25] = 1.0 / fb if fb > 0 else 1.0
    scale[25:28] = 1.0 / tb if tb > 0 else 1.0
    return scale, shift


class Critics(nn.Module):
    """Twin Q networks on the critic's privileged observation (28, scaled to
    order one) and the action (4), 32-h-h-1 with ReLU, evaluated together as
    batched products (weights stacked [2][in][out], initialised like torch
    Linear layers)."""

    def __init__(self, hidden, obs_scale=None):
        super().__init__()
        sc, sh = obs_scale if obs_scale is not None else (torch.ones(28), torch.zeros(28))
        self.register_buffer("obs_scale", sc.clone())
        self.register_buffer("obs_shift", sh.clone())
        dims = [(32, hidden), (hidden, hidden), (hidden, 1)]
        self.W = nn.ParameterList()
        self.b = nn.ParameterList()
        for fi, fo in dims:
            bound = 1.0 / math.sqrt(fi)
            self.W.append(nn.Parameter(torch.empty(2, fi, fo).uniform_(-bound, bound)))
            self.b.append(nn.Parameter(torch.empty(2, 1, fo).uniform_(-bound, bound)))

    def forward(self, oc, a):
        oc = oc * self.obs_scale + self.obs_shift
        x = torch.cat([oc, a], dim=1).unsqueeze(0).expand(2, -1, -1)
        for i in range(3):
            x = torch.baddbmm(self.b[i], x, self.W[i])
            if i < 2:
                x = torch.relu(x)
        return x[0, :, 0], x[1, :, 0]


class Replay:
    """Transitions on the device.  The post-step state and the action are kept
    in the [K][M] layout the reward call reads, so the whole buffer can be
    re-scored in one call."""

    def __init__(self, cap, dev):
        f = dict(dtype=torch.float32, device=dev)
        self.cap, self.size, self.pos = cap, 0, 0
        self.oa = torch.zeros(cap, 146, **f)
        self.oc = torch.zeros(cap, 28, **f)
        self.noa = torch.zeros(cap, 146, **f)
        self.noc = torch.zeros(cap, 28, **f)
        self.a = torch.zeros(cap, 4, **f)
        self.r = torch.zeros(cap, **f)
        self.term = torch.zeros(cap, **f)
        self.s_next = torch.zeros(17, cap, **f)   # post-step state, [17][cap]
        self.a_soa = torch.zeros(4, cap, **f)     # action, [4][cap]

    def add(self, oa, oc, a, r, noa, noc, term, s_next):
        n = oa.shape[0]
        idx = (torch.arange(n, device=oa.device) + self.pos) % self.cap
        self.oa[idx], self.oc[idx], self.noa[idx], self.noc[idx] = oa, oc, noa, noc
        self.a[idx], self.r[idx], self.term[idx] = a, r, term
        self.s_next[:, idx] = s_next
        self.a_soa[:, idx] = a.T
        self.pos = (self.pos + n) % self.cap
        self.size = min(self.size + n, self.cap)

    def add_at(self, pos, ar, oa, oc, a, r, noa, noc, term, s_next):
        """add() with the insert position in a device scalar (pos, advanced
        here) instead of on the host, so the insert can be replayed from a
        graph; ar: arange(n) on the device.  The host's size and pos are
        brought up to date by advance()."""
        idx = (ar + pos) % self.cap
        self.oa[idx], self.oc[idx], self.noa[idx], self.noc[idx] = oa, oc, noa, noc
        self.a[idx], self.r[idx], self.term[idx] = a, r, term
        self.s_next[:, idx] = s_next
        self.a_soa[:, idx] = a.T
        pos.add_(ar.shape[0]).remainder_(self.cap)

    def advance(self, n):
        self.pos = (self.pos + n) % self.cap
        self.size = min(self.size + n, self.cap)

    def sample(self, B, gen):
        i = torch.randint(0, self.size, (B,), device=self.oa.device, generator=gen)
        return self.oa[i], self.oc[i], self.a[i], self.r[i], self.noa[i], self.noc[i], self.term[i]


def training_env_config(n_envs, base=None):
    """The training MDP: terminate outside the box, truncate at 500 steps,
    disturbances and observation noise on, no in-step reset (the learner
    reads every post-step state, then restarts finished envs)."""
    import workloads as wl
    cfg = wl.training_extras(wl.crazyflie_config(n_envs=n_envs, max_episode_steps=500))
    cfg["flags"] = wl.F_RENORM_Q | wl.F_TERMINATE | wl.F_DISTURB | wl.F_OBS_NOISE
    if base:
        cfg.update(base)
    return cfg


def evaluate(ev: QuadSim, flat: torch.Tensor, steps: int, seed: int):
    """Deterministic policy from a fixed set of start states: per env the
    length of its first episode (first termination, else `steps`) and its
    return up to then."""
    ev.reset(seed=seed)
    out = ev.rollout(flat, steps, rewards=True, dones=True)
    d = out["dones"] != 0                                   # [T][N]
    T = d.shape[0]
    t_idx = torch.arange(T, device=d.device).unsqueeze(1).expand_as(d)
    first = torch.where(d, t_idx, torch.full_like(t_idx, T)).min(dim=0).values  # first done
    length = torch.clamp(first + 1, max=T)
    alive = t_idx <= first.unsqueeze(0)
    # after its first termination an env keeps flying without reset and may
    # leave the finite range: only rewards up to the termination count
    ret = torch.where(alive, out["rewards"], torch.zeros_like(out["rewards"])).sum(dim=0)
    return length.float(), ret


class Learner:
    """One TD3 update (Fujimoto et al.): twin critics regressed on the
    clipped double-Q target with target-policy smoothing, and every
    `policy_delay`-th update the actor step and the Polyak update of the
    targets.  The batch indices and the smoothing noise are drawn outside
    the update (idx, eps), so the same update runs eagerly or replayed from
    a captured graph with identical random streams.  With graphs, the
    update's kernels are captured once per variant (critic only; critic,
    actor and targets) after two eager warm-up updates whose effect on the
    parameters and optimiser states is undone before the capture."""

    def __init__(self, cfg, actor, critics, actor_t, critics_t, buf, dev):
        self.cfg, self.buf = cfg, buf
        self.actor, self.critics, self.actor_t, self.critics_t = actor, critics, actor_t, critics_t
        self.opt_a = torch.optim.Adam(actor.parameters(), lr=cfg.lr_actor, capturable=True)
        self.opt_c = torch.optim.Adam(critics.parameters(), lr=cfg.lr_critic, capturable=True)
        self.online = list(actor.parameters()) + list(critics.parameters())
        self.target = list(actor_t.parameters()) + list(critics_t.parameters())
        self.idx = torch.zeros(cfg.batch, dtype=torch.long, device=dev)
        self.eps = torch.zeros(cfg.batch, 4, device=dev)
        self.graphs = None

    def draw(self, gen):
        """The batch indices and the target-policy noise of one update."""
        torch.randint(0, self.buf.size, (self.cfg.batch,), device=self.idx.device, generator=gen,
                      out=self.idx)
        torch.randn(self.eps.shape, device=self.eps.device, generator=gen, out=self.eps)

    def _update(self, do_actor):
        cfg, b = self.cfg, self.buf
        i = self.idx
        boa, boc, ba, br, bnoa, bnoc, bterm = (b.oa[i], b.oc[i], b.a[i], b.r[i], b.noa[i],
                                               b.noc[i], b.term[i])
        with torch.no_grad():
            eps = (self.eps * cfg.target_noise).clamp(-cfg.target_noise_clip,
                                                     cfg.target_noise_clip)
            na = (self.actor_t(bnoa) + eps).clamp(-1.0, 1.0)
            q1t, q2t = self.critics_t(bnoc, na)
            y = br + cfg.gamma * (1.0 - bterm) * torch.minimum(q1t, q2t)
        q1, q2 = self.critics(boc, ba)
        loss_c = ((q1 - y) ** 2).mean() + ((q2 - y) ** 2).mean()
        self.opt_c.zero_grad(set_to_none=True)
        loss_c.backward()
        self.opt_c.step()
        if do_actor:
            q, _ = self.critics(boc, self.actor(boa))
            loss_a = -q.mean()
            self.opt_a.zero_grad(set_to_none=True)
            loss_a.backward()
            self.opt_a.step()
            with torch.no_grad():
                torch._foreach_lerp_(self.target, self.online, cfg.tau)

    def _state(self):
        ts = self.online + self.target
        for opt in (self.opt_a, self.opt_c):
            for st in opt.state.values():
                ts += [v for v in st.values() if torch.is_tensor(v)]
        return ts

    def _capture(self):
        state = self._state()
        saved = [t.detach().clone() for t in state]
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for do_actor in (False, True, False, True):
                self._update(do_actor)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        with torch.no_grad():
            for t, v in zip(state, saved):
                t.copy_(v)
            # optimiser states the warm-up created (the actor's, when the
            # first update was a critic update) go back to Adam's initial
            # state: zero moments, zero steps
            known = {id(t) for t in state}
            for t in self._state():
                if id(t) not in known:
                    t.zero_()
        self.graphs = {}
        for do_actor in (False, True):
            g = torch.cuda.CUDAGraph()
            self.opt_a.zero_grad(set_to_none=True)
            self.opt_c.zero_grad(set_to_none=True)
            with torch.cuda.graph(g):
                self._update(do_actor)
            self.graphs[do_actor] = g
        torch.cuda.synchronize()

    def update(self, gen, do_actor):
        self.draw(gen)
        if not self.cfg.graph_updates:
            self._update(do_actor)
            return
        if self.graphs is None:
            # the first update runs eagerly (it creates the optimiser
            # states), the later ones replay the graphs
            self._update(do_actor)
            self._capture()
            return
        self.graphs[do_actor].replay()


class EnvLoop:
    """The training env's side of one TD3 step: the action (uniform during
    the warm-up, else the policy plus Gaussian exploration noise, clipped),
    the step, the post-step observations and state into the replay buffer,
    the restart of finished envs, the episode statistics and the next
    observation.  With graphs, the policy's action and the rest are replayed
    from two captured graphs (the noise drawn outside them); the step's
    graph is captured again after each change of the reward constants, which
    the step launches take by value."""

    def __init__(self, sim, buf, actor, N, dev, graph):
        self.sim, self.buf, self.actor, self.N, self.graph = sim, buf, actor, N, graph
        self.a = torch.zeros(N, 4, device=dev)
        self.u = torch.zeros(N, 4, device=dev)
        self.sigma = torch.zeros((), device=dev)
        o = sim.observe()
        self.oa, self.oc = o["actor"].T.contiguous(), o["critic"].T.contiguous()
        self.ep_len_sum = torch.zeros((), device=dev)
        self.ep_count = torch.zeros((), device=dev)
        self.pos = torch.zeros((), dtype=torch.long, device=dev)
        self.ar = torch.arange(N, device=dev)
        self.g_act = self.g_step = None
        self.steps = self.act_steps = 0

    def _act(self):
        with torch.no_grad():
            self.a.copy_((self.actor(self.oa) + self.sigma * self.u).clamp(-1.0, 1.0))

    def _step(self):
        sim, buf = self.sim, self.buf
        r, d = sim.step(actions=self.a.T.contiguous())
        no = sim.observe()
        s_next = sim.get_state(parts=("state",))["state"]
        term = (d & 1).float()
        buf.add_at(self.pos, self.ar, self.oa, self.oc, self.a, r, no["actor"].T,
                   no["critic"].T, term, s_next)
        done = d != 0
        sim.reset_envs(done)
        st = sim.get_state(parts=("last_len",))
        self.ep_len_sum += (st["last_len"].float() * done).sum()
        self.ep_count += done.sum()
        o = sim.observe()
        self.oa.copy_(o["actor"].T)
        self.oc.copy_(o["critic"].T)

    def constants_changed(self):
        self.g_step = None

    def _capture(self, fn):
        # the loop's own eager steps before the first capture initialise
        # every library the captured work uses
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            fn()
        return g

    def run(self, gen, warm, sigma):
        """One step: warm = uniform actions; sigma = exploration noise."""
        if warm:
            torch.rand(self.a.shape, device=self.a.device, generator=gen, out=self.u)
            torch.sub(self.u * 2, 1, out=self.a)
        else:
            torch.randn(self.u.shape, device=self.u.device, generator=gen, out=self.u)
            self.sigma.fill_(sigma)
            if self.graph and self.act_steps >= 2:
                if self.g_act is None:
                    self.g_act = self._capture(self._act)
                self.g_act.replay()
            else:
                self._act()
            self.act_steps += 1
        if self.graph and self.steps >= 2:
            if self.g_step is None:
                self.g_step = self._capture(self._step)
            self.g_step.replay()
        else:
            self._step()
        self.buf.advance(self.N)
        self.steps += 1


def train(cfg: TD3Config, log=None, env_overrides=None, stop_after=None):
    """Runs TD3 with the curriculum.  log: callable receiving each evaluation
    record (dict) as it is made; stop_after(record) -> True ends the run.
    Returns dict(records, actor, replay, C (constants in force at the end),
    env_cfg)."""
    dev = torch.device("cuda")
    torch.manual_seed(cfg.seed)
    gen = torch.Generator(device=dev).manual_seed(cfg.seed)
    env_cfg = training_env_config(cfg.n_envs, env_overrides)
    env_cfg["seed"] = 1000 + cfg.seed
    sim = QuadSim(env_cfg)
    ev_cfg = dict(env_cfg, n_envs=cfg.eval_envs, seed=7)
    ev = QuadSim(ev_cfg)
    C_init = {k: float(env_cfg[k]) for k in REWARD_KEYS}
    osc = critic_obs_scale(env_cfg)
    actor, critics = Actor().to(dev), Critics(cfg.critic_hidden, osc).to(dev)
    actor_t, critics_t = Actor().to(dev), Critics(cfg.critic_hidden, osc).to(dev)
    actor_t.load_state_dict(actor.state_dict())
    critics_t.load_state_dict(critics.state_dict())
    for p in list(actor_t.parameters()) + list(critics_t.parameters()):
        p.requires_grad_(False)
    buf = Replay(cfg.total_steps, dev)
    learner = Learner(cfg, actor, critics, actor_t, critics_t, buf, dev)
    flat = torch.empty(13828, dtype=torch.float32, device=dev)
    records = []
    N = cfg.n_envs
    env = EnvLoop(sim, buf, actor, N, dev, cfg.graph_env)
    stage = 0
    sigma = cfg.expl_noise
    n_updates = 0
    update_credit = 0.0
    t0 = time.perf_counter()
    step = 0
    while step < cfg.total_steps:
        # curriculum: new constants (and noise) every curriculum_every steps
        C, sigma, k = curriculum(cfg, C_init, step)
        if k != stage:
            stage = k
            sim.set_reward(**C)
            ev.set_reward(**C)
            env.constants_changed()
            if cfg.recalc_rewards and buf.size:
                sim.reward(buf.s_next, buf.a_soa, out=buf.r)
        env.run(gen, step < cfg.warmup, sigma)
        step += N
        # TD3 updates
        if step >= cfg.warmup:
            update_credit += N * cfg.updates_per_env_step
            while update_credit >= 1.0:
                update_credit -= 1.0
                n_updates += 1
                learner.update(gen, n_updates % cfg.policy_delay == 0)
        if step % cfg.eval_every < N or step >= cfg.total_steps:
            length, ret = evaluate(ev, actor.flat(flat), cfg.eval_steps, seed=7)
            rec = dict(step=step, eval_len_mean=float(length.mean()),
                       eval_len_std=float(length.std()), eval_ret_mean=float(ret.mean()),
                       eval_fly_frac=float((length >= cfg.eval_steps).float().mean()),
                       train_episodes=int(env.ep_count),
                       train_len_mean=float(env.ep_len_sum / env.ep_count.clamp(min=1)),
                       updates=n_updates, sigma=sigma, stage=stage,
                       C={kk: C[kk] for kk in cfg.C_factor}, wall_s=time.perf_counter() - t0)
            env.ep_len_sum.zero_()
            env.ep_count.zero_()
            records.append(rec)
            if log:
                log(rec)
            if stop_after is not None and stop_after(rec):
                break
    sim.close()
    ev.close()
    return dict(records=records, actor=actor, replay=buf, C=C, env_cfg=env_cfg)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--steps", type=int, default=300_000)
    ap.add_argument("--n-envs", type=int, default=1)
    ap.add_argument("--updates-per-env-step", type=float, default=1.0)
    ap.add_argument("--eval-every", type=int, default=10_000)
    ap.add_argument("--warmup", type=int, default=10_000)
    ap.add_argument("--critic-hidden", type=int, default=64)
    ap.add_argument("--no-recalc", action="store_true")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=None, help="JSON lines of the evaluation records")
    ap.add_argument("--save", default=None, help="file for the trained actor's flat parameters")
    ap.add_argument("--track", action="store_true",
                    help="after training, the Lissajous tracking errors of the trained actor")
    a = ap.parse_args(argv)
    cfg = TD3Config(total_steps=a.steps, n_envs=a.n_envs,
                    updates_per_env_step=a.updates_per_env_step, eval_every=a.eval_every,
                    warmup=a.warmup, critic_hidden=a.critic_hidden,
                    recalc_rewards=not a.no_recalc, seed=a.seed)
    fh = open(a.out, "w") if a.out else None

    def log(rec):
        line = json.dumps(rec)
        print(line, flush=True)
        if fh:
            fh.write(line + "\n")
            fh.flush()
    print(json.dumps({"config": asdict(cfg)}), flush=True)
    res = train(cfg, log)
    flat = res["actor"].flat().detach()
    if a.save:
        torch.save(flat.cpu(), a.save)
    if a.track:
        from .tracking import tracking_table
        log({"tracking": tracking_table(flat, res["env_cfg"])})
    if fh:
        fh.close()


if __name__ == "__main__":
    sys.exit(main())
