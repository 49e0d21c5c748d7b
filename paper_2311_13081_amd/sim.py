"""QuadSim: Python handle over the C ABI.  Tensors are passed by device pointer
with torch's current HIP stream; torch only supplies memory and streams."""
from __future__ import annotations

import ctypes
import json
import os

import torch

from . import _lib
from ._lib import check


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class QuadSim:
    """N quadrotor envs on one GPU.  cfg: dict with the sim_config fields (see
    workloads.crazyflie_config)."""

    def __init__(self, cfg: dict, device: int = 0):
        self.L = _lib.load()
        self.cfg = dict(cfg)
        self.N = int(cfg["n_envs"])
        self.device = torch.device("cuda", device)
        c = _lib.make_config(cfg)
        h = ctypes.c_void_p()
        check(self.L.sim_create(ctypes.byref(c), device, ctypes.byref(h)), "sim_create")
        self.h = h
        # Mirror of the handle's tape: the horizon of the last taped rollout
        # (0 once a call has dropped the tape, as the library does) and a
        # count of taped rollouts, so that a backward can tell which tape it
        # would differentiate and size-check its cotangents against it.
        self.tape_T = 0
        self.tape_gen = 0

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            check(self.L.sim_destroy(self.h), "sim_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- buffers ------------------------------------------------------------
    def _f32(self, *shape):
        return torch.empty(*shape, dtype=torch.float32, device=self.device)

    def _need(self, t, shape, dtype, name):
        """The library takes plain pointers: refuse a tensor it would read or
        write out of bounds."""
        if t is None:
            return
        if (t.dtype != dtype or not t.is_contiguous() or t.device.type != "cuda"
                or tuple(t.shape) != tuple(shape)):
            raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor of shape "
                             f"{tuple(shape)}, got {tuple(t.shape)} {t.dtype} on {t.device}")

    def actor_tensor(self, w) -> torch.Tensor:
        t = torch.as_tensor(w, dtype=torch.float32).to(self.device).contiguous()
        if t.numel() != _lib.SIM_NACTOR:
            raise ValueError(f"actor must have {_lib.SIM_NACTOR} parameters")
        return t

    # -- calls ----------------------------------------------------------------
    def reset(self, seed: int | None = None):
        s = self.cfg["seed"] if seed is None else seed
        check(self.L.sim_reset(self.h, ctypes.c_uint64(s), _stream()), "sim_reset")
        self.tape_T = 0

    def step(self, actor: torch.Tensor | None = None, actions: torch.Tensor | None = None):
        """One step; returns (reward [N], done [N] uint8)."""
        self._need(actor, (_lib.SIM_NACTOR,), torch.float32, "actor")
        self._need(actions, (4, self.N), torch.float32, "actions")
        r = self._f32(self.N)
        d = torch.empty(self.N, dtype=torch.uint8, device=self.device)
        check(self.L.sim_step(self.h, _ptr(actor), _ptr(actions), _ptr(r), _ptr(d), _stream()),
              "sim_step")
        self.tape_T = 0
        return r, d

    def rollout(self, actor: torch.Tensor, T: int, rewards=True, dones=True, states=False,
                record_tape=False, out=None):
        """T steps.  Returns dict with rewards [T][N], dones [T][N], states
        [T+1][17][N] (each only when requested).  out= reuses tensors."""
        out = {} if out is None else out
        n = max(int(T), 0)  # the library rejects T < 1 itself
        self._need(actor, (_lib.SIM_NACTOR,), torch.float32, "actor")
        for k, shape, dt in (("rewards", (n, self.N), torch.float32),
                             ("dones", (n, self.N), torch.uint8),
                             ("states", (n + 1, 17, self.N), torch.float32)):
            self._need(out.get(k), shape, dt, k)
        if rewards and "rewards" not in out:
            out["rewards"] = self._f32(n, self.N)
        if dones and "dones" not in out:
            out["dones"] = torch.empty(n, self.N, dtype=torch.uint8, device=self.device)
        if states and "states" not in out:
            out["states"] = self._f32(n + 1, 17, self.N)
        check(self.L.sim_rollout(self.h, _ptr(actor), T, _ptr(out.get("rewards")),
                                 _ptr(out.get("dones")), _ptr(out.get("states")),
                                 1 if record_tape else 0, _stream()), "sim_rollout")
        self.tape_T = int(T) if record_tape else 0
        if record_tape:
            self.tape_gen += 1
        return out

    def observe(self, actor=True, critic=True):
        """Current observations: actor [146][N] (with the coming step's noise)
        and critic [28][N] {p, R, v, w, rotor speeds, f_r, tau_r}."""
        out = {}
        if actor:
            out["actor"] = self._f32(146, self.N)
        if critic:
            out["critic"] = self._f32(28, self.N)
        check(self.L.sim_observe(self.h, _ptr(out.get("actor")), _ptr(out.get("critic")),
                                 _stream()), "sim_observe")
        return out

    def rollout_actions(self, actions: torch.Tensor, T: int, rewards=True, dones=True,
                        states=False):
        """Dynamics-only rollout: actions [4][N] held constant, or [T][4][N]."""
        per_step = actions.dim() == 3
        n = max(int(T), 0)  # the library rejects T < 1 itself
        want = (n, 4, self.N) if per_step else (4, self.N)
        if (actions.dtype != torch.float32 or not actions.is_contiguous()
                or tuple(actions.shape[-2:]) != want[-2:]
                or (per_step and actions.shape[0] < n)):
            raise ValueError(f"actions must be contiguous float32 [4][N] or [>=T][4][N], "
                             f"got {tuple(actions.shape)} {actions.dtype} for T={T}, N={self.N}")
        out = {}
        if rewards:
            out["rewards"] = self._f32(n, self.N)
        if dones:
            out["dones"] = torch.empty(n, self.N, dtype=torch.uint8, device=self.device)
        if states:
            out["states"] = self._f32(n + 1, 17, self.N)
        check(self.L.sim_rollout_actions(self.h, _ptr(actions), 1 if per_step else 0, T,
                                         _ptr(out.get("rewards")), _ptr(out.get("dones")),
                                         _ptr(out.get("states")), _stream()),
              "sim_rollout_actions")
        self.tape_T = 0
        return out

    def backward(self, actor: torch.Tensor, d_rewards=None, d_states=None, want_actor=True,
                 want_params=True, out=None, noalloc=False):
        """Gradients of the last taped rollout: (grad_actor [13828], grad_params
        [8][N]) for the loss sum d_rewards * rewards + sum d_states * states
        (d_rewards None = all ones, d_states None = zeros).  out=(ga, gp)
        reuses output tensors; noalloc=True runs sim_backward_noalloc (the
        library's static scratch array instead of the handle's buffers)."""
        self._need(actor, (_lib.SIM_NACTOR,), torch.float32, "actor")
        T = self.tape_T
        if T > 0:
            self._need(d_rewards, (T, self.N), torch.float32, "d_rewards")
            self._need(d_states, (T + 1, 17, self.N), torch.float32, "d_states")
        # without a tape the library refuses the call (SIM_E_STATE) before it
        # reads any argument
        if out is not None:
            ga, gp = out
            self._need(ga, (_lib.SIM_NACTOR,), torch.float32, "grad_actor")
            self._need(gp, (8, self.N), torch.float32, "grad_params")
        else:
            ga = torch.empty(_lib.SIM_NACTOR, dtype=torch.float32,
                             device=self.device) if want_actor else None
            gp = self._f32(8, self.N) if want_params else None
        fn = self.L.sim_backward_noalloc if noalloc else self.L.sim_backward
        check(fn(self.h, _ptr(actor), _ptr(d_rewards), _ptr(d_states), _ptr(ga), _ptr(gp),
                 _stream()), "sim_backward_noalloc" if noalloc else "sim_backward")
        return ga, gp

    def get_state(self, parts=None):
        """Snapshot: state [17][N], hist [32][4][N], t_ep [N], episode [N],
        returns [2][N] (current episode so far, last finished episode) and
        last_len [N] (steps of the last finished episode).  parts: the keys
        to fetch (default all)."""
        want = set(parts) if parts is not None else {"state", "hist", "t_ep", "episode",
                                                      "returns", "last_len"}
        i32 = dict(dtype=torch.int32, device=self.device)
        out = {}
        if "state" in want:
            out["state"] = self._f32(17, self.N)
        if "hist" in want:
            out["hist"] = self._f32(32, 4, self.N)
        if "t_ep" in want:
            out["t_ep"] = torch.empty(self.N, **i32)
        if "episode" in want:
            out["episode"] = torch.empty(self.N, **i32)
        if "returns" in want:
            out["returns"] = self._f32(2, self.N)
        if "last_len" in want:
            out["last_len"] = torch.empty(self.N, **i32)
        g = out.get
        check(self.L.sim_get_state(self.h, _ptr(g("state")), _ptr(g("hist")), _ptr(g("t_ep")),
                                   _ptr(g("episode")), _ptr(g("returns")), _ptr(g("last_len")),
                                   _stream()), "sim_get_state")
        return out

    def set_state(self, state=None, hist=None, t_ep=None, episode=None, returns=None,
                  last_len=None):
        def dev(x, dt):
            return None if x is None else torch.as_tensor(x, dtype=dt).to(self.device).contiguous()
        s, h = dev(state, torch.float32), dev(hist, torch.float32)
        t, e = dev(t_ep, torch.int32), dev(episode, torch.int32)
        r, ln = dev(returns, torch.float32), dev(last_len, torch.int32)
        self._need(s, (17, self.N), torch.float32, "state")
        self._need(h, (32, 4, self.N), torch.float32, "hist")
        self._need(t, (self.N,), torch.int32, "t_ep")
        self._need(e, (self.N,), torch.int32, "episode")
        self._need(r, (2, self.N), torch.float32, "returns")
        self._need(ln, (self.N,), torch.int32, "last_len")
        check(self.L.sim_set_state(self.h, _ptr(s), _ptr(h), _ptr(t), _ptr(e), _ptr(r), _ptr(ln),
                                   _stream()), "sim_set_state")
        self.tape_T = 0

    REWARD_KEYS = ("C_rp", "C_rq", "C_rv", "C_rw", "C_ra", "C_rab", "C_rs")

    def set_reward(self, **constants):
        """Replaces reward constants (any of REWARD_KEYS) for the steps that
        follow, without touching the envs."""
        unknown = set(constants) - set(self.REWARD_KEYS)
        if unknown:
            raise ValueError(f"unknown reward constants {sorted(unknown)}")
        self.cfg.update({k: float(v) for k, v in constants.items()})
        C = (ctypes.c_double * 7)(*[float(self.cfg[k]) for k in self.REWARD_KEYS])
        check(self.L.sim_set_reward(self.h, C), "sim_set_reward")

    def set_target(self, target=None, pos_clip: float = 0.2, vel_clip: float = 1.0):
        """Set point of the actor's observation: target [6][N] = {p_sp, v_sp}
        per env (None removes it); the actor then observes the clipped
        position and velocity errors."""
        t = None
        if target is not None:
            t = torch.as_tensor(target, dtype=torch.float32).to(self.device).contiguous()
            self._need(t, (6, self.N), torch.float32, "target")
        check(self.L.sim_set_target(self.h, _ptr(t), float(pos_clip), float(vel_clip), _stream()),
              "sim_set_target")
        self.tape_T = 0

    def reset_envs(self, mask: torch.Tensor):
        """Starts the next episode of every env with mask != 0 (uint8 or bool
        [N]), as an in-step reset would."""
        m = mask.to(device=self.device, dtype=torch.uint8).contiguous()
        self._need(m, (self.N,), torch.uint8, "mask")
        check(self.L.sim_reset_envs(self.h, _ptr(m), _stream()), "sim_reset_envs")
        self.tape_T = 0

    def reward(self, states: torch.Tensor, actions: torch.Tensor, out=None):
        """Rewards r(s', a) of M transitions, states [17][M] and actions
        [4][M], under the current reward constants."""
        M = int(states.shape[-1]) if states.dim() == 2 else -1
        self._need(states, (17, M), torch.float32, "states")
        self._need(actions, (4, M), torch.float32, "actions")
        r = self._f32(M) if out is None else out
        self._need(r, (M,), torch.float32, "out")
        check(self.L.sim_reward(self.h, _ptr(states), _ptr(actions), M, _ptr(r), _stream()),
              "sim_reward")
        return r

    def get_params(self):
        th = self._f32(8, self.N)
        check(self.L.sim_get_params(self.h, _ptr(th), _stream()), "sim_get_params")
        return th

    def set_params(self, theta):
        th = torch.as_tensor(theta, dtype=torch.float32).to(self.device).contiguous()
        self._need(th, (8, self.N), torch.float32, "theta")
        check(self.L.sim_set_params(self.h, _ptr(th), _stream()), "sim_set_params")
        self.tape_T = 0

    def set_variant(self, variant: int, steps_per_launch: int = 0, use_graph: bool = True):
        check(self.L.sim_set_variant(self.h, variant, steps_per_launch, 1 if use_graph else 0),
              "sim_set_variant")

    def get_variant(self):
        v, s, g = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        check(self.L.sim_get_variant(self.h, ctypes.byref(v), ctypes.byref(s), ctypes.byref(g)),
              "sim_get_variant")
        return v.value, s.value, g.value

    def autotune(self, actor: torch.Tensor, T: int, cache: str | None = None):
        """Times the variants on a T-step rollout and keeps the fastest.  With
        `cache` (a JSON file path), a result stored for the same (N, flags, T,
        device architecture) is reused instead of timing again, and new
        results are added to the file."""
        key = None
        if cache is not None:
            arch = torch.cuda.get_device_properties(self.device).gcnArchName.split(":")[0]
            key = f"N={self.N} flags={int(self.cfg['flags'])} T={int(T)} arch={arch}"
            table = {}
            if os.path.exists(cache):
                with open(cache) as f:
                    table = json.load(f)
            hit = table.get(key)
            if hit is not None:
                self.set_variant(int(hit["variant"]), int(hit["steps_per_launch"]), True)
                return int(hit["variant"]), float(hit["ms"])
        v, ms = ctypes.c_int(), ctypes.c_float()
        check(self.L.sim_autotune(self.h, _ptr(actor), T, _stream(), ctypes.byref(v),
                                  ctypes.byref(ms)), "sim_autotune")
        self.tape_T = 0
        if key is not None:
            _, spl, _ = self.get_variant()
            table[key] = {"variant": v.value, "steps_per_launch": spl, "ms": ms.value}
            tmp = cache + ".tmp"
            with open(tmp, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return v.value, ms.value

    def last_rollout_timing(self):
        ms, n = ctypes.c_float(), ctypes.c_int()
        check(self.L.sim_last_rollout_timing(self.h, ctypes.byref(ms), ctypes.byref(n)),
              "sim_last_rollout_timing")
        return ms.value, n.value
