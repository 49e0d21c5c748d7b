"""FP64 CPU oracle (ctypes binding of ``quad_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark use this module.  The GPU library never imports it.

Arrays handed to the C side are AoS float64: state [n][17], history
[n][32][4], parameters [n][8].  Helpers here convert from the SoA float32
layouts the GPU library uses ([17][n], [32][4][n], [8][n]) so tests can feed
both sides the same inputs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "quad_oracle.c")
# QS_ORACLE_LIB names another build of the oracle's source to load instead
# (the planted-mistake tests compile mutated copies and run the pins on them)
_LIB = os.environ.get("QS_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

NS, NH, NA, NO, NHID, NP, NW = 17, 32, 4, 146, 64, 8, 13828


def compile_source(src: str, out: str) -> None:
    """gcc build of an oracle source (plain -O2, IEEE double, no fast-math,
    no contraction into fused multiply-adds)."""
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-ffp-contract=off",
           "-Wall", "-Wno-unused-variable", src, "-o", out + ".tmp", "-lm", "-lpthread"]
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)


def build(force: bool = True) -> str:
    """Compile liboracle.so from quad_oracle.c."""
    if force or not os.path.exists(_LIB):
        compile_source(_SRC, _LIB)
    return _LIB


class Cfg(ctypes.Structure):
    _fields_ = [
        ("dt", ctypes.c_double), ("g", ctypes.c_double), ("arm", ctypes.c_double),
        ("k_m", ctypes.c_double), ("rpm_min", ctypes.c_double), ("rpm_max", ctypes.c_double),
        ("nominal", ctypes.c_double * NP), ("dr_lo", ctypes.c_double * NP),
        ("dr_hi", ctypes.c_double * NP),
        ("pos_limit", ctypes.c_double), ("vel_limit", ctypes.c_double),
        ("init_pos", ctypes.c_double), ("init_angle", ctypes.c_double),
        ("init_vel", ctypes.c_double), ("init_angvel", ctypes.c_double),
        ("C_rp", ctypes.c_double), ("C_rq", ctypes.c_double), ("C_rv", ctypes.c_double),
        ("C_rw", ctypes.c_double), ("C_ra", ctypes.c_double), ("C_rab", ctypes.c_double),
        ("C_rs", ctypes.c_double),
        ("max_episode_steps", ctypes.c_int32), ("flags", ctypes.c_int32),
        ("dr_enable", ctypes.c_int32), ("pad_", ctypes.c_int32),
        ("seed", ctypes.c_uint64), ("dr_seed", ctypes.c_uint64),
        ("dist_force", ctypes.c_double), ("dist_torque", ctypes.c_double),
        ("obs_noise", ctypes.c_double * 4),
    ]


def make_cfg(d: dict) -> Cfg:
    c = Cfg()
    for name, typ in Cfg._fields_:
        if name == "pad_":
            continue
        v = d.get(name, 0.0 if name in ("dist_force", "dist_torque") else None)
        if name == "obs_noise":
            setattr(c, name, (ctypes.c_double * 4)(*[float(x) for x in d.get(name, (0, 0, 0, 0))]))
        elif name in ("nominal", "dr_lo", "dr_hi"):
            setattr(c, name, (ctypes.c_double * NP)(*[float(x) for x in v]))
        else:
            setattr(c, name, v)
    return c


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        d, i32, u32, u8 = ctypes.c_double, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint8
        vp = ctypes.c_void_p
        L.orc_philox4x32_10.argtypes = [vp, vp, vp]
        L.orc_uniforms.argtypes = [ctypes.c_uint64, u32, u32, u32, u32, vp]
        L.orc_init.argtypes = [P(Cfg), ctypes.c_int, vp, vp, vp, vp, vp, vp]
        L.orc_env_params.argtypes = [P(Cfg), ctypes.c_int, vp, vp]
        L.orc_reset_state.argtypes = [P(Cfg), ctypes.c_int, vp, vp, vp, vp, vp]
        L.orc_hover_rpm.argtypes = [P(Cfg), vp]
        L.orc_hover_rpm.restype = d
        L.orc_dynamics.argtypes = [P(Cfg), vp, vp, vp, vp, vp]
        L.orc_rk4.argtypes = [P(Cfg), vp, vp, vp, vp, vp]
        L.orc_observe.argtypes = [vp, vp, vp]
        L.orc_disturbance.argtypes = [P(Cfg), u32, u32, vp]
        L.orc_normals18.argtypes = [P(Cfg), u32, u32, i32, vp]
        L.orc_observe_noisy.argtypes = [P(Cfg), u32, u32, i32, vp, vp, vp]
        L.orc_critic_obs.argtypes = [P(Cfg), u32, u32, vp, vp]
        L.orc_actor.argtypes = [vp, vp, vp]
        L.orc_rotmat.argtypes = [vp, vp]
        L.orc_reward.argtypes = [P(Cfg), vp, vp]
        L.orc_reward.restype = d
        L.orc_rollout.argtypes = [P(Cfg), ctypes.c_int, vp, vp, vp, ctypes.c_int, vp, vp, vp, vp,
                                  vp, vp, vp, vp, vp, ctypes.c_int]
        L.orc_grad.argtypes = [P(Cfg), ctypes.c_int, vp, vp, vp, vp, vp, vp, vp, ctypes.c_int, vp,
                               vp, vp, vp, ctypes.c_int]
        L.orc_grad.restype = d
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------- #
# Thin wrappers                                                                 #
# --------------------------------------------------------------------------- #

def philox4x32_10(ctr, key):
    c = np.asarray(ctr, np.uint32)
    k = np.asarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def uniforms(seed, env, episode, block, stream):
    u = np.zeros(4, np.float64)
    lib().orc_uniforms(seed, env, episode, block, stream, _p(u))
    return u


class Batch:
    """AoS FP64 batch state of n envs (ids default to 0..n-1)."""

    def __init__(self, cfg: dict, n: int, ids=None):
        self.cfg = cfg
        self.c = make_cfg(cfg)
        self.n = n
        self.ids = None if ids is None else np.ascontiguousarray(ids, np.uint32)
        self.theta = np.zeros((n, NP))
        self.s = np.zeros((n, NS))
        self.H = np.zeros((n, NH, NA))
        self.t_ep = np.zeros(n, np.int32)
        self.ep = np.zeros(n, np.int32)
        # episode accumulators (Sec. V: episode return and length measure
        # training): return of the running episode, return and length of the
        # last episode that ended with an in-step reset
        self.ret_cur = np.zeros(n)
        self.ret_last = np.zeros(n)
        self.len_last = np.zeros(n, np.int32)

    @classmethod
    def init(cls, cfg: dict, n: int, ids=None) -> "Batch":
        b = cls(cfg, n, ids)
        lib().orc_init(ctypes.byref(b.c), n, _p(b.ids), _p(b.theta), _p(b.s), _p(b.H),
                       _p(b.t_ep), _p(b.ep))
        return b

    def set_soa(self, s_soa, h_soa, t_ep=None, ep=None, theta_soa=None):
        """Load float32 SoA inputs ([17][n], [32][4][n], [8][n]) as FP64."""
        self.s = _f64(np.asarray(s_soa, np.float64).T)
        self.H = _f64(np.transpose(np.asarray(h_soa, np.float64), (2, 0, 1)))
        if t_ep is not None:
            self.t_ep = np.ascontiguousarray(t_ep, np.int32).copy()
        if ep is not None:
            self.ep = np.ascontiguousarray(ep, np.int32).copy()
        if theta_soa is not None:
            self.theta = _f64(np.asarray(theta_soa, np.float64).T)

    def soa(self):
        return self.s.T.copy(), np.transpose(self.H, (1, 2, 0)).copy()

    def copy(self) -> "Batch":
        b = Batch(self.cfg, self.n, self.ids)
        b.theta, b.s, b.H = self.theta.copy(), self.s.copy(), self.H.copy()
        b.t_ep, b.ep = self.t_ep.copy(), self.ep.copy()
        b.ret_cur, b.ret_last = self.ret_cur.copy(), self.ret_last.copy()
        b.len_last = self.len_last.copy()
        return b

    def reset_envs(self, mask):
        """Ends the episodes of the masked envs and starts their next ones:
        the start state and hover-filled history of (env, episode + 1), step
        0, and the accumulators closed (running return and step count become
        the last finished episode's)."""
        idx = np.nonzero(np.asarray(mask) != 0)[0]
        if len(idx) == 0:
            return
        ep1 = np.ascontiguousarray(self.ep[idx] + 1, np.int32)
        ids = np.ascontiguousarray(idx if self.ids is None else self.ids[idx], np.uint32)
        th = _f64(self.theta[idx])
        s = np.zeros((len(idx), NS))
        H = np.zeros((len(idx), NH, NA))
        lib().orc_reset_state(ctypes.byref(self.c), len(idx), _p(ids), _p(ep1), _p(th), _p(s),
                              _p(H))
        self.s[idx] = s
        self.H[idx] = H
        self.ret_last[idx] = self.ret_cur[idx]
        self.len_last[idx] = self.t_ep[idx]
        self.ret_cur[idx] = 0.0
        self.t_ep[idx] = 0
        self.ep[idx] = ep1

    def _accumulate(self, rew, done, t_ep0):
        """Episode accumulators over a rollout's rewards and done flags: every
        reward adds to the running return; a transition that ends the episode
        with an in-step reset (autoreset on) closes it, its return and length
        (steps since its start) becoming the last finished episode's."""
        reset = (int(self.cfg["flags"]) & 2) != 0
        length = np.asarray(t_ep0, np.int64).copy()
        for t in range(rew.shape[0]):
            self.ret_cur = self.ret_cur + rew[t]
            length += 1
            fin = (done[t] != 0) & reset
            self.ret_last = np.where(fin, self.ret_cur, self.ret_last)
            self.len_last = np.where(fin, length, self.len_last).astype(np.int32)
            self.ret_cur = np.where(fin, 0.0, self.ret_cur)
            length = np.where(fin, 0, length)

    def rollout(self, W, T, actions=None, record=False, nthreads=1):
        """T steps in place.  W: flat actor (cast to FP64) or None with actions
        [T][n][4].  Returns dict(rewards [T][n], dones [T][n], states
        [T+1][n][17], acts [T][n][4]) when record, else rewards and dones."""
        n = self.n
        Wd = None if W is None else _f64(W)
        A = None if actions is None else _f64(actions)
        rew = np.zeros((T, n))
        done = np.zeros((T, n), np.uint8)
        states = np.zeros((T + 1, n, NS)) if record else None
        acts = np.zeros((T, n, NA)) if record else None
        t_ep0 = self.t_ep.copy()
        lib().orc_rollout(ctypes.byref(self.c), n, _p(self.ids), _p(Wd), _p(A), T, _p(self.s),
                          _p(self.H), _p(self.t_ep), _p(self.ep), _p(self.theta), _p(rew),
                          _p(done), _p(states), _p(acts), nthreads)
        self._accumulate(rew, done, t_ep0)
        out = dict(rewards=rew, dones=done)
        if record:
            out["states"] = states
            out["acts"] = acts
        return out

    def grad(self, W, T, dR=None, dS=None, want_grad=True, nthreads=1):
        """Differentiable rollout from the current state (not modified).
        Loss J = sum dR[t][i] r + sum dS[t][i].s.  Returns (J, gW, gtheta)."""
        n = self.n
        Wd = _f64(W)
        dRd = None if dR is None else _f64(dR)
        dSd = None if dS is None else _f64(dS)
        gW = np.zeros(NW) if want_grad else None
        gth = np.zeros((n, NP)) if want_grad else None
        t0 = np.ascontiguousarray(self.t_ep, np.int32)
        ep = np.ascontiguousarray(self.ep, np.int32)
        J = lib().orc_grad(ctypes.byref(self.c), n, _p(self.ids), _p(t0), _p(ep), _p(Wd),
                           _p(self.theta), _p(self.s), _p(self.H), T, _p(dRd), _p(dSd), _p(gW),
                           _p(gth), nthreads)
        return J, gW, gth


def hover_rpm(cfg: dict, theta) -> float:
    c = make_cfg(cfg)
    th = _f64(theta)
    return lib().orc_hover_rpm(ctypes.byref(c), _p(th))


def dynamics(cfg: dict, theta, x, u, dist=None):
    """f(x, u; theta) with the episode disturbance dist = {f_r, tau_r} (or none)."""
    c = make_cfg(cfg)
    out = np.zeros(NS)
    d = None if dist is None else _f64(dist)
    lib().orc_dynamics(ctypes.byref(c), _p(_f64(theta)), _p(_f64(x)), _p(_f64(u)), _p(d), _p(out))
    return out


def rk4(cfg: dict, theta, x, u, dist=None):
    c = make_cfg(cfg)
    out = np.zeros(NS)
    d = None if dist is None else _f64(dist)
    lib().orc_rk4(ctypes.byref(c), _p(_f64(theta)), _p(_f64(x)), _p(_f64(u)), _p(d), _p(out))
    return out


def disturbance(cfg: dict, env: int, episode: int):
    c = make_cfg(cfg)
    d = np.zeros(6)
    lib().orc_disturbance(ctypes.byref(c), env, episode, _p(d))
    return d


def normals18(cfg: dict, env: int, episode: int, t_ep: int):
    c = make_cfg(cfg)
    z = np.zeros(18)
    lib().orc_normals18(ctypes.byref(c), env, episode, t_ep, _p(z))
    return z


def observe_noisy(cfg: dict, env: int, episode: int, t_ep: int, s, H):
    c = make_cfg(cfg)
    o = np.zeros(NO)
    lib().orc_observe_noisy(ctypes.byref(c), env, episode, t_ep, _p(_f64(s)), _p(_f64(H)), _p(o))
    return o


def critic_obs(cfg: dict, env: int, episode: int, s):
    c = make_cfg(cfg)
    oc = np.zeros(28)
    lib().orc_critic_obs(ctypes.byref(c), env, episode, _p(_f64(s)), _p(oc))
    return oc


def observe(s, H):
    o = np.zeros(NO)
    lib().orc_observe(_p(_f64(s)), _p(_f64(H)), _p(o))
    return o


def actor(W, o):
    a = np.zeros(NA)
    lib().orc_actor(_p(_f64(W)), _p(_f64(o)), _p(a))
    return a


def rotmat(q):
    R = np.zeros(9)
    lib().orc_rotmat(_p(_f64(q)), _p(R))
    return R.reshape(3, 3)


def reward(cfg: dict, s, a) -> float:
    c = make_cfg(cfg)
    return lib().orc_reward(ctypes.byref(c), _p(_f64(s)), _p(_f64(a)))
