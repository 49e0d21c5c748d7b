"""ctypes binding of libquadsim.so (the C ABI in include/quadsim.h).

Argument marshalling only: every step of the simulation runs in the library's
HIP kernels.  torch is imported first so the library binds to the same HIP
runtime torch uses (device pointers and streams are then interchangeable).
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (must be loaded before the library, see above)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libquadsim.so")

SIM_NSTATE, SIM_NHIST, SIM_NACT, SIM_NOBS, SIM_NHID, SIM_NPARAM, SIM_NACTOR = (
    17, 32, 4, 146, 64, 8, 13828)
SIM_OK, SIM_E_INVAL, SIM_E_NOMEM, SIM_E_DEVICE, SIM_E_STATE, SIM_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
SIM_F_TERMINATE, SIM_F_AUTORESET, SIM_F_RENORM_Q, SIM_F_FP64, SIM_F_ACTOR_BF16 = 1, 2, 4, 8, 16
SIM_F_DISTURB, SIM_F_OBS_NOISE = 32, 64
SIM_V_AUTO, SIM_V_PLAIN, SIM_V_FUSED_VALU, SIM_V_FUSED_MFMA, SIM_V_FUSED_MFMA4 = 0, 1, 2, 3, 4
SIM_V_FUSED_SPLIT = 5

EXPORTS = (
    "sim_create", "sim_destroy", "sim_reset", "sim_step", "sim_rollout", "sim_backward",
    "sim_get_state", "sim_set_state", "sim_get_params", "sim_set_params", "sim_set_variant",
    "sim_get_variant", "sim_autotune", "sim_last_rollout_timing", "sim_n_envs", "sim_last_error",
    "sim_rollout_actions", "sim_observe", "sim_set_reward", "sim_reset_envs", "sim_reward",
    "sim_backward_noalloc", "sim_set_target",
)


class SimConfig(ctypes.Structure):
    _fields_ = [
        ("n_envs", ctypes.c_int32), ("max_episode_steps", ctypes.c_int32),
        ("flags", ctypes.c_int32), ("dr_enable", ctypes.c_int32),
        ("max_tape_horizon", ctypes.c_int32), ("ckpt_every", ctypes.c_int32),
        ("reserved0", ctypes.c_int32), ("reserved1", ctypes.c_int32),
        ("dt", ctypes.c_double), ("g", ctypes.c_double), ("arm", ctypes.c_double),
        ("k_m", ctypes.c_double), ("rpm_min", ctypes.c_double), ("rpm_max", ctypes.c_double),
        ("nominal", ctypes.c_double * 8), ("dr_lo", ctypes.c_double * 8),
        ("dr_hi", ctypes.c_double * 8),
        ("pos_limit", ctypes.c_double), ("vel_limit", ctypes.c_double),
        ("init_pos", ctypes.c_double), ("init_angle", ctypes.c_double),
        ("init_vel", ctypes.c_double), ("init_angvel", ctypes.c_double),
        ("C_rp", ctypes.c_double), ("C_rq", ctypes.c_double), ("C_rv", ctypes.c_double),
        ("C_rw", ctypes.c_double), ("C_ra", ctypes.c_double), ("C_rab", ctypes.c_double),
        ("C_rs", ctypes.c_double),
        ("seed", ctypes.c_uint64), ("dr_seed", ctypes.c_uint64),
        ("dist_force", ctypes.c_double), ("dist_torque", ctypes.c_double),
        ("obs_noise", ctypes.c_double * 4),
    ]


def make_config(d: dict) -> SimConfig:
    c = SimConfig()
    for name, _ in SimConfig._fields_:
        if name.startswith("reserved"):
            continue
        if name == "obs_noise":
            setattr(c, name, (ctypes.c_double * 4)(*[float(x) for x in d.get(name, (0,) * 4)]))
            continue
        v = d.get(name, 0.0) if name in ("dist_force", "dist_torque") else d[name]
        if name in ("nominal", "dr_lo", "dr_hi"):
            setattr(c, name, (ctypes.c_double * 8)(*[float(x) for x in v]))
        else:
            setattr(c, name, v)
    return c


_lib = None


def load(path: str | None = None):
    """Loads the library (built in place by paper_2311_13081_amd.build).
    Raises if it is missing: there is no fallback implementation."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(
            f"{p} is missing: build it with `python -m paper_2311_13081_amd.build` "
            "(the simulator has no non-HIP fallback)")
    L = ctypes.CDLL(p)
    vp, i32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64
    H = ctypes.c_void_p
    sig = {
        "sim_create": ([ctypes.POINTER(SimConfig), ctypes.c_int, ctypes.POINTER(H)], ctypes.c_int),
        "sim_destroy": ([H], ctypes.c_int),
        "sim_reset": ([H, u64, vp], ctypes.c_int),
        "sim_step": ([H, vp, vp, vp, vp, vp], ctypes.c_int),
        "sim_rollout": ([H, vp, i32, vp, vp, vp, i32, vp], ctypes.c_int),
        "sim_backward": ([H, vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "sim_backward_noalloc": ([H, vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "sim_rollout_actions": ([H, vp, i32, i32, vp, vp, vp, vp], ctypes.c_int),
        "sim_observe": ([H, vp, vp, vp], ctypes.c_int),
        "sim_get_state": ([H, vp, vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "sim_set_state": ([H, vp, vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "sim_set_reward": ([H, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
        "sim_reset_envs": ([H, vp, vp], ctypes.c_int),
        "sim_set_target": ([H, vp, ctypes.c_double, ctypes.c_double, vp], ctypes.c_int),
        "sim_reward": ([H, vp, vp, i32, vp, vp], ctypes.c_int),
        "sim_get_params": ([H, vp, vp], ctypes.c_int),
        "sim_set_params": ([H, vp, vp], ctypes.c_int),
        "sim_set_variant": ([H, ctypes.c_int, ctypes.c_int, ctypes.c_int], ctypes.c_int),
        "sim_get_variant": ([H, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                             ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "sim_autotune": ([H, vp, i32, vp, ctypes.POINTER(ctypes.c_int),
                          ctypes.POINTER(ctypes.c_float)], ctypes.c_int),
        "sim_last_rollout_timing": ([H, ctypes.POINTER(ctypes.c_float),
                                     ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "sim_n_envs": ([H], ctypes.c_int),
        "sim_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


class SimError(RuntimeError):
    def __init__(self, code: int, call: str):
        msg = load().sim_last_error().decode(errors="replace")
        super().__init__(f"{call} failed with status {code}: {msg}")
        self.code = code


def check(code: int, call: str):
    if code != SIM_OK:
        raise SimError(code, call)
