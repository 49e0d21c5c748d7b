"""MI355X-native batched quadrotor environment (fused HIP kernels behind a C
ABI).  See include/quadsim.h for the library interface."""
from ._lib import (SIM_F_ACTOR_BF16, SIM_F_AUTORESET, SIM_F_DISTURB, SIM_F_FP64,  # noqa: F401
                   SIM_F_OBS_NOISE, SIM_F_RENORM_Q, SIM_F_TERMINATE, SIM_NACTOR,
                   SIM_V_AUTO, SIM_V_FUSED_MFMA, SIM_V_FUSED_MFMA4, SIM_V_FUSED_SPLIT,
                   SIM_V_FUSED_VALU, SIM_V_PLAIN,
                   SimError, load)
from .autograd import RolloutFn, rollout  # noqa: F401
from .sim import QuadSim  # noqa: F401

__all__ = ["QuadSim", "RolloutFn", "rollout", "load", "SimError"]
