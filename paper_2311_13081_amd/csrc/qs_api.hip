// Host runtime of the C ABI declared in include/quadsim.h: argument checks,
// device memory owned by the handle, variant dispatch, hipGraph replay of
// multi-launch rollouts, HIP-event timing and the autotuner.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/quadsim.h"
#include "qs_backward.h"
#include "qs_forward.h"
#include "qs_precise.h"

using namespace qs;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(e_ == hipErrorOutOfMemory ? SIM_E_NOMEM : SIM_E_DEVICE, "%s: %s (%s:%d)", \
                  #expr, hipGetErrorString(e_), __FILE__, __LINE__);                      \
  } while (0)

// Makes the handle's device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

struct GraphKey {
  int variant = -1, spl = 0, T = 0, tape = 0;
  const void *W = nullptr, *rew = nullptr, *done = nullptr, *states = nullptr;
  bool operator==(const GraphKey& o) const {
    return variant == o.variant && spl == o.spl && T == o.T && tape == o.tape && W == o.W &&
           rew == o.rew && done == o.done && states == o.states;
  }
};

}  // namespace

// Scratch of sim_backward_noalloc: a device array that every GPU the library
// runs on holds until the process ends.  Host code must not use its name as
// an address (it is a host-side stand-in); the device address of each GPU's
// copy is looked up once per device at sim_create and kept in g_scratch.
constexpr size_t NOALLOC_SCRATCH_FLOATS = (size_t)8 << 20;  // 32 MiB
static __device__ __align__(256) float scratch[NOALLOC_SCRATCH_FLOATS];
namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
float* g_scratch[MAX_DEVICES] = {};

// Device address of this device's scratch array (the device is current).
int scratch_lookup(int device) {
  if (device < 0 || device >= MAX_DEVICES) return fail(SIM_E_UNSUPPORTED, "device %d", device);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[device]) return SIM_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(SIM_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
  g_scratch[device] = static_cast<float*>(ptr);
  return SIM_OK;
}
}  // namespace

static_assert(SIM_F_ACTOR_BF16 == F_ACTOR_BF16 && SIM_F_DISTURB == F_DISTURB &&
                  SIM_F_OBS_NOISE == F_OBS_NOISE && SIM_F_TERMINATE == F_TERMINATE &&
                  SIM_F_AUTORESET == F_AUTORESET && SIM_F_RENORM_Q == F_RENORM_Q,
              "public flag values are read by the kernels");

struct sim_handle {
  sim_config cfg{};
  DevCfg dc{};
  int device = 0, N = 0;
  SimBufs b{};
  PlainBufs p{};
  float* tape = nullptr;     // [max_tape_horizon/K + 1][145][N]
  int tape_ckpts = 0;
  int tape_T = 0;            // horizon of the recorded tape (0 = none)
  // segment of the current tape whose record segment buffer b holds (-1: none)
  int seg_held[BWD_NBUF] = {-1, -1, -1, -1};
  BwdBufs bw{};
  int variant = SIM_V_AUTO, spl = 0, use_graph = 1;
  int tuned_variant = SIM_V_FUSED_MFMA, tuned_spl = 0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  GraphKey gkey{};
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  int last_launches = 0;
  bool timing_valid = false;
  bool fp64 = false;          // SIM_F_FP64: double-precision path only
  bool bf16 = false;          // SIM_F_ACTOR_BF16: quarter-lane kernel with bf16 actor
  PreciseCfg pc{};
  PreciseBufs pb{};
  float* target_buf = nullptr;  // [6][N] set points of the actor's observation
  bool target_on = false;
  float pos_clip = 0.0f, vel_clip = 0.0f;
};

namespace {

bool finite_pos(double v) { return std::isfinite(v) && v > 0; }

int check_config(const sim_config* c) {
  if (!c) return fail(SIM_E_INVAL, "config is NULL");
  if (c->n_envs < 1 || c->n_envs > (1 << 24)) return fail(SIM_E_INVAL, "n_envs %d out of range", c->n_envs);
  if (c->max_episode_steps < 0) return fail(SIM_E_INVAL, "max_episode_steps < 0");
  if (c->flags & ~(SIM_F_TERMINATE | SIM_F_AUTORESET | SIM_F_RENORM_Q | SIM_F_FP64 |
                   SIM_F_ACTOR_BF16 | SIM_F_DISTURB | SIM_F_OBS_NOISE))
    return fail(SIM_E_INVAL, "unknown flags 0x%x", c->flags);
  if (!(c->dist_force >= 0) || !(c->dist_torque >= 0) || !std::isfinite(c->dist_force) ||
      !std::isfinite(c->dist_torque))
    return fail(SIM_E_INVAL, "disturbance bounds must be finite and >= 0");
  for (int i = 0; i < 4; ++i)
    if (!(c->obs_noise[i] >= 0) || !std::isfinite(c->obs_noise[i]))
      return fail(SIM_E_INVAL, "observation noise std must be finite and >= 0");
  if ((c->flags & SIM_F_FP64) && (c->flags & SIM_F_ACTOR_BF16))
    return fail(SIM_E_INVAL, "SIM_F_FP64 and SIM_F_ACTOR_BF16 exclude each other");
  if ((c->flags & SIM_F_FP64) && c->max_tape_horizon > 0)
    return fail(SIM_E_UNSUPPORTED, "SIM_F_FP64 handles are forward only (max_tape_horizon 0)");
  if (c->max_tape_horizon < 0 || c->max_tape_horizon > (1 << 20))
    return fail(SIM_E_INVAL, "max_tape_horizon out of range");
  if (c->ckpt_every < 1 || c->ckpt_every > 4096) return fail(SIM_E_INVAL, "ckpt_every must be in [1, 4096]");
  // the backward addresses a segment's record with 32-bit byte offsets
  if (c->max_tape_horizon > 0 &&
      4.0 * (double)rec_floats(c->ckpt_every, c->n_envs) >= 4294967296.0)
    return fail(SIM_E_INVAL, "n_envs %d x ckpt_every %d too large for a differentiable handle",
                c->n_envs, c->ckpt_every);
  if (!finite_pos(c->dt) || !finite_pos(c->g) || !finite_pos(c->arm) || !std::isfinite(c->k_m))
    return fail(SIM_E_INVAL, "dt, g, arm must be finite and positive");
  if (!std::isfinite(c->rpm_min) || !std::isfinite(c->rpm_max) || !(c->rpm_max > c->rpm_min))
    return fail(SIM_E_INVAL, "need rpm_max > rpm_min");
  const double* nom = c->nominal;
  if (!finite_pos(nom[0]) || !finite_pos(nom[1]) || !finite_pos(nom[2]) || !finite_pos(nom[3]) ||
      !finite_pos(nom[7]))
    return fail(SIM_E_INVAL, "mass, inertia and motor time constant must be positive");
  if (!(nom[6] >= 0) || !std::isfinite(nom[4]) || !std::isfinite(nom[5]) || !std::isfinite(nom[6]))
    return fail(SIM_E_INVAL, "thrust coefficients must be finite with c2 >= 0");
  for (int i = 0; i < SIM_NPARAM; ++i)
    if (c->dr_enable && !(c->dr_lo[i] > 0 && c->dr_hi[i] >= c->dr_lo[i] && std::isfinite(c->dr_hi[i])))
      return fail(SIM_E_INVAL, "dr range %d invalid", i);
  if (!finite_pos(c->pos_limit) || !finite_pos(c->vel_limit))
    return fail(SIM_E_INVAL, "limits must be positive");
  const double need = nom[0] * c->g / 4 - nom[4];
  if (!(need > 0) || (nom[6] == 0 && !(nom[5] > 0)))
    return fail(SIM_E_INVAL, "thrust curve cannot hover the nominal body");
  return SIM_OK;
}

DevCfg make_devcfg(const sim_config& c, uint64_t seed) {
  DevCfg d{};
  d.n_envs = c.n_envs;
  d.max_steps = c.max_episode_steps;
  d.flags = c.flags;
  d.dr_enable = c.dr_enable;
  d.dt = (float)c.dt;
  d.g = (float)c.g;
  d.arm = (float)c.arm;
  d.km = (float)c.k_m;
  d.rpm_min = (float)c.rpm_min;
  d.rpm_half_range = (float)(0.5 * (c.rpm_max - c.rpm_min));
  d.pos_limit = (float)c.pos_limit;
  d.vel_limit = (float)c.vel_limit;
  d.init_pos = (float)c.init_pos;
  d.init_angle = (float)c.init_angle;
  d.init_vel = (float)c.init_vel;
  d.init_angvel = (float)c.init_angvel;
  d.C_rp = (float)c.C_rp;
  d.C_rq = (float)c.C_rq;
  d.C_rv = (float)c.C_rv;
  d.C_rw = (float)c.C_rw;
  d.C_ra = (float)c.C_ra;
  d.C_rab = (float)c.C_rab;
  d.C_rs = (float)c.C_rs;
  for (int i = 0; i < NP; ++i) {
    d.nominal[i] = (float)c.nominal[i];
    d.dr_lo[i] = (float)c.dr_lo[i];
    d.dr_hi[i] = (float)c.dr_hi[i];
  }
  d.seed_lo = (uint32_t)seed;
  d.seed_hi = (uint32_t)(seed >> 32);
  d.dr_seed_lo = (uint32_t)c.dr_seed;
  d.dr_seed_hi = (uint32_t)(c.dr_seed >> 32);
  d.dist_force = (float)c.dist_force;
  d.dist_torque = (float)c.dist_torque;
  for (int i = 0; i < 4; ++i) d.noise[i] = (float)c.obs_noise[i];
  return d;
}

PreciseCfg make_precise(const sim_config& c, uint64_t seed) {
  PreciseCfg p{};
  p.n_envs = c.n_envs;
  p.max_steps = c.max_episode_steps;
  p.flags = c.flags;
  p.dr_enable = c.dr_enable;
  p.dt = c.dt;
  p.g = c.g;
  p.arm = c.arm;
  p.km = c.k_m;
  p.rpm_min = c.rpm_min;
  p.rpm_max = c.rpm_max;
  p.pos_limit = c.pos_limit;
  p.vel_limit = c.vel_limit;
  p.init_pos = c.init_pos;
  p.init_angle = c.init_angle;
  p.init_vel = c.init_vel;
  p.init_angvel = c.init_angvel;
  p.C_rp = c.C_rp;
  p.C_rq = c.C_rq;
  p.C_rv = c.C_rv;
  p.C_rw = c.C_rw;
  p.C_ra = c.C_ra;
  p.C_rab = c.C_rab;
  p.C_rs = c.C_rs;
  for (int i = 0; i < NP; ++i) {
    p.nominal[i] = c.nominal[i];
    p.dr_lo[i] = c.dr_lo[i];
    p.dr_hi[i] = c.dr_hi[i];
  }
  p.seed_lo = (uint32_t)seed;
  p.seed_hi = (uint32_t)(seed >> 32);
  p.dr_seed_lo = (uint32_t)c.dr_seed;
  p.dr_seed_hi = (uint32_t)(c.dr_seed >> 32);
  p.dist_force = c.dist_force;
  p.dist_torque = c.dist_torque;
  for (int i = 0; i < 4; ++i) p.noise[i] = c.obs_noise[i];
  return p;
}

// The set point of the actor's observation travels in the device config.
void apply_target(sim_handle* h) {
  h->dc.target = h->target_on ? h->target_buf : nullptr;
  h->dc.pos_clip = h->pos_clip;
  h->dc.vel_clip = h->vel_clip;
}

// Error left by earlier asynchronous work on this device, if any.
int sticky_error() {
  hipError_t e = hipPeekAtLastError();
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(SIM_E_DEVICE, "earlier device error: %s", hipGetErrorString(e));
  }
  return SIM_OK;
}

int effective_variant(const sim_handle* h) {
  return h->variant == SIM_V_AUTO ? h->tuned_variant : h->variant;
}
int effective_spl(const sim_handle* h) { return h->variant == SIM_V_AUTO ? h->tuned_spl : h->spl; }

void drop_graph(sim_handle* h) {
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  h->gexec = nullptr;
  h->graph = nullptr;
  h->gkey = GraphKey{};
}

// Segments of a taped T-step rollout whose backward records the rollout
// writes itself: the last ones, one per segment buffer.  Small batches (the
// split-actor kernel) record only the last: their backward runs the other
// recomputes beside the sweeps on a stream of their own, so recording more
// in the forward, which nothing overlaps, measured slower (1024 x 64: 0.86
// against 0.84 ms).
static_assert(REC_SEGS == BWD_NBUF, "one record segment per segment buffer");
static int recorded_segments(const sim_handle* h, int T) {
  const int J = (T + h->cfg.ckpt_every - 1) / h->cfg.ckpt_every;
  const int m = taped_kernel(h->dc) == TAPED_SPLIT ? 1 : REC_SEGS;
  return J < m ? J : m;
}

// Queues the launches of a T-step rollout on st.
// With tape != NULL the launches also write the backward's record of the
// tape's last m = recorded_segments() segments (steps from (J - m) K on,
// J = ceil(T / K)) into the segment buffers (the last segment into the
// first), so the backward need not recompute those segments.
int enqueue_rollout(sim_handle* h, int variant, int spl, const float* W, int T, float* rew,
                    uint8_t* done, float* states, float* tape, hipStream_t st, int* launches) {
  const int N = h->N;
  const int K = h->cfg.ckpt_every;
  int nl = 0;
  if (variant == SIM_V_PLAIN) {
    if (states) HIP_TRY(launch_copy_state(h->b, N, states, st));
    for (int t = 0; t < T; ++t) {
      HIP_TRY(launch_plain_step(h->dc, h->b, h->p, W, nullptr, rew ? rew + (size_t)t * N : nullptr,
                                done ? done + (size_t)t * N : nullptr,
                                states ? states + (size_t)(t + 1) * NS * N : nullptr, st));
      ++nl;
    }
  } else {
    const bool mfma = variant == SIM_V_FUSED_MFMA;
    const int chunk = (spl <= 0 || spl > T) ? T : spl;
    float* rec = tape ? h->bw.seg[0] : nullptr;
    const int J = (T + K - 1) / K;
    const int rec_from = tape ? (J - recorded_segments(h, T)) * K : 0;
    const int rec_n = T - rec_from;
    const RecSpan rs{{rec, h->bw.seg[1], h->bw.seg[2], h->bw.seg[3]}, rec_from, K, rec_n};
    for (int t0 = 0; t0 < T; t0 += chunk) {
      const int n = (T - t0) < chunk ? (T - t0) : chunk;
      if (variant == SIM_V_FUSED_MFMA4)
        HIP_TRY(launch_fused4(h->dc, h->b, W, n, t0, rew, done, states, tape, K, nullptr, rs, st));
      else if (variant == SIM_V_FUSED_SPLIT)
        HIP_TRY(launch_split(h->dc, h->b, W, n, t0, rew, done, states, tape, K, nullptr, rs, st));
      else if (tape && mfma)
        HIP_TRY(launch_fused_taped(h->dc, h->b, W, n, t0, rew, done, states, tape, K, nullptr, rs,
                                   st));
      else
        HIP_TRY(launch_fused(mfma, h->dc, h->b, W, nullptr, n, t0, rew, done, states, st));
      ++nl;
    }
  }
  *launches = nl;
  return SIM_OK;
}

}  // namespace

extern "C" {

const char* sim_last_error(void) { return g_err.c_str(); }

int sim_n_envs(const sim_handle* h) { return h ? h->N : 0; }

int sim_create(const sim_config* cfg, int device, sim_handle** out) {
  if (!out) return fail(SIM_E_INVAL, "out is NULL");
  *out = nullptr;
  int rc = check_config(cfg);
  if (rc) return rc;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return fail(SIM_E_DEVICE, "no HIP device");
  if (device < 0 || device >= ndev) return fail(SIM_E_INVAL, "device %d not in [0, %d)", device, ndev);
  DeviceGuard g(device);
  if (!g.ok) return fail(SIM_E_DEVICE, "hipSetDevice(%d) failed", device);
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(SIM_E_UNSUPPORTED, "built for gfx950, device is %s", prop.gcnArchName);
  // once per device, with the device current: the address of its copy of
  // the scratch array of sim_backward_noalloc
  rc = scratch_lookup(device);
  if (rc) return rc;

  sim_handle* h = new sim_handle();
  h->cfg = *cfg;
  h->device = device;
  h->N = cfg->n_envs;
  h->dc = make_devcfg(*cfg, cfg->seed);
  const size_t N = (size_t)h->N;
  auto alloc = [&](void** p, size_t bytes) -> int {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? SIM_E_NOMEM : SIM_E_DEVICE, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    return SIM_OK;
  };
  rc = SIM_OK;
  h->fp64 = (cfg->flags & SIM_F_FP64) != 0;
  h->bf16 = (cfg->flags & SIM_F_ACTOR_BF16) != 0;
  if (h->bf16) h->tuned_variant = SIM_V_FUSED_MFMA4;  // the taped rollouts' kernel
  if (h->fp64) {
    h->pc = make_precise(*cfg, cfg->seed);
    rc = rc ? rc : alloc((void**)&h->pb.state, N * NS * 8);
    rc = rc ? rc : alloc((void**)&h->pb.ring, N * NH * NA * 8);
    rc = rc ? rc : alloc((void**)&h->pb.head, N * 4);
    rc = rc ? rc : alloc((void**)&h->pb.t_ep, N * 4);
    rc = rc ? rc : alloc((void**)&h->pb.ep, N * 4);
    rc = rc ? rc : alloc((void**)&h->pb.theta, N * NP * 8);
    rc = rc ? rc : alloc((void**)&h->pb.ret, N * 2 * 8);
    rc = rc ? rc : alloc((void**)&h->pb.last_len, N * 4);
    if (!rc && precise_prepare() != hipSuccess) rc = fail(SIM_E_DEVICE, "fp64 kernel setup failed");
    if (!rc && hipEventCreate(&h->ev0) == hipSuccess && hipEventCreate(&h->ev1) == hipSuccess) {
      hipError_t e = precise_init(h->pc, h->pb, 1, nullptr);
      if (e == hipSuccess) e = hipDeviceSynchronize();
      if (e != hipSuccess) rc = fail(SIM_E_DEVICE, "init: %s", hipGetErrorString(e));
    } else if (!rc) {
      rc = fail(SIM_E_DEVICE, "event creation failed");
    }
    if (rc) {
      sim_destroy(h);
      return rc;
    }
    *out = h;
    return SIM_OK;
  }
  rc = rc ? rc : alloc((void**)&h->b.state, N * NS * 4);
  rc = rc ? rc : alloc((void**)&h->b.ring, N * NH * NA * 4);
  rc = rc ? rc : alloc((void**)&h->b.head, N * 4);
  rc = rc ? rc : alloc((void**)&h->b.t_ep, N * 4);
  rc = rc ? rc : alloc((void**)&h->b.ep, N * 4);
  rc = rc ? rc : alloc((void**)&h->b.theta, N * NP * 4);
  rc = rc ? rc : alloc((void**)&h->b.ret, N * 2 * 4);
  rc = rc ? rc : alloc((void**)&h->b.last_len, N * 4);
  rc = rc ? rc : alloc((void**)&h->p.obs, N * NO * 4);
  rc = rc ? rc : alloc((void**)&h->p.h1, N * NHID * 4);
  rc = rc ? rc : alloc((void**)&h->p.h2, N * NHID * 4);
  rc = rc ? rc : alloc((void**)&h->p.act, N * NA * 4);
  rc = rc ? rc : alloc((void**)&h->target_buf, N * 6 * 4);
  if (!rc && cfg->max_tape_horizon > 0) {
    h->tape_ckpts = (cfg->max_tape_horizon + cfg->ckpt_every - 1) / cfg->ckpt_every + 1;
    rc = alloc((void**)&h->tape, (size_t)h->tape_ckpts * CK_F * N * 4);
    if (!rc) {
      const hipError_t e = bwd_alloc(h->bw, h->N, cfg->ckpt_every, cfg->max_tape_horizon);
      if (e != hipSuccess)
        rc = fail(e == hipErrorOutOfMemory ? SIM_E_NOMEM : SIM_E_DEVICE,
                  "backward scratch set-up: %s", hipGetErrorString(e));
    }
  }
  if (!rc && hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) != hipSuccess)
    rc = fail(SIM_E_DEVICE, "stream creation failed");
  if (!rc && (hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess))
    rc = fail(SIM_E_DEVICE, "event creation failed");
  if (!rc) {
    hipError_t e = launch_init(h->dc, h->b, 1, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) rc = fail(SIM_E_DEVICE, "init: %s", hipGetErrorString(e));
  }
  if (rc) {
    sim_destroy(h);
    return rc;
  }
  *out = h;
  return SIM_OK;
}

int sim_destroy(sim_handle* h) {
  if (!h) return SIM_OK;
  DeviceGuard g(h->device);
  (void)hipDeviceSynchronize();
  drop_graph(h);
  void* ptrs[] = {h->b.state,  h->b.ring,  h->b.head,    h->b.t_ep,  h->b.ep,
                  h->b.theta,  h->b.ret,   h->b.last_len, h->p.obs,   h->p.h1,
                  h->p.h2,     h->p.act,   h->tape,      h->pb.state, h->pb.ring, h->target_buf,
                  h->pb.head,  h->pb.t_ep, h->pb.ep,     h->pb.theta, h->pb.ret,
                  h->pb.last_len};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  bwd_free(h->bw);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  if (h->ev0) (void)hipEventDestroy(h->ev0);
  if (h->ev1) (void)hipEventDestroy(h->ev1);
  delete h;
  return SIM_OK;
}

int sim_reset(sim_handle* h, uint64_t seed, void* stream) {
  if (!h) return fail(SIM_E_INVAL, "handle is NULL");
  DeviceGuard g(h->device);
  int rc = sticky_error();
  if (rc) return rc;
  h->cfg.seed = seed;
  h->dc = make_devcfg(h->cfg, seed);
  apply_target(h);
  h->tape_T = 0;
  drop_graph(h);
  if (h->fp64) {
    h->pc = make_precise(h->cfg, seed);
    HIP_TRY(precise_init(h->pc, h->pb, 0, (hipStream_t)stream));
    return SIM_OK;
  }
  HIP_TRY(launch_init(h->dc, h->b, 0, (hipStream_t)stream));
  return SIM_OK;
}

int sim_step(sim_handle* h, const float* actor, const float* actions, float* reward, uint8_t* done,
             void* stream) {
  if (!h) return fail(SIM_E_INVAL, "handle is NULL");
  if (!actor && !actions) return fail(SIM_E_INVAL, "need actor weights or actions");
  DeviceGuard g(h->device);
  int rc = sticky_error();
  if (rc) return rc;
  h->tape_T = 0;
  hipStream_t st = (hipStream_t)stream;
  if (h->fp64) {
    HIP_TRY(precise_run(h->pc, h->pb, actor, actor ? nullptr : actions, 1, 0, reward, done,
                        nullptr, st));
    return SIM_OK;
  }
  const int v = effective_variant(h);
  if (v == SIM_V_PLAIN) {
    HIP_TRY(launch_plain_step(h->dc, h->b, h->p, actor, actor ? nullptr : actions, reward, done,
                              nullptr, st));
  } else if (v == SIM_V_FUSED_MFMA4 && actor) {
    HIP_TRY(launch_fused4(h->dc, h->b, actor, 1, 0, reward, done, nullptr, nullptr,
                          h->cfg.ckpt_every, nullptr, RecSpan{}, st));
  } else if (v == SIM_V_FUSED_SPLIT && actor) {
    HIP_TRY(launch_split(h->dc, h->b, actor, 1, 0, reward, done, nullptr, nullptr, 1, nullptr,
                         RecSpan{}, st));
  } else {
    // external actions run on the one-env-per-lane kernel (it has the
    // action-input path); both kernels share the state layout
    HIP_TRY(launch_fused(v != SIM_V_FUSED_VALU, h->dc, h->b, actor, actor ? nullptr : actions, 1,
                         0, reward, done, nullptr, st));
  }
  return SIM_OK;
}

int sim_rollout(sim_handle* h, const float* actor, int32_t T, float* rewards, uint8_t* dones,
                float* states, int32_t record_tape, void* stream) {
  if (!h) return fail(SIM_E_INVAL, "handle is NULL");
  if (!actor) return fail(SIM_E_INVAL, "actor is NULL");
  if (T < 1) return fail(SIM_E_INVAL, "T = %d < 1", T);
  if (record_tape) {
    if (h->cfg.max_tape_horizon <= 0 || T > h->cfg.max_tape_horizon)
      return fail(SIM_E_INVAL, "T = %d exceeds max_tape_horizon = %d", T, h->cfg.max_tape_horizon);
    if (h->cfg.flags & (SIM_F_TERMINATE | SIM_F_AUTORESET))
      return fail(SIM_E_STATE, "differentiable rollouts need TERMINATE and AUTORESET off");
    if (h->target_on)
      return fail(SIM_E_STATE, "differentiable rollouts do not take a set point (sim_set_target)");
  }
  DeviceGuard g(h->device);
  int rc = sticky_error();
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  if (h->fp64) {
    HIP_TRY(hipEventRecord(h->ev0, st));
    HIP_TRY(precise_run(h->pc, h->pb, actor, nullptr, T, 0, rewards, dones, states, st));
    HIP_TRY(hipEventRecord(h->ev1, st));
    h->last_launches = 1;
    h->timing_valid = true;
    return SIM_OK;
  }
  // A taped rollout runs on the kernel the backward pass recomputes its
  // segments with (the recompute must reproduce the forward trajectory bit
  // for bit): the split-actor kernel for small fp32 batches, else the
  // quarter-lane kernel.
  const TapedKernel tk = taped_kernel(h->dc);
  const int v = record_tape ? (tk == TAPED_SPLIT ? SIM_V_FUSED_SPLIT
                               : tk == TAPED_LANE ? SIM_V_FUSED_MFMA : SIM_V_FUSED_MFMA4)
                            : effective_variant(h);
  const int spl = effective_spl(h);
  float* tape = record_tape ? h->tape : nullptr;
  h->tape_T = 0;
  int launches = 0;
  const bool multi = (v == SIM_V_PLAIN) || (spl > 0 && spl < T);
  if (h->use_graph && multi) {
    GraphKey key;
    key.variant = v;
    key.spl = spl;
    key.T = T;
    key.tape = record_tape ? 1 : 0;
    key.W = actor;
    key.rew = rewards;
    key.done = dones;
    key.states = states;
    if (!(h->gexec && h->gkey == key)) {
      drop_graph(h);
      HIP_TRY(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
      int rc2 = enqueue_rollout(h, v, spl, actor, T, rewards, dones, states, tape, h->cap_stream,
                                &launches);
      hipGraph_t gr = nullptr;
      hipError_t e = hipStreamEndCapture(h->cap_stream, &gr);
      if (rc2) {
        if (gr) (void)hipGraphDestroy(gr);
        return rc2;
      }
      if (e != hipSuccess) return fail(SIM_E_DEVICE, "graph capture: %s", hipGetErrorString(e));
      h->graph = gr;
      e = hipGraphInstantiate(&h->gexec, gr, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        drop_graph(h);
        return fail(SIM_E_DEVICE, "graph instantiate: %s", hipGetErrorString(e));
      }
      h->gkey = key;
    }
    launches = v == SIM_V_PLAIN ? T : (T + spl - 1) / spl;
    HIP_TRY(hipEventRecord(h->ev0, st));
    HIP_TRY(hipGraphLaunch(h->gexec, st));
    HIP_TRY(hipEventRecord(h->ev1, st));
  } else {
    HIP_TRY(hipEventRecord(h->ev0, st));
    rc = enqueue_rollout(h, v, spl, actor, T, rewards, dones, states, tape, st, &launches);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(h->ev1, st));
  }
  h->last_launches = launches;
  h->timing_valid = true;
  if (record_tape) {
    h->tape_T = T;
    const int J = (T + h->cfg.ckpt_every - 1) / h->cfg.ckpt_every;
    const int m = recorded_segments(h, T);
    for (int i = 0; i < BWD_NBUF; ++i) h->seg_held[i] = i < m ? J - 1 - i : -1;
  }
  return SIM_OK;
}

int sim_observe(sim_handle* h, float* actor_obs, float* critic_obs, void* stream) {
  if (!h) return fail(SIM_E_INVAL, "handle is NULL");
  if (h->fp64) return fail(SIM_E_UNSUPPORTED, "not available on SIM_F_FP64 handles");
  DeviceGuard g(h->device);
  int rc = sticky_error();
  if (rc) return rc;
  if (!actor_obs && !critic_obs) return SIM_OK;
  HIP_TRY(launch_observe(h->dc, h->b, actor_obs, critic_obs, (hipStream_t)stream));
  return SIM_OK;
}

int sim_rollout_actions(sim_handle* h, const float* actions, int32_t actions_per_step, int32_t T,
                        float* rewards, uint8_t* dones, float* states, void* stream) {
  if (!h) return fail(SIM_E_INVAL, "handle is NULL");
  if (!actions) return fail(SIM_E_INVAL, "actions is NULL");
  if (T < 1) return fail(SIM_E_INVAL, "T = %d < 1", T);
  if (h->fp64) return fail(SIM_E_UNSUPPORTED, "not available on SIM_F_FP64 handles");
  DeviceGuard g(h->device);
  int rc = sticky_error();
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  h->tape_T = 0;
  HIP_TRY(hipEventRecord(h->ev0, st));
  HIP_TRY(launch_dyn_rollout(h->dc, h->b, actions, actions_per_step ? NA : 0, T, rewards, dones,
                             states, st));
  HIP_TRY(hipEventRecord(h->ev1, st));
  h->last_launches = 1;
  h->timing_valid = true;
  return SIM_OK;
}

int sim_last_rollout_timing(sim_handle* h, float* ms_per_launch, int* launches) {
  if (!h) return fail(SIM_E_INVAL, "handle is NULL");
  if (!h->timing_valid) return fail(SIM_E_STATE, "no rollout timed yet");
  DeviceGuard g(h->device);
  float ms = 0;
  HIP_TRY(hipEventSynchronize(h->ev1));
  HIP_TRY(hipEventElapsedTime(&ms, h->ev0, h->ev1));
  if (ms_per_launch) *ms_per_launch = h->last_launches ? ms / h->last_launches : ms;
  if (launches) *launches = h->last_launches;
  return SIM_OK;
}

int sim_backward(sim_handle* h, const float* actor, const float* d_rewards, const float* d_states,
                 float* grad_actor, float* grad_params, void* stream) {
  if (!h) return fail(SIM_E_INVAL, "handle is NULL");
  if (!actor) return fail(SIM_E_INVAL, "actor is NULL");
  if (h->tape_T <= 0) return fail(SIM_E_STATE, "no taped rollout to differentiate");
  DeviceGuard g(h->device);
  int rc = sticky_error();
  if (rc) return rc;
  // seg_held is brought up to date with the buffers the recomputes reuse
  HIP_TRY(run_backward(h->dc, h->b, h->bw, actor, h->tape, h->cfg.ckpt_every, h->tape_T, d_rewards,
                       d_states, grad_actor, grad_params, h->seg_held, (hipStream_t)stream));
  return SIM_OK;
}

int sim_backward_noalloc(sim_handle* h, const float* actor, const float* d_rewards,
                         const float* d_states, float* grad_actor, float* grad_params,
                         void* stream) {
  if (!h) return fail(SIM_E_INVAL, "handle is NULL");
  if (!actor) return fail(SIM_E_INVAL, "actor is NULL");
  if (h->tape_T <= 0) return fail(SIM_E_STATE, "no taped rollout to differentiate");
  const size_t need = bwd_scratch_floats(h->bw);
  if (need > NOALLOC_SCRATCH_FLOATS)
    return fail(SIM_E_INVAL,
                "backward of %d envs with checkpoints every %d steps needs %zu bytes of scratch, "
                "more than the %zu bytes of the static scratch array",
                h->N, h->cfg.ckpt_every, need * 4, NOALLOC_SCRATCH_FLOATS * 4);
  DeviceGuard g(h->device);
  int rc = sticky_error();
  if (rc) return rc;
  float* sp = (h->device >= 0 && h->device < MAX_DEVICES) ? g_scratch[h->device] : nullptr;
  if (!sp) return fail(SIM_E_STATE, "scratch array of device %d not set up", h->device);
  HIP_TRY(run_backward_in(h->dc, h->b, h->bw, sp, actor, h->tape, h->cfg.ckpt_every, h->tape_T,
                          d_rewards, d_states, grad_actor, grad_params, (hipStream_t)stream));
  return SIM_OK;
}

int sim_get_state(sim_handle* h, float* state, float* hist, int32_t* t_ep, int32_t* episode,
                  float* returns, int32_t* last_len, void* stream) {
  if (!h) return fail(SIM_E_INVAL, "handle is NULL");
  DeviceGuard g(h->device);
  int rc = sticky_error();
  if (rc) return rc;
  if (h->fp64) {
    HIP_TRY(precise_get(h->pb, h->N, state, hist, t_ep, episode, nullptr, returns, last_len,
                        (hipStream_t)stream));
    return SIM_OK;
  }
  HIP_TRY(launch_get_state(h->b, h->N, state, hist, t_ep, episode, returns, last_len,
                           (hipStream_t)stream));
  return SIM_OK;
}

int sim_set_state(sim_handle* h, const float* state, const float* hist, const int32_t* t_ep,
                  const int32_t* episode, const float* returns, const int32_t* last_len,
                  void* stream) {
  if (!h) return fail(SIM_E_INVAL, "handle is NULL");
  DeviceGuard g(h->device);
  int rc = sticky_error();
  if (rc) return rc;
  h->tape_T = 0;
  if (h->fp64) {
    HIP_TRY(precise_set(h->pb, h->N, state, hist, t_ep, episode, nullptr, returns, last_len,
                        (hipStream_t)stream));
    return SIM_OK;
  }
  HIP_TRY(launch_set_state(h->b, h->N, state, hist, t_ep, episode, returns, last_len,
                           (hipStream_t)stream));
  return SIM_OK;
}

int sim_set_reward(sim_handle* h, const double* C) {
  if (!h || !C) return fail(SIM_E_INVAL, "NULL argument");
  for (int i = 0; i < 7; ++i)
    if (!std::isfinite(C[i])) return fail(SIM_E_INVAL, "reward constant %d is not finite", i);
  DeviceGuard g(h->device);
  h->cfg.C_rp = C[0];
  h->cfg.C_rq = C[1];
  h->cfg.C_rv = C[2];
  h->cfg.C_rw = C[3];
  h->cfg.C_ra = C[4];
  h->cfg.C_rab = C[5];
  h->cfg.C_rs = C[6];
  h->dc = make_devcfg(h->cfg, h->cfg.seed);
  apply_target(h);
  if (h->fp64) h->pc = make_precise(h->cfg, h->cfg.seed);
  // captured graphs hold the old constants in their kernel arguments
  drop_graph(h);
  return SIM_OK;
}

int sim_set_target(sim_handle* h, const float* target, double pos_clip, double vel_clip,
                   void* stream) {
  if (!h) return fail(SIM_E_INVAL, "handle is NULL");
  if (h->fp64) return fail(SIM_E_UNSUPPORTED, "not available on SIM_F_FP64 handles");
  if (target && !(pos_clip > 0 && vel_clip > 0 && std::isfinite(pos_clip) && std::isfinite(vel_clip)))
    return fail(SIM_E_INVAL, "clip bounds must be finite and positive");
  DeviceGuard g(h->device);
  int rc = sticky_error();
  if (rc) return rc;
  if (target) {
    HIP_TRY(hipMemcpyAsync(h->target_buf, target, (size_t)h->N * 6 * 4, hipMemcpyDeviceToDevice,
                           (hipStream_t)stream));
    h->pos_clip = (float)pos_clip;
    h->vel_clip = (float)vel_clip;
  }
  h->target_on = target != nullptr;
  apply_target(h);
  h->tape_T = 0;
  // captured graphs hold the old configuration in their kernel arguments
  drop_graph(h);
  return SIM_OK;
}

int sim_reset_envs(sim_handle* h, const uint8_t* mask, void* stream) {
  if (!h || !mask) return fail(SIM_E_INVAL, "NULL argument");
  if (h->fp64) return fail(SIM_E_UNSUPPORTED, "not available on SIM_F_FP64 handles");
  DeviceGuard g(h->device);
  int rc = sticky_error();
  if (rc) return rc;
  h->tape_T = 0;
  HIP_TRY(launch_reset_envs(h->dc, h->b, mask, (hipStream_t)stream));
  return SIM_OK;
}

int sim_reward(sim_handle* h, const float* states, const float* actions, int32_t M,
               float* rewards, void* stream) {
  if (!h) return fail(SIM_E_INVAL, "handle is NULL");
  if (M < 0) return fail(SIM_E_INVAL, "M = %d < 0", M);
  if (M == 0) return SIM_OK;  // nothing is read or written
  if (!states || !actions || !rewards) return fail(SIM_E_INVAL, "NULL argument");
  DeviceGuard g(h->device);
  int rc = sticky_error();
  if (rc) return rc;
  HIP_TRY(launch_reward_batch(h->dc, states, actions, M, rewards, (hipStream_t)stream));
  return SIM_OK;
}

int sim_get_params(sim_handle* h, float* theta, void* stream) {
  if (!h || !theta) return fail(SIM_E_INVAL, "NULL argument");
  DeviceGuard g(h->device);
  int rc = sticky_error();
  if (rc) return rc;
  if (h->fp64) {
    HIP_TRY(precise_get(h->pb, h->N, nullptr, nullptr, nullptr, nullptr, theta, nullptr,
                        nullptr, (hipStream_t)stream));
    return SIM_OK;
  }
  HIP_TRY(hipMemcpyAsync(theta, h->b.theta, (size_t)h->N * NP * 4, hipMemcpyDeviceToDevice,
                         (hipStream_t)stream));
  return SIM_OK;
}

int sim_set_params(sim_handle* h, const float* theta, void* stream) {
  if (!h || !theta) return fail(SIM_E_INVAL, "NULL argument");
  DeviceGuard g(h->device);
  int rc = sticky_error();
  if (rc) return rc;
  h->tape_T = 0;
  if (h->fp64) {
    HIP_TRY(precise_set(h->pb, h->N, nullptr, nullptr, nullptr, nullptr, theta, nullptr,
                        nullptr, (hipStream_t)stream));
    return SIM_OK;
  }
  HIP_TRY(hipMemcpyAsync(h->b.theta, theta, (size_t)h->N * NP * 4, hipMemcpyDeviceToDevice,
                         (hipStream_t)stream));
  return SIM_OK;
}

int sim_set_variant(sim_handle* h, int variant, int steps_per_launch, int use_graph) {
  if (!h) return fail(SIM_E_INVAL, "handle is NULL");
  if (variant < SIM_V_AUTO || variant > SIM_V_FUSED_SPLIT)
    return fail(SIM_E_INVAL, "unknown variant %d", variant);
  if (steps_per_launch < 0) return fail(SIM_E_INVAL, "steps_per_launch < 0");
  if (h->bf16 && variant != SIM_V_AUTO && variant != SIM_V_FUSED_MFMA4 &&
      variant != SIM_V_FUSED_MFMA)
    return fail(SIM_E_UNSUPPORTED,
                "SIM_F_ACTOR_BF16 handles run the matrix-core kernels (SIM_V_FUSED_MFMA, "
                "SIM_V_FUSED_MFMA4) only");
  h->variant = variant;
  h->spl = steps_per_launch;
  h->use_graph = use_graph ? 1 : 0;
  DeviceGuard g(h->device);
  drop_graph(h);
  return SIM_OK;
}

int sim_get_variant(const sim_handle* h, int* variant, int* steps_per_launch, int* use_graph) {
  if (!h) return fail(SIM_E_INVAL, "handle is NULL");
  if (variant) *variant = effective_variant(h);
  if (steps_per_launch) *steps_per_launch = effective_spl(h);
  if (use_graph) *use_graph = h->use_graph;
  return SIM_OK;
}

int sim_autotune(sim_handle* h, const float* actor, int32_t T, void* stream, int* variant_out,
                 float* ms_out) {
  if (!h) return fail(SIM_E_INVAL, "handle is NULL");
  if (!actor || T < 1) return fail(SIM_E_INVAL, "need actor and T >= 1");
  if (h->fp64) return fail(SIM_E_UNSUPPORTED, "SIM_F_FP64 handles have a single variant");
  DeviceGuard g(h->device);
  int rc = sticky_error();
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  const size_t N = (size_t)h->N;
  // Snapshot so every candidate starts from the same state and the caller's
  // state is restored afterwards.  The snapshot is freed, and the caller's
  // variant restored, on every way out (the guards' destructors run in
  // reverse order: variant first, then the buffers once the stream is idle).
  struct Snapshot {
    hipStream_t st;
    float *state = nullptr, *hist = nullptr, *ret = nullptr;
    int32_t *tep = nullptr, *ep = nullptr, *len = nullptr;
    ~Snapshot() {
      (void)hipStreamSynchronize(st);
      (void)hipFree(state);
      (void)hipFree(hist);
      (void)hipFree(ret);
      (void)hipFree(tep);
      (void)hipFree(ep);
      (void)hipFree(len);
    }
  } snap{st};
  struct VariantRestore {
    sim_handle* h;
    int v, spl;
    ~VariantRestore() {
      h->variant = v;
      h->spl = spl;
      h->tape_T = 0;
      drop_graph(h);
    }
  } restore{h, h->variant, h->spl};
  HIP_TRY(hipMalloc(&snap.state, N * NS * 4));
  HIP_TRY(hipMalloc(&snap.hist, N * NH * NA * 4));
  HIP_TRY(hipMalloc(&snap.tep, N * 4));
  HIP_TRY(hipMalloc(&snap.ep, N * 4));
  HIP_TRY(hipMalloc(&snap.ret, N * 2 * 4));
  HIP_TRY(hipMalloc(&snap.len, N * 4));
  HIP_TRY(launch_get_state(h->b, h->N, snap.state, snap.hist, snap.tep, snap.ep, snap.ret,
                           snap.len, st));
  struct Cand { int v, spl; };
  std::vector<Cand> cands = {{SIM_V_FUSED_MFMA4, 0}, {SIM_V_FUSED_MFMA, 0},
                             {SIM_V_FUSED_SPLIT, 0}, {SIM_V_FUSED_MFMA4, 100},
                             {SIM_V_FUSED_MFMA, 100}, {SIM_V_FUSED_SPLIT, 100},
                             {SIM_V_FUSED_VALU, 0},  {SIM_V_PLAIN, 0}};
  if (h->bf16)
    cands = {{SIM_V_FUSED_MFMA4, 0}, {SIM_V_FUSED_MFMA, 0}, {SIM_V_FUSED_MFMA4, 100},
             {SIM_V_FUSED_MFMA, 100}};
  float best = 1e30f;
  Cand bestc = cands[0];
  for (const Cand& cd : cands) {
    if (cd.spl >= T) continue;
    h->variant = cd.v;
    h->spl = cd.spl;
    drop_graph(h);
    float acc = 0;
    for (int rep = 0; rep < 3; ++rep) {
      HIP_TRY(launch_set_state(h->b, h->N, snap.state, snap.hist, snap.tep, snap.ep, snap.ret,
                               snap.len, st));
      rc = sim_rollout(h, actor, T, nullptr, nullptr, nullptr, 0, stream);
      if (rc) return rc;
      HIP_TRY(hipEventSynchronize(h->ev1));
      float ms = 0;
      HIP_TRY(hipEventElapsedTime(&ms, h->ev0, h->ev1));
      if (rep > 0) acc += ms;  // first run warms up (and captures the graph)
    }
    const float ms = acc / 2;
    if (ms < best) {
      best = ms;
      bestc = cd;
    }
  }
  HIP_TRY(launch_set_state(h->b, h->N, snap.state, snap.hist, snap.tep, snap.ep, snap.ret,
                               snap.len, st));
  h->tuned_variant = bestc.v;
  h->tuned_spl = bestc.spl;
  if (variant_out) *variant_out = bestc.v;
  if (ms_out) *ms_out = best;
  return SIM_OK;
}

}  // extern "C"
