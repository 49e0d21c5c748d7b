"""Pins for the FP64 oracle: closed forms, invariants, library routines and
brute force, each chosen so that a plausible slip in the oracle (a dropped
term, a sign, a transposed index, a wrong RK4 weight) fails one of them.

None of these tests touches the GPU library.
"""
import math
import os

import numpy as np
import pytest

import workloads as wl

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def orc(oracle_lib):
    return oracle_lib


def base_cfg(**kw):
    return wl.crazyflie_config(**kw)


def state(p=(0, 0, 0), q=(1, 0, 0, 0), v=(0, 0, 0), w=(0, 0, 0), wm=(0, 0, 0, 0)):
    return np.array(list(p) + list(q) + list(v) + list(w) + list(wm), np.float64)


def nominal(cfg):
    return np.array(cfg["nominal"], np.float64)


def rpm_to_action(cfg, rpm):
    return 2.0 * (np.asarray(rpm) - cfg["rpm_min"]) / (cfg["rpm_max"] - cfg["rpm_min"]) - 1.0


def one_env(orc, cfg, s, a_seq, theta=None, H=None):
    """Open-loop rollout of one env with external actions [T][4]."""
    b = orc.Batch(cfg, 1)
    b.theta[0] = nominal(cfg) if theta is None else theta
    b.s[0] = s
    if H is not None:
        b.H[0] = H
    a = np.asarray(a_seq, np.float64).reshape(len(a_seq), 1, 4)
    out = b.rollout(None, len(a_seq), actions=a, record=True)
    return out["states"][:, 0, :], out


# --------------------------------------------------------------------------- #
# P14: counter RNG                                                              #
# --------------------------------------------------------------------------- #

def test_philox_known_answers(orc):
    """Philox4x32-10 reproduces the generator's published known-answer vectors."""
    n = 0
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            out = orc.philox4x32_10(v[0:4], v[4:6])
            assert [int(x) for x in out] == v[6:10]
            n += 1
    assert n == 3


def test_uniforms_exact_and_in_range(orc):
    """u = (2k+1) 2^-24 with k the top 23 bits: strictly inside (0,1), exactly
    representable in float32, mean 1/2 and variance 1/12 over many draws."""
    us = np.array([orc.uniforms(7, e, 3, b, 0) for e in range(400) for b in range(4)]).ravel()
    assert np.all(us > 0) and np.all(us < 1)
    assert np.all(us.astype(np.float32).astype(np.float64) == us)
    k = us * 2 ** 24
    assert np.all(np.abs(k - np.round(k)) == 0) and np.all(np.round(k) % 2 == 1)
    assert abs(us.mean() - 0.5) < 0.02
    assert abs(us.var() - 1 / 12) < 0.01
    # distinct streams / counters give distinct draws
    assert not np.array_equal(orc.uniforms(7, 0, 0, 0, 0), orc.uniforms(7, 0, 0, 0, 1))
    assert not np.array_equal(orc.uniforms(7, 0, 0, 0, 0), orc.uniforms(8, 0, 0, 0, 0))


def test_domain_randomisation_ranges(orc):
    cfg = base_cfg(dr_enable=1)
    b = orc.Batch.init(cfg, 2000)
    with np.errstate(divide="ignore", invalid="ignore"):
        f = b.theta / nominal(cfg)[None, :]
    idx = [0, 1, 2, 3, 6, 7]   # c0 = c1 = 0 nominally
    lo = np.array(cfg["dr_lo"])[idx]
    hi = np.array(cfg["dr_hi"])[idx]
    assert np.all(f[:, idx] >= lo) and np.all(f[:, idx] <= hi)
    # uniform: means near the interval centre, spread close to the full range
    assert np.all(np.abs(f[:, idx].mean(0) - (lo + hi) / 2) < 0.02 * (hi - lo) + 0.01)
    assert np.all(f[:, idx].max(0) - f[:, idx].min(0) > 0.95 * (hi - lo))
    # factors are independent across parameters
    cc = np.corrcoef(f[:, idx].T)
    assert np.all(np.abs(cc - np.eye(len(idx))) < 0.1)
    # no randomisation when disabled
    b0 = orc.Batch.init(base_cfg(dr_enable=0), 10)
    assert np.all(b0.theta == nominal(cfg)[None, :])


def test_reset_distribution(orc):
    cfg = base_cfg()
    n = 4000
    b = orc.Batch.init(cfg, n)
    s = b.s
    assert np.all(np.abs(s[:, 0:3]) <= cfg["init_pos"])
    qn = np.linalg.norm(s[:, 3:7], axis=1)
    assert np.all(np.abs(qn - 1) < 1e-14)
    # rotation angle 2 acos(w) uniform in [0, pi/2]
    ang = 2 * np.arccos(np.clip(s[:, 3], -1, 1))
    assert ang.max() <= cfg["init_angle"] + 1e-12 and ang.min() >= 0
    assert abs(ang.mean() - cfg["init_angle"] / 2) < 0.03
    # axis uniform on the sphere: mean ~0, second moments ~1/3
    ax = s[:, 4:7] / np.maximum(np.linalg.norm(s[:, 4:7], axis=1, keepdims=True), 1e-300)
    assert np.all(np.abs(ax.mean(0)) < 0.05)
    assert np.all(np.abs((ax ** 2).mean(0) - 1 / 3) < 0.03)
    assert np.all(np.abs(s[:, 7:10]) <= cfg["init_vel"])
    assert np.all(np.abs(s[:, 10:13]) <= cfg["init_angvel"])
    wh = math.sqrt(0.027 * 9.81 / 4 / 3.16e-10)
    assert np.allclose(s[:, 13:17], wh, rtol=1e-14)
    assert np.allclose(b.H, rpm_to_action(cfg, wh), rtol=1e-14)
    # deterministic per seed, different for another seed
    b2 = orc.Batch.init(cfg, n)
    assert np.array_equal(b.s, b2.s)
    b3 = orc.Batch.init(base_cfg(seed=99), n)
    assert not np.array_equal(b.s, b3.s)


# --------------------------------------------------------------------------- #
# P11 rotation matrix, P9 actor                                                 #
# --------------------------------------------------------------------------- #

def test_rotmat_matches_library_and_invariants(orc):
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(3)
    for _ in range(50):
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        R = orc.rotmat(q)
        # scipy: scalar-last quaternion, active rotation (body -> world)
        Rs = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        assert np.allclose(R, Rs, atol=1e-14)
        assert np.allclose(R.T @ R, np.eye(3), atol=1e-14)
        assert abs(np.linalg.det(R) - 1) < 1e-14
        assert np.allclose(orc.rotmat(-q), R, atol=1e-15)   # double cover
        assert np.allclose(orc.rotmat(3.7 * q), R, atol=1e-14)  # normalised inside


def test_observation_layout(orc):
    rng = np.random.default_rng(4)
    s = rng.normal(size=17)
    H = rng.uniform(-1, 1, size=(32, 4))
    o = orc.observe(s, H)
    assert o.shape == (146,)
    assert np.array_equal(o[0:3], s[0:3])
    assert np.allclose(o[3:12], orc.rotmat(s[3:7]).ravel(), atol=1e-15)
    assert np.array_equal(o[12:15], s[7:10])
    assert np.array_equal(o[15:18], s[10:13])
    assert np.array_equal(o[18:], H.ravel())


def test_actor_matches_numpy(orc):
    W = wl.random_actor(11).astype(np.float64)
    rng = np.random.default_rng(5)
    i = 0
    W1 = W[i:i + 64 * 146].reshape(64, 146); i += 64 * 146
    b1 = W[i:i + 64]; i += 64
    W2 = W[i:i + 64 * 64].reshape(64, 64); i += 64 * 64
    b2 = W[i:i + 64]; i += 64
    W3 = W[i:i + 4 * 64].reshape(4, 64); i += 4 * 64
    b3 = W[i:i + 4]; i += 4
    assert i == wl.NACTOR
    for _ in range(20):
        o = rng.normal(size=146)
        ref = np.tanh(W3 @ np.maximum(W2 @ np.maximum(W1 @ o + b1, 0) + b2, 0) + b3)
        assert np.allclose(orc.actor(W, o), ref, rtol=1e-13, atol=1e-15)


# --------------------------------------------------------------------------- #
# P10 reward                                                                    #
# --------------------------------------------------------------------------- #

def test_reward_hand_values(orc):
    cfg = base_cfg()
    ab = cfg["C_rab"]
    # at the origin, level, still, hover action: survival constant only
    assert orc.reward(cfg, state(), [ab] * 4) == pytest.approx(1.0, abs=1e-15)
    # position 0.1 along x: -1 * 0.01
    assert orc.reward(cfg, state(p=(0.1, 0, 0)), [ab] * 4) == pytest.approx(0.99, abs=1e-15)
    # upside down about x (q_w = 0): -C_rq
    assert orc.reward(cfg, state(q=(0, 1, 0, 0)), [ab] * 4) == pytest.approx(0.0, abs=1e-15)
    # 90 degrees about z: q_w^2 = 1/2
    h = math.sqrt(0.5)
    assert orc.reward(cfg, state(q=(h, 0, 0, h)), [ab] * 4) == pytest.approx(0.5, abs=1e-15)
    # velocity (1,2,2): |v|^2 = 9 -> -0.9; angular velocity (3,0,4): 25 -> -0.25
    assert orc.reward(cfg, state(v=(1, 2, 2)), [ab] * 4) == pytest.approx(0.1, abs=1e-14)
    assert orc.reward(cfg, state(w=(3, 0, 4)), [ab] * 4) == pytest.approx(0.75, abs=1e-14)
    # action offset: a = C_rab + (1, -1, 0.5, 0) -> |.|^2 = 2.25 -> -0.0225
    a = np.array([ab + 1, ab - 1, ab + 0.5, ab])
    assert orc.reward(cfg, state(), a) == pytest.approx(1 - 0.0225, abs=1e-15)
    # q and -q give the same reward
    rng = np.random.default_rng(6)
    for _ in range(10):
        s = rng.normal(size=17)
        a = rng.uniform(-1, 1, 4)
        s2 = s.copy()
        s2[3:7] *= -1
        assert orc.reward(cfg, s, a) == orc.reward(cfg, s2, a)


# --------------------------------------------------------------------------- #
# P1 hover, P2 free fall, P3 motor step, P7 yaw spin-up                          #
# --------------------------------------------------------------------------- #

def test_hover_equilibrium(orc):
    """Level, still, rotors at the hover speed commanding the hover speed: the
    state does not move (thrust = m g, no torque, motors at set point)."""
    for cfg, theta in [
        (base_cfg(), None),
        # a randomised body with non-zero c0, c1 exercises the full thrust curve
        (base_cfg(nominal=[0.031, 4.1e-6, 3.7e-6, 6.2e-6, 0.004, 2.1e-6, 2.9e-10, 0.11]), None),
    ]:
        th = nominal(cfg) if theta is None else theta
        wh = orc.hover_rpm(cfg, th)
        T = th[4] + th[5] * wh + th[6] * wh * wh
        assert 4 * T == pytest.approx(th[0] * cfg["g"], rel=1e-14)
        s0 = state(p=(0.1, -0.2, 0.3), wm=(wh,) * 4)
        a = [rpm_to_action(cfg, wh)] * 4
        S, _ = one_env(orc, cfg, s0, [a] * 200)
        assert np.allclose(S, s0[None, :], rtol=0, atol=1e-11 * np.maximum(1, np.abs(s0)))


def test_thrust_acts_along_body_z(orc):
    """The collective thrust F = sum(c0 + c1 w + c2 w^2) accelerates the body
    along its own z axis, the third column of the library rotation matrix
    (body to world): dv/dt = F/m R e_z - g e_z, for any attitude and rotor
    speeds.  Worked case: a body rolled by +30 degrees about x pushes towards
    -y with F/m sin 30."""
    from scipy.spatial.transform import Rotation
    cfg = base_cfg()
    th = np.array([0.031, 4.1e-6, 3.7e-6, 6.2e-6, 0.004, 2.1e-6, 2.9e-10, 0.11])
    rng = np.random.default_rng(21)
    for _ in range(20):
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        wm = rng.uniform(3000, 20000, size=4)
        x = state(q=q, wm=wm)
        dx = orc.dynamics(cfg, th, x, wm)
        F = np.sum(th[4] + th[5] * wm + th[6] * wm * wm)
        ez = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()[:, 2]
        want = F / th[0] * ez - np.array([0.0, 0.0, cfg["g"]])
        assert np.allclose(dx[7:10], want, rtol=1e-13, atol=1e-13)
    phi = math.radians(30.0)
    wm = np.full(4, 15000.0)
    x = state(q=(math.cos(phi / 2), math.sin(phi / 2), 0.0, 0.0), wm=wm)
    dx = orc.dynamics(cfg, th, x, wm)
    F = 4 * (th[4] + th[5] * 15000.0 + th[6] * 15000.0 ** 2)
    assert dx[7] == pytest.approx(0.0, abs=1e-15)
    assert dx[8] == pytest.approx(-F / th[0] * math.sin(phi), rel=1e-13)
    assert dx[9] == pytest.approx(F / th[0] * math.cos(phi) - cfg["g"], rel=1e-13)


def test_history_push_order(orc):
    """Each step appends its action as the newest of the 32 history slots and
    drops the oldest: after T < 32 steps with given actions a_0 .. a_{T-1}
    the history is the start history's last 32 - T slots followed by
    a_0 .. a_{T-1}, and the observation shows it oldest first."""
    cfg = base_cfg(max_episode_steps=0)
    rng = np.random.default_rng(22)
    H0 = rng.uniform(-1, 1, size=(32, 4))
    A = rng.uniform(-1, 1, size=(5, 4))
    s0 = state(wm=(14000.0,) * 4)
    b = orc.Batch(cfg, 1)
    b.theta[0] = nominal(cfg)
    b.s[0] = s0
    b.H[0] = H0
    b.rollout(None, 5, actions=A.reshape(5, 1, 4))
    want = np.concatenate([H0[5:], A])
    assert np.array_equal(b.H[0], want)
    assert np.array_equal(orc.observe(b.s[0], b.H[0])[18:], want.ravel())


def test_free_fall_exact_under_rk4(orc):
    """No thrust: p(t) = p0 + v0 t - g t^2/2 e_z exactly (RK4 is exact for
    polynomials of degree <= 4); attitude and rotors unchanged."""
    cfg = base_cfg()
    s0 = state(p=(0.1, 0.2, 0.3), v=(0.5, -0.25, 1.0), q=(math.cos(0.3), 0, math.sin(0.3), 0))
    n = 100
    S, _ = one_env(orc, cfg, s0, [[-1.0] * 4] * n)
    t = np.arange(n + 1) * cfg["dt"]
    g = cfg["g"]
    p = s0[0:3][None, :] + s0[7:10][None, :] * t[:, None]
    p[:, 2] -= 0.5 * g * t ** 2
    v = np.tile(s0[7:10], (n + 1, 1))
    v[:, 2] -= g * t
    assert np.allclose(S[:, 0:3], p, rtol=0, atol=1e-13)
    assert np.allclose(S[:, 7:10], v, rtol=0, atol=1e-13)
    assert np.allclose(S[:, 3:7], s0[3:7][None, :], atol=1e-15)
    assert np.all(S[:, 13:17] == 0)


def test_motor_first_order_step(orc):
    """Motor speeds obey the RK4 discretisation of a first-order lag exactly:
    w(n) = u + (w0 - u) rho^n with rho = 1 - h + h^2/2 - h^3/6 + h^4/24,
    h = dt/T_m; and reach 1 - 1/e ~ 63 % of a step at t = T_m (Sec. IV)."""
    cfg = base_cfg()
    Tm = cfg["nominal"][7]
    h = cfg["dt"] / Tm
    rho = 1 - h + h * h / 2 - h ** 3 / 6 + h ** 4 / 24
    u = np.array([3000.0, 9000.0, 15000.0, 21000.0])
    a = rpm_to_action(cfg, u)
    n = 40
    s0 = state(wm=(0, 0, 0, 0))
    S, _ = one_env(orc, cfg, s0, [a] * n)
    k = np.arange(n + 1)[:, None]
    ref = u[None, :] * (1 - rho ** k)
    assert np.allclose(S[:, 13:17], ref, rtol=1e-13, atol=1e-9)
    steps_Tm = round(Tm / cfg["dt"])
    frac = S[steps_Tm, 13:17] / u
    assert np.allclose(frac, 1 - math.exp(-1), atol=2e-7)


def test_yaw_spin_up_linear(orc):
    """Balanced roll/pitch torque with net reaction torque: w_z grows linearly
    as tau_z t / Jzz with tau_z = k_m (-T0 + T1 - T2 + T3), w_x = w_y = 0."""
    cfg = base_cfg()
    th = nominal(cfg)
    wa, wb = 12000.0, 16000.0        # rotors 0,2 and 1,3
    Ta, Tb = th[6] * wa ** 2, th[6] * wb ** 2
    tau_z = cfg["k_m"] * (-Ta + Tb - Ta + Tb)
    u = np.array([wa, wb, wa, wb])
    a = rpm_to_action(cfg, u)
    s0 = state(wm=tuple(u))
    n = 50
    S, _ = one_env(orc, cfg, s0, [a] * n)
    t = np.arange(n + 1) * cfg["dt"]
    assert np.allclose(S[:, 12], tau_z * t / th[3], rtol=1e-12, atol=1e-12)
    assert np.all(np.abs(S[:, 10:12]) < 1e-12)
    # reversing the pair speeds reverses the spin
    s1 = state(wm=(wb, wa, wb, wa))
    S1, _ = one_env(orc, cfg, s1, [rpm_to_action(cfg, [wb, wa, wb, wa])] * n)
    assert np.allclose(S1[:, 12], -S[:, 12], rtol=1e-12, atol=1e-12)


def test_roll_pitch_torque_signs(orc):
    """Speeding up rotors 2,3 (at +y) rolls about +x; rotors 1,2 (at -x)
    pitch about +y (tau = r x F with F along body z)."""
    cfg = base_cfg()
    th = nominal(cfg)
    wh = orc.hover_rpm(cfg, th)
    for fast, axis in (((2, 3), 0), ((1, 2), 1)):
        wm = [wh] * 4
        for i in fast:
            wm[i] = wh * 1.05
        s0 = state(wm=tuple(wm))
        S, _ = one_env(orc, cfg, s0, [rpm_to_action(cfg, wm)])
        assert S[1, 10 + axis] > 0
        other = 1 - axis
        assert abs(S[1, 10 + other]) < 1e-9 * abs(S[1, 10 + axis])


# --------------------------------------------------------------------------- #
# P4 torque-free symmetric body, P5 quaternion norm, P6 RK4 order                #
# --------------------------------------------------------------------------- #

def _torque_free_cfg(**kw):
    nom = [0.027, 3.85e-6, 3.85e-6, 5.9675e-6, 0.0, 0.0, 0.0, 0.15]   # no thrust at all
    return base_cfg(nominal=nom, **kw)


def test_torque_free_symmetric_body(orc):
    """Jxx = Jyy, no torque: w_z constant and (w_x + i w_y) multiplies by the
    RK4 stability polynomial R4(i lambda dt) each step, lambda = (Jzz-Jxx)/Jxx
    w_z; kinetic energy and world angular momentum are conserved up to the
    RK4 truncation error."""
    cfg = _torque_free_cfg()
    th = nominal(cfg)
    w0 = np.array([3.0, -2.0, 7.0])
    s0 = state(w=tuple(w0))
    n = 300
    S, _ = one_env(orc, cfg, s0, [[-1.0] * 4] * n)
    assert np.allclose(S[:, 12], w0[2], rtol=1e-14)
    lam = (th[3] - th[1]) / th[1] * w0[2]
    z = 1j * lam * cfg["dt"]
    R4 = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
    c = (w0[0] + 1j * w0[1]) * R4 ** np.arange(n + 1)
    assert np.allclose(S[:, 10], c.real, rtol=0, atol=1e-12)
    assert np.allclose(S[:, 11], c.imag, rtol=0, atol=1e-12)
    # conservation laws (approximate): energy and world-frame momentum
    J = np.diag(th[1:4])
    E = np.array([0.5 * s[10:13] @ J @ s[10:13] for s in S])
    L = np.array([orc.rotmat(s[3:7]) @ J @ s[10:13] for s in S])
    assert np.max(np.abs(E - E[0])) / E[0] < 1e-6
    assert np.max(np.linalg.norm(L - L[0], axis=1)) / np.linalg.norm(L[0]) < 1e-5


def test_torque_free_momentum_error_is_fourth_order(orc):
    """World angular momentum drift shrinks ~16x per halving of dt."""
    w0 = (3.0, -2.0, 7.0)
    errs = []
    for dt in (0.02, 0.01, 0.005):
        cfg = _torque_free_cfg(dt=dt, flags=0)
        th = nominal(cfg)
        n = int(round(1.0 / dt))
        S, _ = one_env(orc, cfg, state(w=w0), [[-1.0] * 4] * n)
        J = np.diag(th[1:4])
        L0 = J @ np.array(w0)
        Lend = orc.rotmat(S[-1, 3:7]) @ J @ S[-1, 10:13]
        errs.append(np.linalg.norm(Lend - L0) / np.linalg.norm(L0))
    r = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(3.5 < x < 4.5 for x in r), (errs, r)


def test_quaternion_norm(orc):
    """Without renormalisation |q| drifts at the RK4 truncation level; for a
    norm-preserving flow q' = Omega(w) q with Omega skew, RK4 changes the norm
    by O(dt^6) per step, so over a fixed time the drift falls 2^5 = 32x per
    halving of dt.  With renormalisation, |q| = 1 to rounding."""
    w0 = (3.0, -2.0, 7.0)
    drift = []
    for dt in (0.01, 0.005):
        cfg = _torque_free_cfg(dt=dt, flags=0)
        n = int(round(5.0 / dt))
        S, _ = one_env(orc, cfg, state(w=w0), [[-1.0] * 4] * n)
        drift.append(np.max(np.abs(np.linalg.norm(S[:, 3:7], axis=1) - 1)))
    assert drift[0] > 1e-12
    assert 26 < drift[0] / drift[1] < 38
    cfg = _torque_free_cfg()
    S, _ = one_env(orc, cfg, state(w=w0), [[-1.0] * 4] * 500)
    assert np.max(np.abs(np.linalg.norm(S[:, 3:7], axis=1) - 1)) < 1e-15


def test_rk4_global_order_four(orc):
    """Open loop with constant non-hover set points for 1 s: the end-state
    error against a dt/256 reference falls ~16x per halving of dt."""
    base = base_cfg(flags=0)
    s0 = state(p=(0.1, 0, 0), q=(math.cos(0.2), math.sin(0.2), 0, 0), v=(0.3, 0.1, -0.2),
               w=(0.5, -0.4, 0.3), wm=(14000, 14500, 15000, 14200))
    u = np.array([15500.0, 13000.0, 14800.0, 14100.0])

    def run(dt):
        cfg = dict(base, dt=dt)
        a = rpm_to_action(cfg, u)
        n = int(round(1.0 / dt))
        S, _ = one_env(orc, cfg, s0, [a] * n)
        return S[-1]

    ref = run(0.02 / 256)
    scale = np.array([1] * 3 + [1] * 4 + [1] * 3 + [1] * 3 + [1000] * 4)
    errs = [np.max(np.abs(run(dt) - ref) / scale) for dt in (0.02, 0.01, 0.005, 0.0025)]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert all(3.7 <= r <= 4.3 for r in rates), (errs, rates)


# --------------------------------------------------------------------------- #
# Episode logic: termination box, truncation, reset                              #
# --------------------------------------------------------------------------- #

def test_termination_truncation_and_reset(orc):
    from workloads import F_AUTORESET, F_RENORM_Q, F_TERMINATE
    cfg = base_cfg(flags=F_TERMINATE | F_AUTORESET | F_RENORM_Q, max_episode_steps=5)
    b = orc.Batch.init(cfg, 5)
    wh = orc.hover_rpm(cfg, nominal(cfg))
    ah = rpm_to_action(cfg, wh)
    hov = state(wm=(wh,) * 4)
    b.s[:] = hov
    b.s[1, 0] = 0.61           # outside the position box
    b.s[2, 8] = -2.2            # outside the velocity box
    b.s[3, 5] = np.nan          # non-finite
    b.t_ep[4] = 4               # reaches the cap at the next step
    A = np.full((1, 5, 4), ah)
    s_before = b.s.copy()
    out = b.rollout(None, 1, actions=A)
    d = out["dones"][0]
    assert list(d) == [0, 1, 1, 1, 2]
    assert np.allclose(b.s[0], hov, atol=1e-11)
    assert b.t_ep.tolist() == [1, 0, 0, 0, 0]
    assert b.ep.tolist() == [0, 1, 1, 1, 1]
    # reset states are the episode-1 draws of those envs
    ref = orc.Batch(cfg, 5)
    ref.theta[:] = nominal(cfg)
    lib = orc.lib()
    import ctypes
    eps = np.ones(5, np.int32)
    lib.orc_reset_state(ctypes.byref(ref.c), 5, None, orc._p(eps), orc._p(ref.theta),
                        orc._p(ref.s), orc._p(ref.H))
    for i in (1, 2, 3, 4):
        assert np.array_equal(b.s[i], ref.s[i])
        assert np.array_equal(b.H[i], ref.H[i])
    assert not np.array_equal(b.s[1], s_before[1])
    # reward of a terminated transition is still reported (finite for 1, 2)
    assert np.isfinite(out["rewards"][0, 1]) and np.isfinite(out["rewards"][0, 2])


def test_no_termination_flag_keeps_going(orc):
    cfg = base_cfg(flags=4, max_episode_steps=0)
    b = orc.Batch.init(cfg, 2)
    b.s[0, 0] = 5.0
    out = b.rollout(None, 3, actions=np.zeros((3, 2, 4)))
    assert np.all(out["dones"] == 0)
    assert b.ep.tolist() == [0, 0]


# --------------------------------------------------------------------------- #
# P8: batch = brute force, thread and permutation invariance                    #
# --------------------------------------------------------------------------- #

def test_batch_equals_single_env_runs(orc):
    from workloads import F_AUTORESET, F_RENORM_Q, F_TERMINATE
    cfg = base_cfg(flags=F_TERMINATE | F_AUTORESET | F_RENORM_Q, dr_enable=1, max_episode_steps=40)
    W = wl.xavier_actor(0)
    n, T = 8, 120
    b = orc.Batch.init(cfg, n)
    full = b.rollout(W, T, record=True)
    for i in range(n):
        bi = orc.Batch.init(cfg, 1, ids=[i])
        oi = bi.rollout(W, T, record=True)
        assert np.array_equal(oi["states"][:, 0], full["states"][:, i])
        assert np.array_equal(oi["rewards"][:, 0], full["rewards"][:, i])
        assert np.array_equal(oi["dones"][:, 0], full["dones"][:, i])
    # a permutation of env ids permutes the results
    perm = np.array([5, 2, 7, 0, 1, 6, 3, 4])
    bp = orc.Batch.init(cfg, n, ids=perm)
    op = bp.rollout(W, T, record=True)
    assert np.array_equal(op["states"], full["states"][:, perm])
    # threads do not change results
    bt = orc.Batch.init(cfg, n)
    ot = bt.rollout(W, T, record=True, nthreads=3)
    assert np.array_equal(ot["states"], full["states"])
    assert full["dones"].any()   # the test exercised resets
