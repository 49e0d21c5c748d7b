"""Pins for the oracle's discrete adjoint: central finite differences of the
oracle's own forward loss (the definition of the derivative), and the
system-identification special case whose loss and gradient vanish exactly.
"""
import numpy as np
import pytest

import workloads as wl

def _setup(orc, n=4, T=16, seed=3, dr=1):
    cfg = wl.crazyflie_config(flags=wl.F_RENORM_Q, dr_enable=dr, max_episode_steps=0)
    b = orc.Batch.init(cfg, n)
    W = wl.random_actor(seed).astype(np.float64)
    rng = np.random.default_rng(seed)
    dR = rng.uniform(0.5, 1.5, size=(T, n))
    dS = rng.normal(size=(T + 1, n, 17)) * 1e-2
    dS[:, :, 13:17] *= 1e-4          # rotor speeds are ~1e4 RPM
    return cfg, b, W, dR, dS


def _param_scales(cfg, theta):
    """FD step scale per dynamics parameter: its value, or for parameters that
    are zero the size that makes the term comparable (c0 ~ m g / 4,
    c1 ~ m g / (4 w_hover))."""
    th = np.array(theta, np.float64)
    s = np.abs(th).copy()
    mg4 = th[0] * cfg["g"] / 4
    wh = np.sqrt(mg4 / th[6])
    if s[4] == 0:
        s[4] = mg4
    if s[5] == 0:
        s[5] = mg4 / wh
    return s


def test_adjoint_matches_central_fd_params(oracle_lib):
    orc = oracle_lib
    cfg, b, W, dR, dS = _setup(orc)
    T = dR.shape[0]
    J, gW, gth = b.grad(W, T, dR=dR, dS=dS)
    eps = 1e-6
    for i in range(b.n):
        sc = _param_scales(cfg, b.theta[i])
        fd = np.zeros(8)
        for k in range(8):
            h = eps * sc[k]
            bp = b.copy()
            bp.theta[i, k] += h
            bm = b.copy()
            bm.theta[i, k] -= h
            Jp, _, _ = bp.grad(W, T, dR=dR, dS=dS, want_grad=False)
            Jm, _, _ = bm.grad(W, T, dR=dR, dS=dS, want_grad=False)
            fd[k] = (Jp - Jm) / (2 * h)
        g = gth[i] * sc
        f = fd * sc
        err = np.linalg.norm(g - f) / np.linalg.norm(f)
        assert err < 1e-6, (i, err, g, f)


def test_adjoint_matches_central_fd_actor(oracle_lib):
    orc = oracle_lib
    cfg, b, W, dR, dS = _setup(orc, n=3, T=12, seed=5)
    T = dR.shape[0]
    J, gW, gth = b.grad(W, T, dR=dR, dS=dS)
    rng = np.random.default_rng(9)
    # every bias, plus a random sample of weights from each layer
    idx = list(range(9344, 9408)) + list(range(13504, 13568)) + list(range(13824, 13828))
    idx += list(rng.choice(9344, 60, replace=False))
    idx += list(9408 + rng.choice(4096, 30, replace=False))
    idx += list(13568 + rng.choice(256, 20, replace=False))
    eps = 1e-6
    fd = np.zeros(len(idx))
    for j, k in enumerate(idx):
        Wp = W.copy(); Wp[k] += eps
        Wm = W.copy(); Wm[k] -= eps
        Jp, _, _ = b.grad(Wp, T, dR=dR, dS=dS, want_grad=False)
        Jm, _, _ = b.grad(Wm, T, dR=dR, dS=dS, want_grad=False)
        fd[j] = (Jp - Jm) / (2 * eps)
    g = gW[idx]
    err = np.linalg.norm(g - fd) / np.linalg.norm(fd)
    assert err < 1e-6, err
    # the comparison is not vacuous
    assert np.linalg.norm(fd) > 1e-3


def test_loss_only_path_matches(oracle_lib):
    orc = oracle_lib
    cfg, b, W, dR, dS = _setup(orc, n=3, T=10)
    J1, _, _ = b.grad(W, 10, dR=dR, dS=dS, want_grad=False)
    J2, gW, _ = b.grad(W, 10, dR=dR, dS=dS)
    assert J1 == J2
    # with dR = ones and dS = 0 the loss is the summed reward of the rollout
    J3, _, _ = b.grad(W, 10, want_grad=False)
    bb = b.copy()
    out = bb.rollout(W, 10)
    assert J3 == pytest.approx(out["rewards"].sum(), rel=1e-13)


def test_threads_do_not_change_gradient(oracle_lib):
    orc = oracle_lib
    cfg, b, W, dR, dS = _setup(orc, n=6, T=8)
    J1, g1, t1 = b.grad(W, 8, dR=dR, dS=dS, nthreads=1)
    J2, g2, t2 = b.grad(W, 8, dR=dR, dS=dS, nthreads=1)
    assert np.array_equal(g1, g2) and np.array_equal(t1, t2)
    J3, g3, t3 = b.grad(W, 8, dR=dR, dS=dS, nthreads=3)
    assert np.array_equal(t1, t3)
    assert np.allclose(g1, g3, rtol=1e-12, atol=1e-15)


def test_sysid_zero_at_truth(oracle_lib):
    """Trajectory MSE against the same parameters: loss 0 and gradient 0
    exactly; a perturbed body gives a positive loss that decreases along the
    negative gradient."""
    orc = oracle_lib
    cfg = wl.crazyflie_config(flags=wl.F_RENORM_Q, dr_enable=1, max_episode_steps=0)
    n, T = 4, 20
    truth = orc.Batch.init(cfg, n)
    W = wl.xavier_actor(0).astype(np.float64)
    ref = truth.copy().rollout(W, T, record=True)["states"]      # [T+1][n][17]

    def mse_and_grad(theta):
        b = truth.copy()
        b.theta = theta.copy()
        S = b.copy().rollout(W, T, record=True)["states"]
        d = S[:, :, :13] - ref[:, :, :13]
        L = np.mean(d ** 2)
        dS = np.zeros_like(S)
        dS[:, :, :13] = 2 * d / d.size
        J, gW, gth = b.grad(W, T, dS=dS, dR=np.zeros((T, n)))
        return L, J, gth

    L0, J0, g0 = mse_and_grad(truth.theta)
    assert L0 == 0.0 and J0 == 0.0
    assert np.all(g0 == 0.0)
    rng = np.random.default_rng(3)
    delta = rng.uniform(-0.1, 0.1, size=truth.theta.shape)
    th = truth.theta * (1 + delta)
    L1, J1, g1 = mse_and_grad(th)
    assert L1 > 0
    sc = np.array([_param_scales(cfg, t) for t in truth.theta])
    step = -1e-3 * g1 * sc ** 2 / np.max(np.abs(g1 * sc))
    L2, _, _ = mse_and_grad(th + step)
    assert L2 < L1
