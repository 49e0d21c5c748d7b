"""Planted mistakes in the oracle.

Each mutant is a copy of the oracle's C source with one plausible slip (a
flipped sign, a dropped term or factor, a transposed or swapped index, a wrong
RK4 weight or stage, a wrong constant of the counter RNG), compiled with the
oracle's own flags on the CPU.  The oracle's pins (closed forms, invariants,
library routines, known-answer vectors, central differences) run against
each mutant in a child process and must fail on every one: this is what makes
them a check of the oracle and not a restatement of it.  A control build of
the unmodified source must pass the same run.

The replacement is applied to the first occurrence of the snippet; where the
forward function and its adjoint share a line (the thrust curve, the torque
sums), that is the forward function, which comes first in the source.  Such a
slip is also caught by the adjoint's central differences; the consistent
mutants below make the same slip in the forward step, in the differentiable
rollout's own forward and in the adjoint, so that only a pin of the forward
model itself can catch them.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_FILES = ["tests/test_oracle_pins.py", "tests/test_oracle_grad.py",
             "tests/test_oracle_extras.py"]

# (name, snippet of the oracle source, replacement)
MUTANTS = [
    # counter RNG and start states
    ("philox key schedule constant", "k0 += 0x9E3779B9u;", "k0 += 0xBB67AE85u;"),
    ("philox round count", "for (int r = 0; r < 10; ++r) {", "for (int r = 0; r < 7; ++r) {"),
    ("uniform mantissa shift", "((double)(x[i] >> 9) + 0.5)", "((double)(x[i] >> 8) + 0.5)"),
    ("reset tilt range doubled", "double alpha = c->init_angle * u[5];",
     "double alpha = 2.0 * c->init_angle * u[5];"),
    # rigid body and rotors
    ("rotation matrix entry sign", "R[1] = 2 * (x * y - w * z);", "R[1] = 2 * (x * y + w * z);"),
    ("thrust curve square dropped", "T[i] = c0 + c1 * wm[i] + c2 * wm[i] * wm[i];",
     "T[i] = c0 + c1 * wm[i] + c2 * wm[i];"),
    ("pitch torque sign", "tau[1] += -c->arm * RSX[i] * T[i];",
     "tau[1] += c->arm * RSX[i] * T[i];"),
    ("yaw torque sign", "tau[2] += c->k_m * RD[i] * T[i];", "tau[2] += -c->k_m * RD[i] * T[i];"),
    ("quaternion kinematics sign", "dx[4] = 0.5 * (q[0] * w[0] + q[2] * w[2] - q[3] * w[1]);",
     "dx[4] = 0.5 * (q[0] * w[0] - q[2] * w[2] + q[3] * w[1]);"),
    ("thrust along a row of R", "dx[7 + i] = (R[3 * i + 2] * F", "dx[7 + i] = (R[6 + i] * F"),
    ("gravity sign", "dx[9] -= c->g;", "dx[9] += c->g;"),
    ("gyroscopic term sign", "- cr[i]) / J[i];", "+ cr[i]) / J[i];"),
    ("motor constant multiplies", "dx[13 + i] = (u[i] - wm[i]) / Tm;",
     "dx[13 + i] = (u[i] - wm[i]) * Tm;"),
    # RK4
    ("RK4 weights", "(k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i])",
     "(k1[i] + 2.0 * k2[i] + k3[i] + 2.0 * k4[i])"),
    ("RK4 last stage at half step", "t[i] = x[i] + h * k3[i];", "t[i] = x[i] + 0.5 * h * k3[i];"),
    ("quaternion renormalisation skipped", "if (c->flags & F_RENORM_Q) {", "if (0) {"),
    # observation, actor, action map, reward, episode logic
    ("velocity and rate swapped in the observation", "o[12 + i] = s[7 + i];",
     "o[12 + i] = s[10 + i];"),
    ("history newest first", "o[18 + i] = H[i];", "o[18 + i] = H[NH * NA - 1 - i];"),
    ("first layer transposed", "acc += W[OFF_W1 + n * NO + k] * o[k];",
     "acc += W[OFF_W1 + k * NHID + n] * o[k];"),
    ("second ReLU dropped", "h2[n] = acc > 0.0 ? acc : 0.0;", "h2[n] = acc;"),
    ("action map half-width", "u[i] = c->rpm_min + 0.5 * (a[i] + 1.0) *",
     "u[i] = c->rpm_min + (a[i] + 1.0) *"),
    ("attitude reward on q_w, not q_w^2", "c->C_rq * (1.0 - s[3] * s[3])",
     "c->C_rq * (1.0 - s[3])"),
    ("velocity reward dropped", " - c->C_rv * vv", ""),
    ("history push at the oldest slot", "memcpy(H + (NH - 1) * NA, a, sizeof a);",
     "memcpy(H, a, sizeof a);"),
    ("position bound uses the velocity limit", "if (fabsf((float)sn[i]) > pl) term = 1;",
     "if (fabsf((float)sn[i]) > vl) term = 1;"),
    # adjoint
    ("gyroscopic VJP sign", "gx[11] += -hq[0] * (J[2] - J[1]) * w[2];",
     "gx[11] += hq[0] * (J[2] - J[1]) * w[2];"),
    ("RK4 VJP weight", "gk2[i] = h / 3.0 * g[i];", "gk2[i] = h / 6.0 * g[i];"),
    ("motor VJP sign", "gx[13 + i] += -gm[i] / Tm;", "gx[13 + i] += gm[i] / Tm;"),
    ("thrust curve VJP factor 2 dropped", "gx[13 + i] += gT[i] * (c1 + 2.0 * c2 * wm[i]);",
     "gx[13 + i] += gT[i] * (c1 + c2 * wm[i]);"),
    ("mass VJP power", "(R[3 * i + 2] * F + (d ? d[i] : 0.0)) / (m * m);",
     "(R[3 * i + 2] * F + (d ? d[i] : 0.0)) / m;"),
    ("ReLU mask dropped in the actor VJP", "gz1[n] = z1[n] > 0.0 ? gh1[n] : 0.0;",
     "gz1[n] = gh1[n];"),
    ("attitude reward VJP sign", "gs[3] += 2.0 * c->C_rq * s[3] * gr;",
     "gs[3] += -2.0 * c->C_rq * s[3] * gr;"),
    ("observation VJP index", "gs[7 + i] += go[12 + i];", "gs[7 + i] += go[15 + i];"),
]


# (name, [(snippet, replacement), ...]), every occurrence of each snippet
CONSISTENT = [
    ("thrust along a row of R, forward and adjoint", [("[3 * i + 2]", "[6 + i]")]),
    ("history push at the oldest slot, forward and adjoint", [
        ("memcpy(H + (NH - 1) * NA, a, sizeof a);", "memcpy(H, a, sizeof a);"),
        ("memcpy(Hn + (NH - 1) * NA, a, sizeof(double) * NA);", "memcpy(Hn, a, sizeof(double) * NA);"),
        ("ga[i] += lH[(NH - 1) * NA + i];", "ga[i] += lH[i];")]),
    ("gyroscopic term sign, forward and adjoint", [
        ("- cr[i]) / J[i];", "+ cr[i]) / J[i];"),
        ("- cr[i]) / (J[i] * J[i]);", "+ cr[i]) / (J[i] * J[i]);"),
        ("gx[11] += -hq[0]", "gx[11] += hq[0]"), ("gx[12] += -hq[0]", "gx[12] += hq[0]"),
        ("gx[12] += -hq[1]", "gx[12] += hq[1]"), ("gx[10] += -hq[1]", "gx[10] += hq[1]"),
        ("gx[10] += -hq[2]", "gx[10] += hq[2]"), ("gx[11] += -hq[2]", "gx[11] += hq[2]"),
        ("gth[3] += -hq[0]", "gth[3] += hq[0]"), ("gth[2] += hq[0]", "gth[2] += -hq[0]"),
        ("gth[1] += -hq[1]", "gth[1] += hq[1]"), ("gth[3] += hq[1]", "gth[3] += -hq[1]"),
        ("gth[2] += -hq[2]", "gth[2] += hq[2]"), ("gth[1] += hq[2]", "gth[1] += -hq[2]")]),
]


def _apply(src, edits):
    for old, new in edits:
        src = src.replace(old, new)
    return src


def _source():
    with open(os.path.join(ROOT, "oracle", "quad_oracle.c")) as f:
        return f.read()


def _run_pins(lib_path):
    env = dict(os.environ, QS_ORACLE_LIB=lib_path, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        *PIN_FILES], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    return r.returncode, r.stdout[-2000:]


def _build_and_run(tmp, idx, src):
    path = os.path.join(tmp, f"mutant{idx}.c")
    with open(path, "w") as f:
        f.write(src)
    lib = os.path.join(tmp, f"liboracle_mutant{idx}.so")
    oracle.compile_source(path, lib)
    return _run_pins(lib)


def test_every_snippet_is_in_the_source():
    src = _source()
    names = [m[0] for m in MUTANTS]
    assert len(set(names)) == len(names)
    for name, old, new in MUTANTS:
        assert old in src, name
        assert old != new, name
    for name, edits in CONSISTENT:
        for old, new in edits:
            assert old in src, (name, old)


def test_pins_catch_every_planted_mistake(tmp_path):
    src = _source()
    jobs = [("control (unmodified)", src)]
    jobs += [(name, src.replace(old, new, 1)) for name, old, new in MUTANTS]
    jobs += [(name, _apply(src, edits)) for name, edits in CONSISTENT]
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        futs = [ex.submit(_build_and_run, str(tmp_path), i, s) for i, (_, s) in enumerate(jobs)]
        results = [f.result() for f in futs]
    rc0, out0 = results[0]
    assert rc0 == 0, f"the unmodified oracle must pass its pins:\n{out0}"
    survivors = [name for (name, _), (rc, _) in zip(jobs[1:], results[1:]) if rc != 1]
    assert not survivors, f"mutants the pins did not catch (or that crashed): {survivors}"
