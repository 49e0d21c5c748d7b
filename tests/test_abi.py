"""The C-ABI library loads, exports every entry point include/quadsim.h
declares, its config struct matches the Python mirror, and argument errors are
reported before any device work (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "quadsim.h")


@pytest.fixture(scope="module")
def L():
    from paper_2311_13081_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2311_13081_amd import build
        build.build()
    return _lib.load()


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(sim_\w+)\s*\(", text, re.M)))


def test_header_declares_expected_calls():
    names = declared_functions()
    for required in ("sim_create", "sim_reset", "sim_step", "sim_rollout", "sim_backward"):
        assert required in names


def test_library_exports_every_declared_symbol(L):
    from paper_2311_13081_amd import _lib
    names = declared_functions()
    assert set(names) == set(_lib.EXPORTS)
    for n in names:
        assert hasattr(L, n), n


def test_config_struct_layout_matches_header(tmp_path):
    from paper_2311_13081_amd import _lib
    src = tmp_path / "layout.c"
    fields = [n for n, _ in _lib.SimConfig._fields_]
    body = "\n".join(f'printf("{f} %zu\\n", offsetof(sim_config, {f}));' for f in fields)
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "quadsim.h"\n'
        "int main(void){" + body + 'printf("sizeof %zu\\n", sizeof(sim_config)); return 0;}\n')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src),
                           "-o", str(exe)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    got = dict(line.split() for line in out if line.strip())
    for name, _ in _lib.SimConfig._fields_:
        assert int(got[name]) == getattr(_lib.SimConfig, name).offset, name
    assert int(got["sizeof"]) == ctypes.sizeof(_lib.SimConfig)


def _cfg(**kw):
    import workloads
    return workloads.crazyflie_config(**kw)


@pytest.mark.parametrize("bad", [
    dict(n_envs=0), dict(n_envs=(1 << 24) + 1), dict(dt=-0.01), dict(flags=128),
    dict(ckpt_every=0),
    dict(flags=8 | 16), dict(dist_force=-1.0), dict(dist_torque=float("nan")),
    dict(obs_noise=(0.0, -0.1, 0.0, 0.0)),
    dict(nominal=[0.0, 3.85e-6, 3.85e-6, 5.9675e-6, 0, 0, 3.16e-10, 0.15]),
    dict(nominal=[0.027, 3.85e-6, 3.85e-6, 5.9675e-6, 0, 0, 0.0, 0.15]),
    dict(rpm_max=-1.0), dict(max_tape_horizon=-3),
    dict(dr_enable=1, dr_lo=[0.8] * 7 + [-0.5]),
    # a segment's backward record above 4 GiB (2M envs x 16 steps)
    dict(n_envs=2_000_000, max_tape_horizon=64, ckpt_every=16),
])
def test_invalid_config_rejected_before_device(L, bad):
    from paper_2311_13081_amd import _lib
    c = _lib.make_config(_cfg(**bad))
    h = ctypes.c_void_p()
    rc = L.sim_create(ctypes.byref(c), 0, ctypes.byref(h))
    assert rc == _lib.SIM_E_INVAL
    assert not h.value
    assert L.sim_last_error()


def test_null_arguments_rejected(L):
    from paper_2311_13081_amd import _lib
    assert L.sim_create(None, 0, None) == _lib.SIM_E_INVAL
    assert L.sim_rollout(None, None, 10, None, None, None, 0, None) == _lib.SIM_E_INVAL
    assert L.sim_backward(None, None, None, None, None, None, None) == _lib.SIM_E_INVAL
    assert L.sim_step(None, None, None, None, None, None) == _lib.SIM_E_INVAL
    assert L.sim_destroy(None) == _lib.SIM_OK
    assert L.sim_n_envs(None) == 0


def test_no_device_reports_device_error(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    from paper_2311_13081_amd import _lib
    c = _lib.make_config(_cfg())
    h = ctypes.c_void_p()
    assert L.sim_create(ctypes.byref(c), 0, ctypes.byref(h)) == _lib.SIM_E_DEVICE
    assert b"device" in L.sim_last_error()
