"""The curriculum schedule of the training loop (Sec. IV: every 100 000
steps the penalty weights are multiplied by their factors until they reach
their targets; the exploration noise decays on the same schedule), checked
against values worked out by hand."""
import pytest

torch = pytest.importorskip("torch")

from paper_2311_13081_amd.td3 import TD3Config, curriculum  # noqa: E402

C0 = dict(C_rp=1.0, C_rq=1.0, C_rv=0.1, C_rw=0.01, C_ra=0.01, C_rab=0.334053, C_rs=1.0)


def test_first_round_keeps_initial_constants():
    cfg = TD3Config()
    for step in (0, 1, 99_999):
        C, sigma, k = curriculum(cfg, C0, step)
        assert k == 0 and C == C0 and sigma == 0.5


def test_rounds_multiply_until_the_targets():
    cfg = TD3Config()
    C, sigma, k = curriculum(cfg, C0, 100_000)
    assert k == 1
    assert C["C_rp"] == pytest.approx(1.2) and C["C_ra"] == pytest.approx(0.014)
    assert sigma == pytest.approx(0.4)
    C, sigma, k = curriculum(cfg, C0, 300_000)
    assert C["C_rp"] == pytest.approx(1.728) and C["C_ra"] == pytest.approx(0.02744)
    assert sigma == pytest.approx(0.256)
    # 1.2^4 = 2.07 > 2: clamped; 1.4^5 = 5.38 -> 0.0538 > 0.05: clamped
    C, sigma, k = curriculum(cfg, C0, 500_000)
    assert C["C_rp"] == 2.0 and C["C_ra"] == 0.05
    assert sigma == pytest.approx(0.16384)
    C, sigma, k = curriculum(cfg, C0, 3_000_000)
    assert C["C_rp"] == 2.0 and C["C_ra"] == 0.05 and sigma == 0.1
    # constants without a factor never move
    for key in ("C_rq", "C_rv", "C_rw", "C_rab", "C_rs"):
        assert C[key] == C0[key]


def test_decreasing_factor_clamps_from_above():
    cfg = TD3Config(C_factor=dict(C_rs=0.5), C_target=dict(C_rs=0.3))
    assert curriculum(cfg, C0, 100_000)[0]["C_rs"] == 0.5
    assert curriculum(cfg, C0, 200_000)[0]["C_rs"] == 0.3
