"""CPU checks of the operand-precision study (tests/precision_study.py):
its rounding primitive against values worked out by hand from the format
definitions, and the study's conclusions on a 1-s window (BF16 and FP16
inside their bounds, FP8 on every layer outside the 2e-2 BF16 bound)."""
import numpy as np
import pytest

import precision_study as ps


@pytest.mark.parametrize("fmt,x,expected", [
    # bf16: 8 significant bits; 0.1 = 1.6 x 2^-4 -> 205/128 x 2^-4
    ("bf16", 0.1, 205 / 128 / 16),
    # fp16: 11 significant bits; 0.1 -> 1638/1024 x 2^-4 (0.1 x 16384 = 1638.4)
    ("fp16", 0.1, 1638 / 16384),
    # e4m3: 4 significant bits; 0.1 = 1.6 x 2^-4 -> 13/8 x 2^-4
    ("e4m3", 0.1, 13 / 8 / 16),
    ("e4m3", 448.0, 448.0),          # largest finite value
    ("e4m3", 500.0, 448.0),          # saturates
    ("e4m3", 0.001, 2.0 ** -9),      # subnormal quantum 2^-9 (0.512 quanta rounds up)
    ("e4m3", 0.0009, 0.0),           # 0.46 quanta rounds to zero
    ("e4m3", 1.0625, 1.0),           # tie between 1 and 1.125 goes to the even 1
    # e5m2: 3 significant bits; 0.1 -> 6/4 x 2^-4 (1.6 x 4 = 6.4)
    ("e5m2", 0.1, 6 / 4 / 16),
    ("e5m2", 1e6, 57344.0),
])
def test_rounding_matches_format_definitions(fmt, x, expected):
    assert ps.round_to(np.array([x, -x]), fmt).tolist() == [expected, -expected]


def test_scaled_rounding_uses_power_of_two_and_undoes_it():
    x = np.array([0.003, -0.0011, 0.0007])
    y = ps.round_to(x, "e4m3", scaled=True)
    # scale 2^17 maps max |x| = 0.003 to 393 <= 448; 0.0007 is no longer subnormal
    k = 17
    assert np.array_equal(y, ps.round_to(x * 2.0 ** k, "e4m3") / 2.0 ** k)
    assert abs(y[2] - 0.0007) / 0.0007 < 2.0 ** -4


def test_study_conclusions_on_a_one_second_window():
    t = ps.deepclean_table(W=4096, batch=1, seed=22)
    w = t["whole"]
    assert w["bf16"] <= 2e-2 and w["fp16"] <= 2.5e-3
    assert w["fp16"] < w["bf16"] / 4
    for f in ("e4m3", "e5m2", "e4m3_scaled", "e5m2_scaled"):
        assert w[f] > 2e-2, (f, w[f])
    # the output conv alone in FP8 already exceeds the bound
    assert t["per_layer"]["e4m3_scaled"][8] > 2e-2
    b = ps.bbhnet_table(batch=16, seed=24)
    assert b["bf16"] <= 2e-2 and b["fp16"] <= 2.5e-3
