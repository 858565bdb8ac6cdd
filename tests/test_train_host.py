"""Host-side schedule of the training loop against the oracle's (CPU)."""
import numpy as np

from paper_2406_11836_amd import train


def test_position_schedule_matches_oracle(orc):
    for step in (0, 1, 17, 5000, 14999, 15000, 29999, 30000, 45000):
        a = train.expon_lr(step, 1.6e-4, 1.6e-6, 30000)
        b = orc.expon_lr(step, 1.6e-4, 1.6e-6, 30000)
        assert abs(a - b) <= 1e-15 * b, step


def test_default_group_rates():
    lr = train.DEFAULT_LR
    assert lr["means_init"] == 1.6e-4 and lr["means_final"] == 1.6e-6
    assert np.isclose(lr["sh_rest"], lr["sh_dc"] / 20)
