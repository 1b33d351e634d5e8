"""The product's training schedule (Sec. 4.1: 3DGS learning rates, position rate decaying over
training, sigma_d frozen until the LoD mechanism switches on) against the oracle's formula.
No GPU needed."""
import numpy as np

from oracle import train_oracle as TO
from paper_2510_09997_amd.train import DEFAULT_LRS, LodSchedule


def test_schedule_learning_rates_match_oracle():
    sched = LodSchedule(s_max=8.0, enable_at=5000, total=30000)
    for it in (0, 1, 17, 2500, 4999, 5000, 5001, 12345, 29999, 30000, 45000):
        got = sched.lrs_at(it)
        want = TO.schedule_lrs(it, DEFAULT_LRS, enable_at=5000, total=30000)
        assert got.keys() == want.keys()
        for k in got:
            assert abs(got[k] - want[k]) <= 1e-12 * abs(want[k]), (it, k, got[k], want[k])
            assert np.float32(got[k]) == np.float32(want[k]), (it, k)
    assert sched.lrs_at(4999)["decay"] == 0.0 and sched.lrs_at(5000)["decay"] == DEFAULT_LRS["decay"]


def test_schedule_endpoints():
    sched = LodSchedule(s_max=8.0, enable_at=10, total=100)
    assert abs(sched.lrs_at(0)["mean"] - 1.6e-4) < 1e-18
    assert abs(sched.lrs_at(100)["mean"] - 1.6e-6) < 1e-18
    assert abs(sched.lrs_at(50)["mean"] - (1.6e-4 * 1.6e-6) ** 0.5) < 1e-15
