"""Host-side helpers of bench.py that need no GPU."""
import importlib.util
import math
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _times(last):
    t, d = [], 1
    while d <= last:
        t += [x * d for x in (1, 2, 5) if x * d <= last]
        d *= 10
    return t


@pytest.mark.parametrize("tau", [3.0, 47.0, 1800.0, 21000.0])
def test_crossing_time_of_a_stretched_exponential(bench, tau):
    # exp(-(t/tau)^beta) crosses 1/e at tau exactly; between samples a factor
    # 2 or 2.5 apart, interpolation linear in log t is within a few percent
    for beta in (0.6, 1.0):
        t = _times(100000)
        c = [math.exp(-((x / tau) ** beta)) for x in t]
        assert bench.crossing_time(t, c) == pytest.approx(tau, rel=0.06)


def test_crossing_time_exact_on_a_sample_and_none_when_not_reached(bench):
    t = [1, 2, 5, 10]
    assert bench.crossing_time(t, [0.9, 0.6, math.exp(-1.0), 0.1]) == pytest.approx(5.0, rel=1e-12)
    assert bench.crossing_time(t, [0.9, 0.8, 0.7, 0.6]) is None
