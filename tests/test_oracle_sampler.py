"""Pins of the cloud sampler oracle (Sec. 3 and 3.1 of arXiv:1705.04374:
uniform positions in the cloud, log-normal radii clipped to a range)."""
import math

import numpy as np
from scipy import stats

from oracle.sampler import SplitMix64, sample_cloud, stream
from workloads.configs import cloud_spec


def test_splitmix64_published_first_output():
    # SplitMix64 started from state 0: first output 0xE220A8397B1DCDAF
    g = SplitMix64(0)
    assert g.next() == 0xE220A8397B1DCDAF


def test_uniform_range_and_streams_differ():
    g = stream(1, 2, 3)
    u = np.array([g.uniform() for _ in range(20000)])
    assert u.min() >= 0.0 and u.max() < 1.0
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    a = [stream(1, 0, 0).next() for _ in range(1)]
    b = [stream(1, 0, 1).next() for _ in range(1)]
    c = [stream(1, 1, 0).next() for _ in range(1)]
    assert a != b and a != c and b != c


def test_cloud_invariants_and_distributions():
    spec = cloud_spec("cloud50")
    radii, rad_pos = [], []
    for idx in range(40):
        b = sample_cloud(spec, 99, 0, idx)
        assert b.shape == (50, 4)
        d = np.linalg.norm(b[:, None, :3] - b[None, :, :3], axis=-1)
        s = b[:, None, 3] + b[None, :, 3]
        np.fill_diagonal(d, np.inf)
        assert np.all(d >= s)                         # no overlap
        r = np.linalg.norm(b[:, :3] - 0.5, axis=1)
        assert np.all(r < 0.25)                        # centres in the ball
        radii.extend(b[:, 3])
        rad_pos.extend(r / 0.25)
    z = np.log(np.array(radii) / 0.02) / 0.3
    # rejection of overlaps biases large radii slightly; the law stays close
    assert abs(np.mean(z)) < 0.1 and abs(np.std(z) - 1) < 0.1
    # radial CDF of a uniform ball: P(r/R < x) = x^3
    assert stats.kstest(np.array(rad_pos) ** 3, "uniform").pvalue > 1e-3


def test_clipped_radii_and_determinism():
    spec = cloud_spec("cloud500")
    b1 = sample_cloud(spec, 7, 2, 5)
    b2 = sample_cloud(spec, 7, 2, 5)
    assert np.array_equal(b1, b2)
    assert np.all(b1[:, 3] >= 0.012) and np.all(b1[:, 3] <= 0.018)
    b3 = sample_cloud(spec, 7, 2, 6)
    assert not np.array_equal(b1, b3)


def test_two_dimensional_cloud():
    spec = cloud_spec("cloud2d")
    b = sample_cloud(spec, 3, 0, 0)
    assert b.shape == (8, 4) and np.all(b[:, 2] == 0.0)
    assert np.all(np.hypot(b[:, 0] - 0.5, b[:, 1] - 0.5) < 0.3)
