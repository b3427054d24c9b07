"""Pins of the noise contract: Philox4x32-10 against its published
known-answer vectors, the series log/sin/cos against libm, and the law of the
Box-Muller normals."""
import os

import numpy as np
import scipy.stats

from oracle import philox

HERE = os.path.dirname(__file__)


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append([int(x, 16) for x in line.split()])
    return np.array(rows, dtype=np.uint64)


def test_philox_known_answers():
    k = _kat()
    out = philox.philox4x32_10(k[:, :4].astype(np.uint32), k[:, 4:6].astype(np.uint32))
    assert np.array_equal(out.astype(np.uint64), k[:, 6:10])


def test_uniform_open_interval():
    u = philox.uniform_open(np.array([0, 1, 2**31, 2**32 - 1], dtype=np.uint32))
    assert u[0] > 0 and u[-1] < 1
    assert u[0] == 0.5 / 2**32


def test_series_log_matches_libm():
    rng = np.random.default_rng(0)
    u = np.concatenate([rng.uniform(0, 1, 200000), [0.5 / 2**32, 1 - 0.5 / 2**32, 0.5, 0.70710678]])
    ref = np.log(u)
    assert np.abs(philox.series_log(u) - ref).max() <= 4e-16 * np.abs(ref).max()
    assert np.abs(philox.series_log(u) - ref).max() < 4e-15


def test_series_sincos_matches_libm():
    rng = np.random.default_rng(1)
    u = np.concatenate([rng.uniform(0, 1, 200000), [0.125, 0.25, 0.375, 0.5, 0.875, 1 - 2**-33]])
    s, c = philox.series_sincos_2pi(u)
    assert np.abs(s - np.sin(2 * np.pi * u)).max() < 2e-15
    assert np.abs(c - np.cos(2 * np.pi * u)).max() < 2e-15


def test_normals_law():
    z = philox.normals(12345, np.arange(250000), 3, 7).ravel()
    assert abs(z.mean()) < 5 / np.sqrt(z.size)
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / z.size)
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-4
    # pairs from one word pair are independent (r cos, r sin)
    w = philox.normals(99, np.arange(100000), 0, 0)
    assert abs(np.corrcoef(w[:, 0], w[:, 1])[0, 1]) < 5 / np.sqrt(1e5)


def test_counter_fields_change_stream():
    a = philox.normals(1, np.arange(8), 0, 0)
    for b in [philox.normals(2, np.arange(8), 0, 0), philox.normals(1, np.arange(8), 1, 0),
              philox.normals(1, np.arange(8), 0, 1), philox.normals(1, np.arange(8), 0, 2**32)]:
        assert not np.any(a == b)
