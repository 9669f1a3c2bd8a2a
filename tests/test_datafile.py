"""The paper's file formats and workflow options (Sec. 2.2), host side: the
byte layout of the data, location and result files, the prediction location
modes, and the default number of levels."""
import struct

import numpy as np
import pytest

from paper_1905_00141_amd import datafile as df


def test_data_file_layout_and_round_trip(tmp_path):
    rng = np.random.default_rng(1)
    x, y, z = rng.random(5), rng.random(5), rng.standard_normal(5)
    z[2] = np.nan
    p = tmp_path / "data.bin"
    df.write_data_file(p, x, y, z)
    raw = p.read_bytes()
    assert len(raw) == 8 + 3 * 5 * 8
    assert struct.unpack("<Q", raw[:8])[0] == 5
    vals = struct.unpack("<15d", raw[8:])
    assert np.array_equal(np.array(vals[:5]), x) and np.array_equal(np.array(vals[5:10]), y)
    assert np.isnan(vals[12]) and vals[10] == z[0]
    x2, y2, z2 = df.read_data_file(p)
    assert np.array_equal(x2, x) and np.array_equal(y2, y) and np.array_equal(z2, z, equal_nan=True)


def test_location_and_result_files(tmp_path):
    x, y = np.array([0.1, 0.2, 0.3]), np.array([0.4, 0.5, 0.6])
    p = tmp_path / "loc.bin"
    df.write_location_file(p, x, y)
    assert struct.unpack("<Q", p.read_bytes()[:8])[0] == 3 and len(p.read_bytes()) == 8 + 48
    a, b = df.read_location_file(p)
    assert np.array_equal(a, x) and np.array_equal(b, y)
    q = tmp_path / "res.bin"
    df.write_prediction_file(q, x, y, x + 1, y + 2)
    r = df.read_prediction_file(q)
    assert len(q.read_bytes()) == 8 + 4 * 24 and np.array_equal(r[2], x + 1) and np.array_equal(r[3], y + 2)


def test_truncated_file_is_an_error(tmp_path):
    p = tmp_path / "bad.bin"
    p.write_bytes(struct.pack("<Q", 4) + b"\0" * 40)
    with pytest.raises(ValueError):
        df.read_data_file(p)


def test_prediction_location_modes(tmp_path):
    x, y = np.array([0.1, 0.2, 0.3, 0.4]), np.array([0.5, 0.6, 0.7, 0.8])
    z = np.array([1.0, np.nan, 2.0, np.nan])
    px, py = df.prediction_locations("N", x, y, z)
    assert np.array_equal(px, [0.2, 0.4]) and np.array_equal(py, [0.6, 0.8])
    px, py = df.prediction_locations("D", x, y, z)
    assert np.array_equal(px, x) and np.array_equal(py, y)
    p = tmp_path / "loc.bin"
    df.write_location_file(p, [0.9], [0.1])
    px, py = df.prediction_locations("A", location_file=p)
    assert px.tolist() == [0.9] and py.tolist() == [0.1]
    with pytest.raises(ValueError):
        df.prediction_locations("X", x, y, z)


@pytest.mark.parametrize("J,r", [(4, 64), (4, 32), (2, 16), (2, 49)])
def test_default_levels(J, r):
    nx = int(np.ceil(np.sqrt(r)))
    rhat = nx * (r // nx)
    # exact powers: the finest level then averages r_hat observations per region
    for k in range(0, 8):
        assert df.default_levels(rhat * J ** k, J, r) == k + 1
    # the chosen level's average count is within a factor sqrt(J) of r_hat
    for n in [rhat + 1, 5 * rhat, 1000, 123457, 1 << 20]:
        M = df.default_levels(n, J, r)
        avg = n / J ** (M - 1)
        assert rhat / np.sqrt(J) * 0.999 <= avg <= rhat * np.sqrt(J) * 1.001 or M == 1
    assert df.default_levels(1, J, r) == 1 and df.default_levels(rhat, J, r) == 1
