"""The paper's file formats and workflow options (Sec. 2.2, user parameters),
as host-side helpers around the C ABI.

* Data file (DATA_FILE_NAME): an unsigned 64-bit count n, then n longitudes,
  n latitudes and n values, each a 64-bit real; a NaN value marks a location
  without an observation.
* Prediction location file (PREDICTION_LOCATION_FILE): an unsigned 64-bit
  count np, then np longitudes and np latitudes (64-bit reals).
* Prediction result file (PREDICTION_RESULT_FILE_NAME): an unsigned 64-bit
  count nr, then nr longitudes, nr latitudes, nr means and nr variances.
* Prediction locations (PREDICTION_LOCATION_MODE): 'N' the data file's
  locations whose value is NaN, 'D' all its locations, 'A' the locations of a
  prediction location file.
* Number of levels 'default' (NUM_LEVELS_M): mra_build_tree with M = 0 takes
  the number of levels for which the finest level's average observation count
  per region is closest to the number of knots of the coarser levels
  (default_levels below states the same rule).
All values are little-endian, as written by the machines the paper uses.
"""
from __future__ import annotations

import math

import numpy as np

_U64 = np.dtype("<u8")
_F64 = np.dtype("<f8")


def _read(path, arrays):
    with open(path, "rb") as f:
        head = f.read(8)
        if len(head) != 8:
            raise ValueError(f"{path}: missing the 64-bit count")
        n = int(np.frombuffer(head, dtype=_U64)[0])
        body = np.fromfile(f, dtype=_F64, count=arrays * n)
    if body.size != arrays * n:
        raise ValueError(f"{path}: {arrays} x {n} values expected, {body.size} found")
    return [body[i * n:(i + 1) * n].astype(np.float64) for i in range(arrays)]


def _write(path, cols):
    n = len(cols[0])
    with open(path, "wb") as f:
        f.write(np.array([n], dtype=_U64).tobytes())
        for c in cols:
            c = np.ascontiguousarray(c, dtype=_F64)
            if len(c) != n:
                raise ValueError("columns of different lengths")
            f.write(c.tobytes())


def read_data_file(path):
    """(x, y, z) of a data file."""
    x, y, z = _read(path, 3)
    return x, y, z


def write_data_file(path, x, y, z):
    _write(path, [x, y, z])


def read_location_file(path):
    """(x, y) of a prediction location file."""
    x, y = _read(path, 2)
    return x, y


def write_location_file(path, x, y):
    _write(path, [x, y])


def write_prediction_file(path, x, y, mean, var):
    _write(path, [x, y, mean, var])


def read_prediction_file(path):
    """(x, y, mean, var) of a prediction result file."""
    return tuple(_read(path, 4))


def prediction_locations(mode, x=None, y=None, z=None, location_file=None):
    """Locations to predict at for PREDICTION_LOCATION_MODE 'N', 'D' or 'A'."""
    if mode == "N":
        keep = np.isnan(np.asarray(z, dtype=np.float64))
        return np.asarray(x, dtype=np.float64)[keep], np.asarray(y, dtype=np.float64)[keep]
    if mode == "D":
        return np.asarray(x, dtype=np.float64).copy(), np.asarray(y, dtype=np.float64).copy()
    if mode == "A":
        if location_file is None:
            raise ValueError("mode 'A' needs a prediction location file")
        return read_location_file(location_file)
    raise ValueError("mode must be 'N', 'D' or 'A'")


def default_levels(n_obs: int, J: int, r: int) -> int:
    """The 'default' number of levels: M such that n_obs / J^(M-1), the
    average observation count of a finest-level region, is closest (on a log
    scale) to r_hat, the knots per region above the finest level; at least 1."""
    nx = 1
    while nx * nx < r:
        nx += 1
    rhat = nx * (r // nx)
    if n_obs <= rhat:
        return 1
    return 1 + max(0, int(math.floor(math.log(n_obs / rhat) / math.log(J) + 0.5)))
