"""FP64 oracle of the redigitisation that follows the filterbank (Sec. 3, the
paragraph after the transpose; Alg. 1 "redigitize").

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper fixes the procedure but not the mapping: per DM trial and channel,
the offset and scale of the 8-bit codes come from the average and standard
deviation of that channel's time series over the processed samples.  The
reading used here (shared with the library's documented interface):

* mean  mu = (1/T) sum_t x_t, standard deviation sigma = sqrt((1/T) sum_t
  (x_t - mu)^2) (population form), both in FP64, two passes;
* the per-(DM, channel) parameters handed to the quantiser are mu and
  k = counts_per_sigma / sigma, each rounded once to FP32 (k = 0 when
  sigma = 0);
* code = clamp(rint(((x - mu) * k) + zero), 0, 255) evaluated in FP32 with
  each of the three operations rounded separately (subtract, multiply, add),
  rint rounding half to even.  zero is the code of the mean and
  counts_per_sigma the codes per standard deviation.

Written as the plain definition with numpy; no blocking or reordering.
"""
from __future__ import annotations

import numpy as np


def stats(fb: np.ndarray):
    """Per (DM, channel) mean and population standard deviation in FP64 of a
    filterbank [ndm][ntime][nchan] (Sec. 3: "average and standard deviation of
    the floating point time-series of each channel")."""
    x = np.asarray(fb, dtype=np.float64)
    if x.ndim != 3 or x.shape[1] < 1:
        raise ValueError("filterbank must be [ndm][ntime >= 1][nchan]")
    mu = x.mean(axis=1)
    sigma = np.sqrt(((x - mu[:, None, :]) ** 2).mean(axis=1))
    return mu, sigma


def parameters(fb: np.ndarray, counts_per_sigma: float):
    """FP32 quantiser parameters (mean, scale) per (DM, channel)."""
    mu, sigma = stats(fb)
    with np.errstate(divide="ignore"):
        k = np.where(sigma > 0, float(counts_per_sigma) / np.where(sigma > 0, sigma, 1.0), 0.0)
    return mu.astype(np.float32), k.astype(np.float32)


def quantise(fb: np.ndarray, mean32: np.ndarray, scale32: np.ndarray, zero: float) -> np.ndarray:
    """8-bit codes from FP32 parameters, FP32 arithmetic, one rounding per
    operation, round half to even, clamp to [0, 255]."""
    x = np.asarray(fb, dtype=np.float32)
    t = np.subtract(x, mean32[:, None, :], dtype=np.float32)
    t = np.multiply(t, scale32[:, None, :], dtype=np.float32)
    t = np.add(t, np.float32(zero), dtype=np.float32)
    return np.clip(np.rint(t), 0, 255).astype(np.uint8)


def redigitise(fb: np.ndarray, zero: float = 64.0, counts_per_sigma: float = 16.0):
    """The whole step: (codes uint8 [ndm][ntime][nchan], mean float32
    [ndm][nchan], scale float32 [ndm][nchan])."""
    mean32, scale32 = parameters(fb, counts_per_sigma)
    return quantise(fb, mean32, scale32, zero), mean32, scale32
