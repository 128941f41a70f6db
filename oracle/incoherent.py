"""FP64 oracle of the incoherent stage of a semi-coherent search (Sec. 1 and
Sec. 4: each coherently dedispersed filterbank is dedispersed incoherently
at fine DM steps around its coherent trial DM).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Incoherent dedispersion shifts each channel's time series by its dispersion
delay and sums the channels (Sec. 1).  The delay of a channel relative to the
highest one follows Eq. 2 with nu_min = the channel's frequency and nu_max =
the highest channel's.  Reading: the frequency of a channel is the one it was
coherently referred to (its centre in the per-channel mode, its subband's
centre in the per-subband mode), delays are rounded to whole output samples
(rint, half to even) in FP64 as written below, and the output covers the
samples for which every channel has data.
"""
from __future__ import annotations

import numpy as np

from . import Config, kdm


def channel_frequencies(cfg: Config) -> np.ndarray:
    """Reference frequency (MHz) of every output channel, in the filterbank's
    decreasing-frequency order ch = (nsub-1-s) nchan + (nchan-1-c)."""
    out = np.empty(cfg.nsub * cfg.nchan)
    for s in range(cfg.nsub):
        fs = cfg.f_centre + (s - (cfg.nsub - 1) / 2.0) * cfg.bw
        for c in range(cfg.nchan):
            nu = fs if cfg.chirp_ref == 1 else fs - cfg.bw / 2.0 + (c + 0.5) * cfg.bw / cfg.nchan
            out[(cfg.nsub - 1 - s) * cfg.nchan + (cfg.nchan - 1 - c)] = nu
    return out


def sample_seconds(cfg: Config) -> float:
    """Duration of one filterbank sample: nchan * ndec subband samples."""
    return cfg.nchan * cfg.ndec / (cfg.bw * 1e6)


def delays(cfg: Config, dm: float) -> np.ndarray:
    """Whole-sample delay of every channel behind the highest (Eq. 2)."""
    nu = channel_frequencies(cfg)
    top = nu.max()
    u = 1.0 / (nu * nu) - 1.0 / (top * top)
    return np.rint(kdm() * dm * u / sample_seconds(cfg)).astype(np.int64)


def trial_dms(dm_coh, ddm0: float, ddm: float, ntrial: int) -> np.ndarray:
    """[ndm][ntrial] fine trials dm_coh[d] + ddm0 + k ddm."""
    return np.asarray(dm_coh, np.float64)[:, None] + (ddm0 + ddm * np.arange(ntrial))[None, :]


def dedisperse(cfg: Config, fb: np.ndarray, dm_coh, ddm0: float, ddm: float, ntrial: int):
    """T[d][k][t] = sum_ch fb[d][t + D(ch, DM_dk)][ch] for t < nout, nout =
    ntime - largest delay over all trials.  fb is [ndm][ntime][nsub*nchan]."""
    fb = np.asarray(fb, dtype=np.float64)
    dms = trial_dms(dm_coh, ddm0, ddm, ntrial)
    D = np.stack([np.stack([delays(cfg, dm) for dm in row]) for row in dms])  # [d][k][ch]
    nout = fb.shape[1] - int(D.max())
    if nout <= 0:
        raise ValueError("the largest delay leaves no complete output sample")
    out = np.zeros((fb.shape[0], ntrial, nout))
    for d in range(fb.shape[0]):
        for k in range(ntrial):
            for ch in range(fb.shape[2]):
                out[d, k] += fb[d, D[d, k, ch]:D[d, k, ch] + nout, ch]
    return out


def sample(cfg: Config, fb_d: np.ndarray, dm: float, ts) -> np.ndarray:
    """Single outputs of one trial: sum_ch fb_d[t + D(ch, dm)][ch] for each t
    in ts, fb_d one filterbank [ntime][nsub*nchan] (FP64 sums)."""
    D = delays(cfg, dm)
    ch = np.arange(fb_d.shape[1])
    return np.array([np.asarray(fb_d[int(t) + D, ch], dtype=np.float64).sum() for t in ts])
