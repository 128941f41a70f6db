"""Seeded synthetic inputs and workload shapes.

This module is shared by the tests, the benchmark and the oracle-side checks,
so it holds none of the dedispersion arithmetic: only random voltages, their
8-bit encoding, random draws (pulse DMs and times) and the workload shapes.
Dispersed test pulses are made elsewhere (by the oracle in the tests).

Voltages are arrays [nsub][ntime][2 pol][2 re/im] (int8 or float32), i.e. one
dual-polarisation complex sample is 4 bytes (int8) or 16 bytes (float32).
The paper's LOFAR data are not available; Gaussian noise with the stated sigma
per real component stands in for them, with the LOFAR HBA subband setup of
Sec. 4 (195.3125 kHz Nyquist-sampled complex subbands).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SUBBAND_MHZ = 0.1953125  # 195.3125 kHz LOFAR subbands (Sec. 4)


@dataclass(frozen=True)
class Workload:
    name: str
    nsub: int
    f_centre: float          # MHz
    bw: float                # MHz
    nfft: int
    noverlap: int
    nchan: int
    ndec: int
    nblock: int
    dms: tuple
    input_kind: str          # "cf32" or "ci8"
    sigma: float
    pulses: int
    pulse_amp_sigma: float = 20.0
    seed: int = 1607
    extra: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return self.nfft // self.nchan

    @property
    def nd(self) -> int:
        return self.noverlap // self.nchan

    @property
    def tblk(self) -> int:
        return (self.m - self.nd) // self.ndec

    @property
    def ntime_in(self) -> int:
        return self.nblock * (self.nfft - self.noverlap) + self.noverlap

    @property
    def ntime_out(self) -> int:
        return self.nblock * self.tblk

    @property
    def data_seconds(self) -> float:
        return self.nblock * (self.nfft - self.noverlap) / (self.bw * 1e6)


def _dm_grid(start: float, step: float, n: int) -> tuple:
    return tuple(float(start + step * i) for i in range(n))


# Tiny case: 8 subbands spanning 120.0-121.5625 MHz, cf32 noise sigma=1,
# one 20-sigma impulse at DM 10, nfft 16384 / noverlap 4096 over 4 blocks,
# 16 DM trials 0..15, 8 channels, x4 downsampling.
TINY = Workload("tiny-8sub-16dm", nsub=8, f_centre=120.78125, bw=SUBBAND_MHZ,
                nfft=16384, noverlap=4096, nchan=8, ndec=4, nblock=4,
                dms=_dm_grid(0.0, 1.0, 16), input_kind="cf32", sigma=1.0, pulses=1,
                extra={"pulse_dm": 10.0})

# LOFAR-HBA-shaped: 288 subbands centred on 138 MHz (109.875-166.125 MHz),
# ci8 noise sigma=16, 10.02 s of data in 39 blocks of nfft 65536 with
# noverlap 15360 (the sweep across the lowest subband at DM 63.5, rounded up),
# 128 DM trials 0..63.5, 16 channels, x8 downsampling (81.92 us samples).
LOFAR = Workload("lofar-hba-288sub-128dm", nsub=288, f_centre=138.0, bw=SUBBAND_MHZ,
                 nfft=65536, noverlap=15360, nchan=16, ndec=8, nblock=39,
                 dms=_dm_grid(0.0, 0.5, 128), input_kind="ci8", sigma=16.0, pulses=5)

WORKLOADS = {w.name: w for w in (TINY, LOFAR)}


@dataclass(frozen=True)
class BeamDraw:
    """One beam of the batched workload: its own subband count and centre,
    N_bin (with n_c = N_bin / 4096, so every beam has M_bin = 4096), DM range
    and trial count.  The overlap follows from the beam's lowest channel and
    largest DM (Sec. 2), the block count from about one second of data."""
    nsub: int
    f_centre: float
    nfft: int
    nchan: int
    ndec: int
    dm_max: float
    ndm: int

    @property
    def dms(self) -> tuple:
        step = self.dm_max / (self.ndm - 1)
        return tuple(float(i * step) for i in range(self.ndm))

    @property
    def f_lo(self) -> float:
        return self.f_centre - self.nsub * SUBBAND_MHZ / 2


def batch_draws(nbeam: int = 24, seed: int = 1607) -> list:
    """Batched workload (several tied-array beams, Sec. 4): 32-288 subbands
    inside 110-190 MHz, N_bin from {2^14, 2^15, 2^16, 2^17}, channels so that
    M_bin = N_bin / n_c is 1024, 2048 or 4096, 16-256 DM trials from 0 to a
    beam-specific maximum in [20, 200]."""
    g = np.random.default_rng(np.random.SeedSequence([seed, 7331]))
    out = []
    for _ in range(nbeam):
        nsub = int(g.integers(32, 289))
        nfft = int(2 ** int(g.integers(14, 18)))
        m = int(2 ** int(g.integers(10, 13)))
        half = nsub * SUBBAND_MHZ / 2
        f_centre = float(g.uniform(110.0 + half, 190.0 - half))
        out.append(BeamDraw(nsub, f_centre, nfft, nfft // m, 8,
                            float(g.uniform(20.0, 200.0)), int(g.integers(16, 257))))
    return out


def subband_rng(seed: int, s: int) -> np.random.Generator:
    """Independent stream per subband, so any subset regenerates alone."""
    return np.random.default_rng(np.random.SeedSequence([seed, s]))


def gaussian_voltages(nsub: int, ntime: int, sigma: float, seed: int,
                      subbands=None) -> np.ndarray:
    """Complex128 noise [len(subbands)][ntime][2 pol], sigma per real component."""
    subs = range(nsub) if subbands is None else subbands
    out = np.empty((len(subs), ntime, 2), dtype=np.complex128)
    for i, s in enumerate(subs):
        g = subband_rng(seed, s)
        re = g.standard_normal((ntime, 2))
        im = g.standard_normal((ntime, 2))
        out[i] = sigma * (re + 1j * im)
    return out


def encode_cf32(x: np.ndarray) -> np.ndarray:
    """complex [nsub][ntime][2] -> float32 [nsub][ntime][2][2]."""
    y = np.empty(x.shape + (2,), dtype=np.float32)
    y[..., 0] = x.real
    y[..., 1] = x.imag
    return y


def encode_ci8(x: np.ndarray):
    """complex [nsub][ntime][2] -> int8 [nsub][ntime][2][2]: round half to
    even, clip to [-127, 127].  Returns (array, number of clipped components)."""
    r = np.rint(np.stack([x.real, x.imag], axis=-1))
    clipped = int(np.count_nonzero(np.abs(r) > 127))
    return np.clip(r, -127, 127).astype(np.int8), clipped


def decode(v: np.ndarray) -> np.ndarray:
    """[..][2][2] int8/float32 -> complex128 [..][2]."""
    return v[..., 0].astype(np.float64) + 1j * v[..., 1].astype(np.float64)


def pulse_draws(w: Workload, seed: int | None = None):
    """Random pulse parameters: (dm, t0) pairs.  DMs are drawn from the trial
    grid between 5 and 60 (on-grid), output samples t0 at least one block
    away from both ends of the stream."""
    g = np.random.default_rng(np.random.SeedSequence([w.seed if seed is None else seed, 99991]))
    grid = [d for d in w.dms if 5.0 <= d <= 60.0] or list(w.dms)
    out = []
    for _ in range(w.pulses):
        dm = float(grid[int(g.integers(len(grid)))])
        lo, hi = w.tblk, max(w.tblk + 1, w.ntime_out - w.tblk)
        out.append((dm, int(g.integers(lo, hi))))
    return out


def candidate_draws(n: int = 64, seed: int = 1607, lo: float = 5.0, hi: float = 60.0):
    """Refinement candidates: (true DM, pulse output sample, noise seed) with
    the DM uniform in [lo, hi) (continuous, off the trial grid) and the
    output sample in the middle block of a 4-block segment."""
    g = np.random.default_rng(np.random.SeedSequence([seed, 4711]))
    return [(float(g.uniform(lo, hi)), int(g.integers(0, 1 << 30)),
             int(g.integers(0, 1 << 30))) for _ in range(n)]


def device_noise(kind: str, nsub: int, ntime: int, sigma: float, seed: int, device):
    """Large noise generated directly in device memory with torch's seeded
    generator (for workloads too big to build on the host): a torch tensor
    [nsub][ntime][2][2], int8 ("ci8": rounded half to even and clipped as
    encode_ci8) or float32 ("cf32")."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    dt = torch.int8 if kind == "ci8" else torch.float32
    out = torch.empty((nsub, ntime, 2, 2), dtype=dt, device=device)
    rows = max(1, (1 << 26) // (ntime * 4))
    for s0 in range(0, nsub, rows):
        s1 = min(nsub, s0 + rows)
        z = torch.randn((s1 - s0, ntime, 2, 2), generator=gen, device=device, dtype=torch.float32)
        z *= sigma
        if kind == "ci8":
            out[s0:s1] = torch.clamp(torch.round(z), -127, 127).to(torch.int8)
        else:
            out[s0:s1] = z
        del z
    return out


def filterbank(ndm: int, ntime: int, nch: int, seed: int, kind: str = "power") -> np.ndarray:
    """Synthetic detected filterbanks [ndm][ntime][nch] float32: "power" is
    what detection of complex Gaussian noise in two polarisations gives (a
    sum of four squared unit normals, chi-square with 4 degrees of freedom);
    "codes" are integers 0..255 (exactly representable, so sums of a few
    thousand of them are exact in float32)."""
    g = np.random.default_rng(np.random.SeedSequence([seed, 424242]))
    if kind == "codes":
        return g.integers(0, 256, size=(ndm, ntime, nch)).astype(np.float32)
    z = g.standard_normal((ndm, ntime, nch, 4))
    return (z * z).sum(axis=3).astype(np.float32)


def device_filterbank(ndm: int, ntime: int, nch: int, seed: int, device):
    """The "power" filterbank of the same distribution generated in device
    memory with torch's seeded generator (for sizes too big for the host)."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    out = torch.empty((ndm, ntime, nch), dtype=torch.float32, device=device)
    for d in range(ndm):
        z = torch.randn((ntime, nch, 4), generator=gen, device=device, dtype=torch.float32)
        out[d] = (z * z).sum(dim=2)
        del z
    return out
