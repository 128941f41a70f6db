"""FP64 CPU oracle for coherent dedispersion to many DM trials.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow definition that the
GPU library is checked against.  Only the test suite, ``__graft_entry__.smoke``
and the CPU-baseline leg of ``bench.py`` may import it; the library itself never
does.  It shares no code with the HIP implementation: the arithmetic lives in
``cdmt_oracle.c`` (double precision, its own radix-2 FFT), and this module only
marshals numpy arrays through ctypes.

Every function cites the passage of Bassa, Pleunis & Hessels (2016) it follows;
the C file carries the step-by-step citations.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cdmt_oracle.c")
_LIB = os.environ.get("CDMT_ORACLE_LIB") or os.path.join(_HERE, "libcdmt_oracle.so")

CF32, CI8, CF64 = 0, 1, 2
CHANNEL, SUBBAND = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, -O2, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
             "-fno-fast-math", _SRC, "-o", tmp, "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
_lock = threading.Lock()


class _Cfg(ctypes.Structure):
    _fields_ = [("nsub", ctypes.c_int), ("f_centre", ctypes.c_double),
                ("bw", ctypes.c_double), ("nfft", ctypes.c_int),
                ("noverlap", ctypes.c_int), ("nchan", ctypes.c_int),
                ("ndec", ctypes.c_int), ("chirp_ref", ctypes.c_int),
                ("sign", ctypes.c_int)]


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if "CDMT_ORACLE_LIB" not in os.environ and (
                    not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
                build(force=True)
            lib = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            lib.orc_dft.argtypes = [P, P, ctypes.c_long, ctypes.c_int]
            lib.orc_fft.argtypes = [P, P, ctypes.c_long, ctypes.c_int]
            lib.orc_fft.restype = ctypes.c_int
            lib.orc_chirp_cycles.argtypes = [ctypes.c_double] * 3
            lib.orc_chirp_cycles.restype = ctypes.c_double
            lib.orc_sweep_seconds.argtypes = [ctypes.c_double] * 3
            lib.orc_sweep_seconds.restype = ctypes.c_double
            lib.orc_kdm.restype = ctypes.c_double
            lib.orc_validate.argtypes = [ctypes.POINTER(_Cfg)]
            lib.orc_tblk.argtypes = [ctypes.POINTER(_Cfg)]
            lib.orc_subband_block.argtypes = [ctypes.POINTER(_Cfg), ctypes.c_int, P, ctypes.c_long,
                                              ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P]
            lib.orc_dm_gradient.argtypes = [ctypes.POINTER(_Cfg), ctypes.c_int, P, ctypes.c_long,
                                            ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P, P, P]
            lib.orc_voltage_gradient.argtypes = [ctypes.POINTER(_Cfg), ctypes.c_int, P,
                                                 ctypes.c_long, ctypes.c_int, ctypes.c_int,
                                                 ctypes.c_double, P, P]
            lib.orc_dedisperse.argtypes = [ctypes.POINTER(_Cfg), ctypes.c_int, P, ctypes.c_long,
                                           ctypes.c_int, P, ctypes.c_int, P, ctypes.c_int]
            lib.orc_inject_impulse.argtypes = [ctypes.POINTER(_Cfg), ctypes.c_int, P, ctypes.c_long,
                                               ctypes.c_double, ctypes.c_long, ctypes.c_double,
                                               ctypes.c_long]
            _lib = lib
    return _lib


@dataclass(frozen=True)
class Config:
    """Plan parameters in the paper's notation (Sec. 2-3).

    nsub = n_s, nfft = N_bin, noverlap = n_d * n_c (subband samples),
    nchan = n_c, ndec = time-downsampling factor, bw = subband width in MHz
    (equal to the complex sample rate in MHz), f_centre = band centre in MHz.
    """
    nsub: int
    f_centre: float
    bw: float
    nfft: int
    noverlap: int
    nchan: int
    ndec: int
    chirp_ref: int = CHANNEL
    sign: int = -1

    def c(self) -> _Cfg:
        return _Cfg(self.nsub, self.f_centre, self.bw, self.nfft, self.noverlap,
                    self.nchan, self.ndec, self.chirp_ref, self.sign)

    @property
    def m(self) -> int:
        return self.nfft // self.nchan

    @property
    def nd(self) -> int:
        return self.noverlap // self.nchan

    @property
    def tblk(self) -> int:
        return (self.m - self.nd) // self.ndec

    def ntime_in(self, nblock: int) -> int:
        return nblock * (self.nfft - self.noverlap) + self.noverlap

    def sub_centre(self, s: int) -> float:
        return self.f_centre + (s - (self.nsub - 1) / 2.0) * self.bw


def _kind_of(x: np.ndarray) -> int:
    if x.dtype == np.int8:
        return CI8
    if x.dtype == np.float32:
        return CF32
    if x.dtype == np.float64:
        return CF64
    raise TypeError(f"unsupported voltage dtype {x.dtype}")


def _as_voltages(x: np.ndarray) -> np.ndarray:
    """Voltages as a C-contiguous real array [nsub][ntime][2 pol][2 re/im]."""
    if np.iscomplexobj(x):
        x = np.ascontiguousarray(x)
        x = x.view(np.float64 if x.dtype == np.complex128 else np.float32).reshape(*x.shape, 2)
    x = np.ascontiguousarray(x)
    if x.ndim != 4 or x.shape[2:] != (2, 2):
        raise ValueError("voltages must be [nsub][ntime][2][2] (or complex [nsub][ntime][2])")
    return x


def validate(cfg: Config) -> bool:
    return _load().orc_validate(ctypes.byref(cfg.c())) == 0


def dft(x: np.ndarray, sign: int) -> np.ndarray:
    """Brute-force O(n^2) DFT, exp(sign 2 pi i k n / N)."""
    x = np.ascontiguousarray(x, dtype=np.complex128)
    y = np.empty_like(x)
    _load().orc_dft(x.ctypes.data, y.ctypes.data, x.size, sign)
    return y


def fft(x: np.ndarray, sign: int) -> np.ndarray:
    """The oracle's own radix-2 FFT, exp(sign 2 pi i k n / N), unnormalised."""
    x = np.ascontiguousarray(x, dtype=np.complex128)
    y = np.empty_like(x)
    if _load().orc_fft(x.ctypes.data, y.ctypes.data, x.size, sign) != 0:
        raise ValueError("length must be a power of two")
    return y


def chirp_cycles(nu: float, nu0: float, dm: float) -> float:
    """Phase of the transfer function of Eq. 1 in cycles (nu, nu0 in MHz)."""
    return _load().orc_chirp_cycles(nu, nu0, dm)


def sweep_seconds(nu_min: float, nu_max: float, dm: float) -> float:
    """Dispersion sweep of Eq. 2 in seconds."""
    return _load().orc_sweep_seconds(nu_min, nu_max, dm)


def kdm() -> float:
    return _load().orc_kdm()


def subband_block(cfg: Config, x: np.ndarray, s: int, b: int, dms) -> np.ndarray:
    """Filterbank of one subband s and one block b: [ndm][tblk][nchan] in
    increasing channel frequency (Sec. 3 steps, Alg. 1 loop body)."""
    x = _as_voltages(x)
    dms = np.ascontiguousarray(dms, dtype=np.float64)
    xs = np.ascontiguousarray(x[s])
    out = np.empty((dms.size, cfg.tblk, cfg.nchan), dtype=np.float64)
    st = _load().orc_subband_block(ctypes.byref(cfg.c()), _kind_of(xs), xs.ctypes.data,
                                   xs.shape[0], s, b, dms.ctypes.data, dms.size,
                                   out.ctypes.data)
    if st != 0:
        raise ValueError(f"orc_subband_block failed ({st})")
    return out


def dm_gradient(cfg: Config, x: np.ndarray, s: int, b: int, dms, G: np.ndarray,
                with_abs: bool = False):
    """d/dDM of L = sum G * F over one subband s and block b, one value per DM
    (F and G as [ndm][tblk][nchan] in increasing channel frequency): the
    adjoint of the per-DM chain of Sec. 3 (chirp of Eq. 1, swap, backward FFT,
    detection, downsampling), each step's adjoint written out in the C file.
    with_abs: also return, per DM, the sum of the absolute values of the
    per-bin terms whose sum is the derivative."""
    x = _as_voltages(x)
    dms = np.ascontiguousarray(dms, dtype=np.float64)
    G = np.ascontiguousarray(G, dtype=np.float64)
    if G.shape != (dms.size, cfg.tblk, cfg.nchan):
        raise ValueError("G must be [ndm][tblk][nchan]")
    xs = np.ascontiguousarray(x[s])
    out = np.empty(dms.size, dtype=np.float64)
    absterms = np.empty(dms.size, dtype=np.float64)
    st = _load().orc_dm_gradient(ctypes.byref(cfg.c()), _kind_of(xs), xs.ctypes.data,
                                 xs.shape[0], s, b, dms.ctypes.data, dms.size,
                                 G.ctypes.data, out.ctypes.data, absterms.ctypes.data)
    if st != 0:
        raise ValueError(f"orc_dm_gradient failed ({st})")
    return (out, absterms) if with_abs else out


def voltage_gradient(cfg: Config, x: np.ndarray, s: int, nblock: int, dm: float,
                     G: np.ndarray) -> np.ndarray:
    """dL/dx for L = sum G * F at one DM over subband s and blocks 0..nblock-1
    (G [nblock*tblk][nchan] in increasing channel frequency): complex128
    [ntime][2], dL/dRe x = real part, dL/dIm x = imaginary part.  The adjoint
    through the per-DM chain and the forward stage of Sec. 3, block by block,
    overlap-added."""
    x = _as_voltages(x)
    G = np.ascontiguousarray(G, dtype=np.float64)
    if G.shape != (nblock * cfg.tblk, cfg.nchan):
        raise ValueError("G must be [nblock*tblk][nchan]")
    xs = np.ascontiguousarray(x[s])
    gx = np.zeros((xs.shape[0], 2, 2), dtype=np.float64)
    for b in range(nblock):
        gb = np.ascontiguousarray(G[b * cfg.tblk:(b + 1) * cfg.tblk])
        st = _load().orc_voltage_gradient(ctypes.byref(cfg.c()), _kind_of(xs), xs.ctypes.data,
                                          xs.shape[0], s, b, float(dm), gb.ctypes.data,
                                          gx.ctypes.data)
        if st != 0:
            raise ValueError(f"orc_voltage_gradient failed ({st})")
    return gx[..., 0] + 1j * gx[..., 1]


def dedisperse(cfg: Config, x: np.ndarray, nblock: int, dms, nthreads: int = 0) -> np.ndarray:
    """Whole filterbank [ndm][nblock*tblk][nsub*nchan], channels in decreasing
    frequency (Sec. 3).  nthreads=0 uses every core."""
    x = _as_voltages(x)
    dms = np.ascontiguousarray(dms, dtype=np.float64)
    if nthreads <= 0:
        nthreads = os.cpu_count() or 1
    out = np.zeros((dms.size, nblock * cfg.tblk, cfg.nsub * cfg.nchan), dtype=np.float64)
    st = _load().orc_dedisperse(ctypes.byref(cfg.c()), _kind_of(x), x.ctypes.data, x.shape[1],
                                nblock, dms.ctypes.data, dms.size, out.ctypes.data, nthreads)
    if st != 0:
        raise ValueError(f"orc_dedisperse failed ({st})")
    return out


def inject_impulse(cfg: Config, x: np.ndarray, s: int, dm: float, n0: int, amp: float,
                   window: int | None = None) -> None:
    """Add, in place, a real impulse of amplitude amp at sample n0 (both pols)
    of subband s, dispersed by the inverse of the plan's transfer function at
    DM dm.  x is complex128 [nsub][ntime][2]."""
    if x.dtype != np.complex128 or not x.flags.c_contiguous or x.ndim != 3 or x.shape[2] != 2:
        raise TypeError("x must be C-contiguous complex128 [nsub][ntime][2]")
    L = window or cfg.nfft
    xs = x[s]
    st = _load().orc_inject_impulse(ctypes.byref(cfg.c()), s, xs.ctypes.data, xs.shape[0],
                                    float(dm), int(n0), float(amp), int(L))
    if st != 0:
        raise ValueError(f"orc_inject_impulse failed ({st})")


def pulse_sample(cfg: Config, t0: int) -> int:
    """Input sample at the centre of output sample t0 (output sample t covers
    input samples noverlap/2 + t*nchan*ndec + [0, nchan*ndec))."""
    return cfg.noverlap // 2 + t0 * cfg.nchan * cfg.ndec + (cfg.nchan * cfg.ndec) // 2
