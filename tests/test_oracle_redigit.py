"""Pins of the redigitisation oracle (Sec. 3, the paragraph after the
transpose): per DM and channel, offset and scale from the mean and standard
deviation of the time series, then 8-bit codes.  The paper prints no worked
numbers for this step, so the pins are a hand-worked example, closed forms
and invariants; planted mistakes (sample instead of population deviation, a
flipped sign, a dropped zero level, truncation instead of rounding, a wrong
clamp, a transposed axis) must each fail one of them."""
import math
import types

import numpy as np
import pytest

from oracle import redigit


def _hand_cases(fn):
    # channel 0: 1..5 -> mean 3, population sigma sqrt(2); k = 16 / sqrt(2)
    #   codes rint(64 + (x - 3) * 11.3137085) = 41.37, 52.69, 64, 75.31, 86.63
    # channel 1: constant -> sigma 0, scale 0, every code at the zero level
    # channel 2: 0,0,0,0,100 -> mean 20, sigma 40, k 0.4 -> 56 x4, 96
    fb = np.array([[[1, 7, 0], [2, 7, 0], [3, 7, 0], [4, 7, 0], [5, 7, 100]]], dtype=np.float32)
    codes, mean, scale = fn(fb, 64.0, 16.0)
    assert codes.shape == fb.shape and codes.dtype == np.uint8
    assert list(codes[0, :, 0]) == [41, 53, 64, 75, 87]
    assert list(codes[0, :, 1]) == [64] * 5
    assert list(codes[0, :, 2]) == [56, 56, 56, 56, 96]
    assert mean[0, 0] == np.float32(3.0) and mean[0, 2] == np.float32(20.0)
    assert scale[0, 0] == np.float32(16.0 / math.sqrt(2.0))
    assert scale[0, 1] == 0.0 and scale[0, 2] == np.float32(0.4)
    # clamping: zero level 250 pushes the 100 to 282 -> 255; zero level 4 pulls 0 to -4 -> 0
    hi, _, _ = fn(fb, 250.0, 16.0)
    lo, _, _ = fn(fb, 4.0, 16.0)
    assert hi[0, 4, 2] == 255 and hi[0, 0, 2] == 242
    assert lo[0, 0, 2] == 0 and lo[0, 4, 2] == 36
    # ties round to even: mean 0, sigma 1 (x = -1, +1), k = 0.5 -> 64 -/+ 0.5
    tie = np.array([[[-1.0], [1.0]]], dtype=np.float32)
    c, _, _ = fn(tie, 64.0, 0.5)
    assert list(c[0, :, 0]) == [64, 64]


def _gaussian(fn):
    g = np.random.default_rng(5)
    fb = (1e5 + 300.0 * g.standard_normal((2, 200000, 3))).astype(np.float32)
    fb[1] *= 7.0
    codes, _, _ = fn(fb, 64.0, 16.0)
    c = codes.astype(np.float64)
    # mean of the codes at the zero level, spread counts_per_sigma (+1/12 from rounding)
    assert np.all(np.abs(c.mean(axis=1) - 64.0) < 0.15)
    assert np.all(np.abs(c.std(axis=1) - math.sqrt(256 + 1 / 12)) < 0.2)


def _invariants(fn):
    g = np.random.default_rng(6)
    fb = g.gamma(8.0, 100.0, size=(3, 777, 5)).astype(np.float32)
    base, m, k = fn(fb, 64.0, 16.0)
    # exact power-of-two rescaling of the data leaves every code unchanged
    scaled, m4, k4 = fn(fb * np.float32(4.0), 64.0, 16.0)
    assert np.array_equal(base, scaled)
    # channels and DMs are independent series
    perm = fn(fb[::-1, :, ::-1].copy(), 64.0, 16.0)[0]
    assert np.array_equal(perm, base[::-1, :, ::-1])
    # the codes follow from the FP32 parameters alone
    assert np.array_equal(redigit.quantise(fb, m, k, 64.0), base)
    # time order does not change the statistics
    rev = fn(fb[:, ::-1, :].copy(), 64.0, 16.0)[0]
    assert np.array_equal(rev, base[:, ::-1, :])


PINS = (_hand_cases, _gaussian, _invariants)


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__.strip("_") for p in PINS])
def test_redigitise_pins(pin):
    pin(redigit.redigitise)


def _mutant(src_old: str, src_new: str):
    import inspect
    mod_src = inspect.getsource(redigit)
    assert src_old in mod_src, src_old
    m = types.ModuleType("redigit_mutant")
    exec(compile(mod_src.replace(src_old, src_new), "redigit_mutant", "exec"), m.__dict__)
    return m.redigitise


MUTANTS = {
    "sample-std": ("((x - mu[:, None, :]) ** 2).mean(axis=1)",
                   "((x - mu[:, None, :]) ** 2).sum(axis=1) / (x.shape[1] - 1)"),
    "sign": ("np.subtract(x, mean32[:, None, :], dtype=np.float32)",
             "np.subtract(mean32[:, None, :], x, dtype=np.float32)"),
    "no-zero-level": ("np.add(t, np.float32(zero), dtype=np.float32)", "t"),
    "truncate": ("np.clip(np.rint(t), 0, 255)", "np.clip(np.trunc(t), 0, 255)"),
    "clamp-127": ("np.clip(np.rint(t), 0, 255)", "np.clip(np.rint(t), 0, 127)"),
    "axis": ("mu = x.mean(axis=1)", "mu = x.mean(axis=1) * 0 + x.mean(axis=(1, 2))[:, None]"),
    "sigma-not-sqrt": ("sigma = np.sqrt(", "sigma = np.abs("),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_redigitise_mutants_are_caught(name):
    fn = _mutant(*MUTANTS[name])
    caught = 0
    for pin in PINS:
        try:
            with np.errstate(all="ignore"):
                pin(fn)
        except (AssertionError, ValueError, FloatingPointError):
            caught += 1
    assert caught > 0, f"mutant {name} survived every pin"
