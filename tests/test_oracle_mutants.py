"""The oracle's pins are strong enough: plant one plausible mistake at a time
in a copy of the oracle's C source (on the CPU), build it, and check that the
pin suite fails.  The one mutant that must survive is the dropped swap of
halves per channel: rotating an M-bin spectrum by M/2 only multiplies the
channel's time series by (-1)^m, which detection removes."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "cdmt_oracle.c")
PINS = os.path.join(ROOT, "tests", "test_oracle_pins.py")
GRAD_PINS = os.path.join(ROOT, "tests", "test_oracle_gradient.py")

# (description, exact source text, replacement)
MUTANTS = [
    ("dedispersion sign", "h[j] = cexp(I *", "h[j] = cexp(-I *"),
    ("Eq. 1 denominator nu0^3", "nu0 * nu0 * (nu0 + nu)", "nu0 * nu0 * nu0"),
    ("no swap of halves per subband", "spec[p * n + j] = seg[(j + n / 2) % n]",
     "spec[p * n + j] = seg[j]"),
    ("no unpad offset", "acc += inten[nd / 2 + t * c->ndec + q]", "acc += inten[t * c->ndec + q]"),
    ("increasing channel order", "(c->nchan - 1 - ch);", "ch;"),
    ("missing 1/N", "cyc) / (double)n;", "cyc);"),
    ("channel centre off by half", "(ch + 0.5) * c->bw", "(ch + 0.0) * c->bw"),
    ("backward FFT sign", "orc_fft_inplace(z, m, +1)", "orc_fft_inplace(z, m, -1)"),
    ("one polarisation detected", "for (int p = 0; p < 2; ++p) {\n                /* swap",
     "for (int p = 0; p < 1; ++p) {\n                /* swap"),
    ("no downsampling sum", "for (long q = 0; q < c->ndec; ++q)", "for (long q = 0; q < 1; ++q)"),
    ("blocks without overlap", "(long)b * (n - c->noverlap)", "(long)b * n"),
    ("subbands in increasing order", "(long)(c->nsub - 1 - s) * c->nchan", "(long)s * c->nchan"),
    ("frequency grid off by one bin", "((double)j - n / 2.0)", "((double)j - n / 2.0 + 1)"),
    ("other k_DM value", "return 1e6 * ORC_KDM", "return 1e6 * 4148.808"),
    ("FFT twiddle sign", "double a = sign * 2.0 * ORC_PI * (double)k / (double)len;",
     "double a = -sign * 2.0 * ORC_PI * (double)k / (double)len;"),
]
# mistakes in the DM gradient, each of which the gradient pins must catch
GRAD_MUTANTS = [
    ("gradient: detection factor 2 dropped", "zp[i] = 2.0 * gi[i] * zp[i];", "zp[i] = gi[i] * zp[i];"),
    ("gradient: adjoint transform with e^+", "orc_fft_inplace(zp, m, -1);", "orc_fft_inplace(zp, m, +1);"),
    ("gradient: derivative of Eq. 1 with the wrong sign", "cplx ds = (double)c->sign * 2.0",
     "cplx ds = -(double)c->sign * 2.0"),
    ("gradient: upstream gradient without the unpad offset",
     "gi[nd / 2 + t * c->ndec + q] = G[", "gi[t * c->ndec + q] = G["),
    ("gradient: imaginary part taken", "const double term = creal(conj(zp[i]) * ds);",
     "const double term = cimag(conj(zp[i]) * ds);"),
    ("gradient: channel swap not inverted", "long j = ch * m + (i + m / 2) % m;       /* g_S' at bin j */",
     "long j = ch * m + i;"),
    ("gradient: one polarisation", "cplx *zp = z + p * m;", "cplx *zp = z + p * m; if (p) continue;"),
    ("voltage gradient: transfer function not conjugated", "gspec[j] = z[i] * conj(h[j]);",
     "gspec[j] = z[i] * h[j];"),
    ("voltage gradient: subband swap not inverted", "seg[k] = gspec[(k + n / 2) % n];",
     "seg[k] = gspec[k];"),
    ("voltage gradient: adjoint transform with e^-", "orc_fft_inplace(seg, n, +1);",
     "orc_fft_inplace(seg, n, -1);"),
    ("voltage gradient: scattered one sample late", "gx[((start + i) * 2 + p) * 2] += creal(seg[i]);",
     "gx[((start + i + 1) * 2 + p) * 2] += creal(seg[i]);"),
]
EQUIVALENT = ("no swap of halves per channel", "long j = ch * m + (i + m / 2) % m;",
              "long j = ch * m + i;")


def _build_and_run(tmp_path, name, old, new, pins=PINS):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"pattern for '{name}' not found"
    mut = src.replace(old, new, 1)
    c = tmp_path / "m.c"
    so = tmp_path / "m.so"
    c.write_text(mut)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", str(c), "-o", str(so),
                           "-lm", "-lpthread"])
    env = dict(os.environ, CDMT_ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", pins, "-q", "-x", "-p", "no:cacheprovider"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_kill_mutant(tmp_path, name, old, new):
    assert _build_and_run(tmp_path, name, old, new) != 0, f"mutant '{name}' survived the pins"


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_channel_half_swap_is_invisible_after_detection(tmp_path):
    name, old, new = EQUIVALENT
    assert _build_and_run(tmp_path, name, old, new) == 0


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
@pytest.mark.parametrize("name,old,new", GRAD_MUTANTS, ids=[m[0] for m in GRAD_MUTANTS])
def test_gradient_pins_kill_mutant(tmp_path, name, old, new):
    assert _build_and_run(tmp_path, name, old, new, GRAD_PINS) != 0, \
        f"mutant '{name}' survived the gradient pins"
