"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/cdmt.h declares, validates plans as documented, and
its size helpers agree with the method's formulas (Sec. 2-3)."""
import os
import re

import pytest

import oracle
import paper_1607_00909_amd as cdmt
from paper_1607_00909_amd import build as cbuild
from paper_1607_00909_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if cbuild.stale():
        cbuild.build()
    return cdmt.load()


def _declared():
    src = open(os.path.join(ROOT, "include", "cdmt.h")).read()
    return set(re.findall(r"^\s*(?:int|void|size_t|const char \*)\s*(cdmt_\w+)\s*\(", src, re.M))


def test_header_and_binding_agree():
    assert _declared() == set(cdmt.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_status_strings(lib):
    for st in (0, -1, -2, -3, -4, -5):
        assert cdmt.cdmt_status_string(st)
    assert cdmt.cdmt_status_string(-99) == "unknown status"


def _plan_status(*args):
    import ctypes
    h = ctypes.c_void_p()
    st = cdmt.load().cdmt_plan(ctypes.byref(h), *args)
    if st == 0:
        cdmt.cdmt_destroy(h.value)
    else:
        assert h.value is None
    return st


GOOD = (8, 120.78125, 0.1953125, 16384, 4096, 8, 4)


def test_plan_validation(lib):
    assert _plan_status(*GOOD) == cdmt.CDMT_OK
    bad = {
        "nsub 0": ((0,) + GOOD[1:], cdmt.CDMT_E_SHAPE),
        "nfft not pow2": (GOOD[:3] + (16000,) + GOOD[4:], cdmt.CDMT_E_SHAPE),
        "noverlap >= nfft": (GOOD[:4] + (16384,) + GOOD[5:], cdmt.CDMT_E_SHAPE),
        "noverlap odd multiple": (GOOD[:4] + (4100,) + GOOD[5:], cdmt.CDMT_E_SHAPE),
        "nchan not pow2": (GOOD[:5] + (6, 4), cdmt.CDMT_E_SHAPE),
        "ndec not dividing": (GOOD[:6] + (5,), cdmt.CDMT_E_SHAPE),
        "bw <= 0": (GOOD[:2] + (-0.1,) + GOOD[3:], cdmt.CDMT_E_SHAPE),
        "band below 0": ((8, 0.5) + GOOD[2:], cdmt.CDMT_E_SHAPE),
        "nan centre": ((8, float("nan")) + GOOD[2:], cdmt.CDMT_E_ARG),
        "nfft too small": (GOOD[:3] + (512, 0, 8, 1), cdmt.CDMT_E_UNSUPPORTED),
        "nfft too large": (GOOD[:3] + (1 << 18, 0, 8, 1), cdmt.CDMT_E_UNSUPPORTED),
        "M too small": (GOOD[:3] + (16384, 0, 512, 1), cdmt.CDMT_E_UNSUPPORTED),
        "M too large": (GOOD[:3] + (1 << 17, 0, 8, 1), cdmt.CDMT_E_UNSUPPORTED),
    }
    for name, (args, want) in bad.items():
        assert _plan_status(*args) == want, name


def test_options(lib):
    p = cdmt.cdmt_plan(*GOOD)
    try:
        assert cdmt.cdmt_plan_get(p, cdmt.CDMT_OPT_SIGN) == -1
        assert cdmt.cdmt_plan_get(p, cdmt.CDMT_OPT_CHIRP_REF) == 0
        assert cdmt.cdmt_plan_get(p, cdmt.CDMT_OPT_INPUT) == 0
        cdmt.cdmt_plan_set(p, cdmt.CDMT_OPT_SIGN, 1)
        assert cdmt.cdmt_plan_get(p, cdmt.CDMT_OPT_SIGN) == 1
        cdmt.cdmt_plan_set(p, cdmt.CDMT_OPT_DM_TILE, 7)
        assert cdmt.cdmt_plan_get(p, cdmt.CDMT_OPT_DM_TILE) == 7
        assert cdmt.cdmt_plan_get(p, cdmt.CDMT_OPT_CHIRP_EXACT) == 0
        cdmt.cdmt_plan_set(p, cdmt.CDMT_OPT_CHIRP_EXACT, 1)
        assert cdmt.cdmt_plan_get(p, cdmt.CDMT_OPT_CHIRP_EXACT) == 1
        assert lib.cdmt_plan_set(p, cdmt.CDMT_OPT_CHIRP_EXACT, 2) == cdmt.CDMT_E_ARG
        assert cdmt.cdmt_plan_get(p, cdmt.CDMT_OPT_LANE_BINS) == 16
        cdmt.cdmt_plan_set(p, cdmt.CDMT_OPT_LANE_BINS, 8)
        assert cdmt.cdmt_plan_get(p, cdmt.CDMT_OPT_LANE_BINS) == 8
        assert lib.cdmt_plan_set(p, cdmt.CDMT_OPT_LANE_BINS, 4) == cdmt.CDMT_E_ARG
        # forward split of N_bin = 16384: 2^7 x 2^7 by default; N2 in {64, 128, 256}
        assert cdmt.cdmt_plan_get(p, cdmt.CDMT_OPT_FWD_N2) == 128
        for n2 in (64, 256, 128):
            cdmt.cdmt_plan_set(p, cdmt.CDMT_OPT_FWD_N2, n2)
            assert cdmt.cdmt_plan_get(p, cdmt.CDMT_OPT_FWD_N2) == n2
        for n2 in (32, 512, 100, 0):
            assert lib.cdmt_plan_set(p, cdmt.CDMT_OPT_FWD_N2, n2) == cdmt.CDMT_E_ARG
        assert cdmt.cdmt_plan_get(p, cdmt.CDMT_OPT_OUT_LAYOUT) == 0
        cdmt.cdmt_plan_set(p, cdmt.CDMT_OPT_OUT_LAYOUT, 1)
        assert cdmt.cdmt_plan_get(p, cdmt.CDMT_OPT_OUT_LAYOUT) == 1
        assert lib.cdmt_plan_set(p, cdmt.CDMT_OPT_OUT_LAYOUT, 2) == cdmt.CDMT_E_ARG
        for opt, val, want in ((cdmt.CDMT_OPT_SIGN, 0, cdmt.CDMT_E_ARG),
                               (cdmt.CDMT_OPT_INPUT, 2, cdmt.CDMT_E_ARG),
                               (cdmt.CDMT_OPT_DM_TILE, 0, cdmt.CDMT_E_ARG),
                               (cdmt.CDMT_OPT_DM_TILE, 65, cdmt.CDMT_E_ARG),
                               (cdmt.CDMT_OPT_PRECISION, 1, cdmt.CDMT_E_UNSUPPORTED),
                               (99, 0, cdmt.CDMT_E_ARG)):
            assert lib.cdmt_plan_set(p, opt, val) == want
    finally:
        cdmt.cdmt_destroy(p)


@pytest.mark.parametrize("w", [synth.TINY, synth.LOFAR], ids=lambda w: w.name)
def test_shapes_follow_section3(lib, w):
    p = cdmt.cdmt_plan(w.nsub, w.f_centre, w.bw, w.nfft, w.noverlap, w.nchan, w.ndec)
    try:
        ntin, ntout, nch = cdmt.cdmt_output_shape(p, w.nblock)
        assert ntin == w.ntime_in
        assert ntout == w.nblock * (w.m - w.nd) // w.ndec
        assert nch == w.nsub * w.nchan
        ws = cdmt.cdmt_workspace_size(p, w.nblock)
        assert ws == 2 * w.nblock * w.nsub * w.nfft * 16
    finally:
        cdmt.cdmt_destroy(p)
    if w is synth.LOFAR:
        assert (ntin, ntout, nch) == (1972224, 15288, 4608)


def test_noverlap_helper_matches_eq2(lib):
    w = synth.LOFAR
    f_lo = w.f_centre - w.nsub * w.bw / 2
    # subband-wide sweep at DM 63.5 -> 15360 (the LOFAR workload's overlap)
    nov = cdmt.cdmt_noverlap_for(f_lo, w.bw, 63.5, w.nchan, w.ndec, cdmt.CHIRP_SUBBAND)
    assert nov == w.noverlap
    for ref, nc, ndec, dm in ((cdmt.CHIRP_CHANNEL, 16, 8, 63.5), (cdmt.CHIRP_SUBBAND, 8, 4, 15.0),
                              (cdmt.CHIRP_CHANNEL, 8, 1, 80.0), (cdmt.CHIRP_SUBBAND, 1, 1, 0.0)):
        nov = cdmt.cdmt_noverlap_for(110.0, 0.1953125, dm, nc, ndec, ref)
        hi = 110.0 + (0.1953125 / nc if ref == cdmt.CHIRP_CHANNEL else 0.1953125)
        need = 0.1953125e6 * oracle.sweep_seconds(110.0, hi, dm)
        unit = 2 * nc * ndec
        assert nov % unit == 0 and need <= nov < need + unit, (nov, need)


def test_noverlap_helper_rejects_bad_args(lib):
    import ctypes
    v = ctypes.c_int()
    for args in ((-1.0, 0.2, 10.0, 8, 1, 0), (110.0, 0.0, 10.0, 8, 1, 0),
                 (110.0, 0.2, -1.0, 8, 1, 0), (110.0, 0.2, 10.0, 6, 1, 0),
                 (110.0, 0.2, 10.0, 8, 0, 0), (110.0, 0.2, 10.0, 8, 1, 2)):
        assert lib.cdmt_noverlap_for(*args, ctypes.byref(v)) == cdmt.CDMT_E_ARG


def test_noop_calls_touch_nothing(lib):
    """ndm = 0 and nblock = 0 return CDMT_OK before any device work."""
    import ctypes
    p = cdmt.cdmt_plan(*GOOD)
    try:
        dm = (ctypes.c_double * 1)(0.0)
        assert lib.cdmt_dedisperse(p, None, 0, None, 0, dm, 1, None, None) == cdmt.CDMT_OK
        assert lib.cdmt_dedisperse_spectra(p, ctypes.c_void_p(16), 1 << 40, 2, dm, 0, None,
                                           None) == cdmt.CDMT_OK
        assert lib.cdmt_dedisperse(p, None, 0, None, 1, dm, 1, None, None) == cdmt.CDMT_E_ARG
        assert lib.cdmt_dedisperse(p, ctypes.c_void_p(16), 10, ctypes.c_void_p(16), 1, dm, 1,
                                   ctypes.c_void_p(16), None) == cdmt.CDMT_E_WORKSPACE
        bad = (ctypes.c_double * 1)(float("inf"))
        assert lib.cdmt_dedisperse_spectra(p, ctypes.c_void_p(16), 1 << 40, 1, bad, 1,
                                           ctypes.c_void_p(16), None) == cdmt.CDMT_E_ARG
        assert lib.cdmt_forward(None, None, 0, None, 1, None) == cdmt.CDMT_E_ARG
    finally:
        cdmt.cdmt_destroy(p)


def test_redigitise_validation(lib):
    """Workspace formula and the error paths of cdmt_redigitise, all returned
    before any device work."""
    import ctypes
    z = ctypes.c_size_t()
    assert lib.cdmt_redigitise_workspace_size(3, 2049, 10, ctypes.byref(z)) == cdmt.CDMT_OK
    assert z.value == 3 * 3 * 10 * 16          # ceil(2049 / 1024) segments x (mean, M2) FP64
    assert lib.cdmt_redigitise_workspace_size(0, 1, 1, ctypes.byref(z)) == cdmt.CDMT_OK
    assert z.value == 0
    for args in ((-1, 1, 1), (1, 0, 1), (1, 1, 0)):
        assert lib.cdmt_redigitise_workspace_size(*args, ctypes.byref(z)) == cdmt.CDMT_E_ARG
    P = ctypes.c_void_p(16)
    call = lib.cdmt_redigitise
    # ndm = 0: no-op, whatever the pointers
    assert call(None, 0, 5, 4, 64.0, 16.0, None, 0, None, None, None, None) == cdmt.CDMT_OK
    # bad shapes and parameters
    assert call(P, 1, 0, 4, 64.0, 16.0, P, 1 << 30, P, P, P, None) == cdmt.CDMT_E_ARG
    assert call(P, 1, 5, 0, 64.0, 16.0, P, 1 << 30, P, P, P, None) == cdmt.CDMT_E_ARG
    assert call(P, 1, 5, 4, float("nan"), 16.0, P, 1 << 30, P, P, P, None) == cdmt.CDMT_E_ARG
    assert call(P, 1, 5, 4, 64.0, 0.0, P, 1 << 30, P, P, P, None) == cdmt.CDMT_E_ARG
    assert call(P, 1, 5, 4, 64.0, float("inf"), P, 1 << 30, P, P, P, None) == cdmt.CDMT_E_ARG
    assert call(None, 1, 5, 4, 64.0, 16.0, P, 1 << 30, P, P, P, None) == cdmt.CDMT_E_ARG
    assert call(P, 1, 5, 4, 64.0, 16.0, P, 1 << 30, None, P, P, None) == cdmt.CDMT_E_ARG
    # too many DMs or segments for one launch
    assert call(P, 65536, 5, 4, 64.0, 16.0, P, 1 << 40, P, P, P, None) == cdmt.CDMT_E_SHAPE
    assert call(P, 1, 65536 * 1024 + 1, 4, 64.0, 16.0, P, 1 << 40, P, P, P,
                None) == cdmt.CDMT_E_SHAPE
    # workspace one byte short
    assert call(P, 2, 1025, 4, 64.0, 16.0, P, 2 * 2 * 4 * 16 - 1, P, P, P,
                None) == cdmt.CDMT_E_WORKSPACE


def test_batch_validation(lib):
    """cdmt_batch_* argument checks, all returned before any device work."""
    import ctypes
    p1 = cdmt.cdmt_plan(*GOOD)                                   # M = 2048
    p2 = cdmt.cdmt_plan(2, 120.0, 0.1953125, 65536, 4096, 8, 4)  # M = 8192
    p3 = cdmt.cdmt_plan(2, 120.0, 0.1953125, 65536, 4096, 16, 4)
    try:
        dms = (ctypes.c_double * 3)(0.0, 1.0, 2.0)
        P = ctypes.c_void_p(256)

        def beams(*specs):
            arr = (cdmt.Beam * len(specs))()
            for i, (plan, nblock, ndm, d) in enumerate(specs):
                arr[i] = cdmt.Beam(plan, nblock, P.value, d, ndm, P.value)
            return arr

        z = ctypes.c_size_t()
        good = beams((p1, 2, 3, dms), (p3, 1, 3, dms))
        assert lib.cdmt_batch_workspace_size(good, 2, ctypes.byref(z)) == cdmt.CDMT_OK
        w1 = cdmt.cdmt_workspace_size(p1, 2)
        w3 = cdmt.cdmt_workspace_size(p3, 1)
        up = lambda v: (v + 255) // 256 * 256
        # spectra of each beam, the DM lists, the table, 14 x 8 queue counters
        assert z.value > up(up(w1) + w3) + 6 * 8
        assert z.value < up(up(w1) + w3) + 4096 + 14 * 8 * 8
        h = ctypes.c_void_p()
        assert lib.cdmt_batch_create(ctypes.byref(h), good, 0, P, 1 << 40) == cdmt.CDMT_E_ARG
        assert lib.cdmt_batch_create(ctypes.byref(h), good, 2, None, 1 << 40) == cdmt.CDMT_E_ARG
        assert lib.cdmt_batch_create(ctypes.byref(h), good, 2, P, z.value - 1) == \
            cdmt.CDMT_E_WORKSPACE
        assert lib.cdmt_batch_create(ctypes.byref(h), beams((p2, 1, 3, dms)), 1, P,
                                     1 << 40) == cdmt.CDMT_E_UNSUPPORTED      # M = 8192
        cdmt.cdmt_plan_set(p3, cdmt.CDMT_OPT_PRECISION, 2)
        assert lib.cdmt_batch_create(ctypes.byref(h), beams((p3, 1, 3, dms)), 1, P,
                                     1 << 40) == cdmt.CDMT_E_UNSUPPORTED      # FP32 only
        cdmt.cdmt_plan_set(p3, cdmt.CDMT_OPT_PRECISION, 0)
        assert lib.cdmt_batch_create(ctypes.byref(h), beams((p1, 0, 3, dms)), 1, P,
                                     1 << 40) == cdmt.CDMT_E_ARG
        assert lib.cdmt_batch_create(ctypes.byref(h), beams((p1, 1, 0, dms)), 1, P,
                                     1 << 40) == cdmt.CDMT_E_ARG
        bad = (ctypes.c_double * 3)(0.0, float("nan"), 2.0)
        assert lib.cdmt_batch_create(ctypes.byref(h), beams((p1, 1, 3, bad)), 1, P,
                                     1 << 40) == cdmt.CDMT_E_ARG
        assert h.value is None
        v = ctypes.c_longlong()
        assert lib.cdmt_batch_set(None, 0, 4) == cdmt.CDMT_E_ARG
        assert lib.cdmt_batch_get(None, 0, ctypes.byref(v)) == cdmt.CDMT_E_ARG
        assert lib.cdmt_batch_run(None, None) == cdmt.CDMT_E_ARG
        assert lib.cdmt_batch_run_graph(None, P) == cdmt.CDMT_E_ARG
        iv = ctypes.c_int()
        assert lib.cdmt_batch_beam_set(None, 0, cdmt.CDMT_BATCH_BEAM_FWD_N2, 128) == cdmt.CDMT_E_ARG
        assert lib.cdmt_batch_beam_get(None, 0, cdmt.CDMT_BATCH_BEAM_FWD_N2,
                                       ctypes.byref(iv)) == cdmt.CDMT_E_ARG
        lib.cdmt_batch_destroy(None)
    finally:
        for p in (p1, p2, p3):
            cdmt.cdmt_destroy(p)


def test_gradient_validation(lib):
    """cdmt_dm_gradient argument checks, returned before any device work."""
    import ctypes
    p = cdmt.cdmt_plan(*GOOD)                                    # M = 2048
    p8 = cdmt.cdmt_plan(2, 120.0, 0.1953125, 65536, 4096, 8, 4)  # M = 8192
    try:
        z = ctypes.c_size_t()
        assert lib.cdmt_gradient_workspace_size(p, 3, 5, ctypes.byref(z)) == cdmt.CDMT_OK
        assert z.value == 5 * (3 * 8 * 8 // 2) * 8        # DMs x chunk groups (2 chunks each) x 8 B
        assert lib.cdmt_gradient_workspace_size(p8, 1, 5, ctypes.byref(z)) == \
            cdmt.CDMT_E_UNSUPPORTED
        assert lib.cdmt_gradient_workspace_size(p, -1, 5, ctypes.byref(z)) == cdmt.CDMT_E_ARG
        P = ctypes.c_void_p(256)
        dm = (ctypes.c_double * 2)(1.0, 2.0)
        g = lib.cdmt_dm_gradient
        big = 1 << 40
        assert g(p, P, big, 2, dm, 0, None, None, 0, None, None) == cdmt.CDMT_OK     # no-op
        assert g(p, P, big, 2, dm, -1, P, P, big, P, None) == cdmt.CDMT_E_ARG
        assert g(p, P, big, 2, dm, 2, None, P, big, P, None) == cdmt.CDMT_E_ARG
        assert g(p, P, big, 2, dm, 2, P, P, 8, P, None) == cdmt.CDMT_E_WORKSPACE
        assert g(p, P, 16, 2, dm, 2, P, P, big, P, None) == cdmt.CDMT_E_WORKSPACE
        assert g(p8, P, big, 1, dm, 2, P, P, big, P, None) == cdmt.CDMT_E_UNSUPPORTED
        bad = (ctypes.c_double * 2)(1.0, float("inf"))
        assert g(p, P, big, 2, bad, 2, P, P, big, P, None) == cdmt.CDMT_E_ARG
    finally:
        cdmt.cdmt_destroy(p)
        cdmt.cdmt_destroy(p8)


def test_voltage_gradient_validation(lib):
    """cdmt_voltage_gradient argument checks, returned before any device work."""
    import ctypes
    p = cdmt.cdmt_plan(*GOOD)
    try:
        z = ctypes.c_size_t()
        assert lib.cdmt_voltage_gradient_workspace_size(p, 2, ctypes.byref(z)) == cdmt.CDMT_OK
        assert z.value == 3 * 2 * 8 * 16384 * 16          # three spectrum-sized buffers
        P = ctypes.c_void_p(256)
        big = 1 << 40
        f = lib.cdmt_voltage_gradient
        assert f(p, P, big, 0, 1.0, None, None, 0, None, 0, None) == cdmt.CDMT_OK       # no-op
        assert f(p, P, big, 2, 1.0, None, P, big, P, 0, None) == cdmt.CDMT_E_ARG
        assert f(p, P, big, 2, float("nan"), P, P, big, P, 0, None) == cdmt.CDMT_E_ARG
        assert f(p, P, big, 2, 1.0, P, P, big, P, 2, None) == cdmt.CDMT_E_ARG           # flag
        assert f(p, P, big, 2, 1.0, P, P, z.value - 1, P, 0, None) == cdmt.CDMT_E_WORKSPACE
    finally:
        cdmt.cdmt_destroy(p)


def test_incoherent_validation(lib):
    """cdmt_incoherent_shape agrees with the oracle's output length (the
    largest Eq. 2 delay), and the argument checks return before device work."""
    import ctypes
    from oracle import incoherent
    p = cdmt.cdmt_plan(*GOOD)
    try:
        cfg = oracle.Config(*GOOD)
        tblk = (16384 // 8 - 4096 // 8) // 4
        for dms, ddm0, ddm, n in (([0.5, 10.0, 20.0], -0.5, 0.01, 101), ([3.0], 0.0, 0.0, 1),
                                  ([1.0, 2.0], 0.0, 2.0, 10)):
            nout = cdmt.cdmt_incoherent_shape(p, 4, dms, ddm0, ddm, n)
            dmax = max(dms) + (ddm0 + ddm * (n - 1))
            assert nout == 4 * tblk - int(incoherent.delays(cfg, dmax).max())
        z = ctypes.c_size_t()
        assert lib.cdmt_incoherent_workspace_size(p, 4, 3, 101, ctypes.byref(z)) == cdmt.CDMT_OK
        # transposed copy, then the delay table (101 trials padded to 108 = 9 groups of 12)
        assert z.value == 3 * 64 * 4 * tblk * 4 + 3 * 108 * 64 * 4
        # a channel-major plan's filterbanks are read as they are: the table only
        cdmt.cdmt_plan_set(p, cdmt.CDMT_OPT_OUT_LAYOUT, 1)
        z1 = ctypes.c_size_t()
        assert lib.cdmt_incoherent_workspace_size(p, 4, 3, 101, ctypes.byref(z1)) == cdmt.CDMT_OK
        assert z1.value == 3 * 108 * 64 * 4
        cdmt.cdmt_plan_set(p, cdmt.CDMT_OPT_OUT_LAYOUT, 0)
        arr = (ctypes.c_double * 3)(0.5, 10.0, 20.0)
        nout = ctypes.c_longlong()
        shape = lib.cdmt_incoherent_shape
        assert shape(p, 4, arr, 3, -0.5, 0.01, 101, ctypes.byref(nout)) == cdmt.CDMT_OK
        assert shape(p, 4, arr, 3, -0.6, 0.01, 101, ctypes.byref(nout)) == cdmt.CDMT_E_ARG  # DM < 0
        assert shape(p, 4, arr, 3, 0.0, 0.0, 2, ctypes.byref(nout)) == cdmt.CDMT_E_ARG      # step
        assert shape(p, 4, arr, 3, 0.0, -0.1, 2, ctypes.byref(nout)) == cdmt.CDMT_E_ARG
        assert shape(p, 4, arr, 3, float("nan"), 0.1, 2, ctypes.byref(nout)) == cdmt.CDMT_E_ARG
        assert shape(p, 4, arr, 0, 0.0, 0.1, 2, ctypes.byref(nout)) == cdmt.CDMT_E_ARG
        assert shape(p, 4, arr, 3, 0.0, 0.1, 0, ctypes.byref(nout)) == cdmt.CDMT_E_ARG
        assert shape(p, 1, arr, 3, 0.0, 1.0, 900, ctypes.byref(nout)) == cdmt.CDMT_E_SHAPE  # no sample
        P = ctypes.c_void_p(256)
        f = lib.cdmt_incoherent
        assert f(p, 4, P, arr, 3, -0.5, 0.01, 101, P, z.value - 1, P, None) == cdmt.CDMT_E_WORKSPACE
        assert f(p, 4, None, arr, 3, -0.5, 0.01, 101, P, z.value, P, None) == cdmt.CDMT_E_ARG
        assert f(p, 4, P, arr, 3, -0.5, 0.01, 101, P, z.value, None, None) == cdmt.CDMT_E_ARG
    finally:
        cdmt.cdmt_destroy(p)


def _eq2_limit(f_lo, bw, nchan, nov, chirp_ref):
    """Largest DM whose Eq. 2 sweep (Sec. 2) over the lowest channel (or
    subband), times the sample rate bw, is at most the overlap."""
    hi = f_lo + (bw / nchan if chirp_ref == cdmt.CHIRP_CHANNEL else bw)
    return nov / (bw * 1e6 * oracle.sweep_seconds(f_lo, hi, 1.0))


def test_dm_limit_is_eq2_for_the_overlap(lib):
    """cdmt_dm_limit inverts the overlap sizing of Sec. 2 / Eq. 2: the LOFAR
    plan (overlap sized for DM 63.5 over the lowest subband) supports its
    128 trials in both nu0 modes, and cdmt_noverlap_for at the limit gives
    back the plan's overlap."""
    import ctypes
    w = synth.LOFAR
    f_lo = w.f_centre - w.nsub * w.bw / 2
    for ref in (cdmt.CHIRP_CHANNEL, cdmt.CHIRP_SUBBAND):
        p = cdmt.cdmt_plan(w.nsub, w.f_centre, w.bw, w.nfft, w.noverlap, w.nchan, w.ndec)
        try:
            cdmt.cdmt_plan_set(p, cdmt.CDMT_OPT_CHIRP_REF, ref)
            lim = cdmt.cdmt_dm_limit(p)
            assert lim == pytest.approx(_eq2_limit(f_lo, w.bw, w.nchan, w.noverlap, ref),
                                        rel=1e-12)
            assert lim >= 63.5
            nov = cdmt.cdmt_noverlap_for(f_lo, w.bw, lim, w.nchan, w.ndec, ref)
            assert nov == w.noverlap
        finally:
            cdmt.cdmt_destroy(p)
    # nu0 per subband: the subband-wide sweep of DM 63.5 is 15114.5 samples
    p = cdmt.cdmt_plan(w.nsub, w.f_centre, w.bw, w.nfft, w.noverlap, w.nchan, w.ndec)
    try:
        cdmt.cdmt_plan_set(p, cdmt.CDMT_OPT_CHIRP_REF, cdmt.CHIRP_SUBBAND)
        assert 63.5 * w.noverlap / 15115 < cdmt.cdmt_dm_limit(p) < 63.5 * w.noverlap / 15114
    finally:
        cdmt.cdmt_destroy(p)
    v = ctypes.c_double()
    assert lib.cdmt_dm_limit(None, ctypes.byref(v)) == cdmt.CDMT_E_ARG


def test_dm_beyond_the_overlap_is_rejected(lib):
    """Every call that takes DMs rejects |DM| above cdmt_dm_limit with
    CDMT_E_SHAPE before any device work, accepts DM 63.5 and the limit
    itself on the LOFAR plan (nu0 per subband), and CDMT_OPT_DM_CHECK = 0
    lifts the check."""
    import ctypes
    import math
    w = synth.LOFAR
    p = cdmt.cdmt_plan(w.nsub, w.f_centre, w.bw, w.nfft, w.noverlap, w.nchan, w.ndec)
    try:
        cdmt.cdmt_plan_set(p, cdmt.CDMT_OPT_CHIRP_REF, cdmt.CHIRP_SUBBAND)
        assert cdmt.cdmt_plan_get(p, cdmt.CDMT_OPT_DM_CHECK) == 1
        lim = cdmt.cdmt_dm_limit(p)
        past = math.nextafter(lim * (1 + 1e-12), math.inf)
        P = ctypes.c_void_p(256)
        big = 1 << 44
        arr = lambda *d: (ctypes.c_double * len(d))(*d)
        beams = lambda d: (cdmt.Beam * 1)(cdmt.Beam(p, 1, P.value, d, len(d), P.value))
        z = ctypes.c_size_t()
        # the batch sizing validates DM lists without touching the device
        for good in (arr(0.0, 63.5), arr(lim), arr(-lim)):
            assert lib.cdmt_batch_workspace_size(beams(good), 1, ctypes.byref(z)) == cdmt.CDMT_OK
        for bad in (arr(0.0, past), arr(-past)):
            assert lib.cdmt_batch_workspace_size(beams(bad), 1, ctypes.byref(z)) == \
                cdmt.CDMT_E_SHAPE
            n = len(bad)
            assert lib.cdmt_dedisperse_spectra(p, P, big, 1, bad, n, P, None) == cdmt.CDMT_E_SHAPE
            assert lib.cdmt_dedisperse(p, P, big, P, 1, bad, n, P, None) == cdmt.CDMT_E_SHAPE
            assert lib.cdmt_dm_gradient(p, P, big, 1, bad, n, P, P, big, P,
                                        None) == cdmt.CDMT_E_SHAPE
            h = ctypes.c_void_p()
            assert lib.cdmt_batch_create(ctypes.byref(h), beams(bad), 1, P, big) == \
                cdmt.CDMT_E_SHAPE
        assert lib.cdmt_voltage_gradient(p, P, big, 1, past, P, P, big, P, 0,
                                         None) == cdmt.CDMT_E_SHAPE
        cdmt.cdmt_plan_set(p, cdmt.CDMT_OPT_DM_CHECK, 0)
        assert lib.cdmt_batch_workspace_size(beams(arr(0.0, past, 2 * lim)), 1,
                                             ctypes.byref(z)) == cdmt.CDMT_OK
        assert lib.cdmt_plan_set(p, cdmt.CDMT_OPT_DM_CHECK, 2) == cdmt.CDMT_E_ARG
    finally:
        cdmt.cdmt_destroy(p)


def test_nfft_range_is_2_10_to_2_17(lib):
    """N_bin from 2^10 (one-pass forward transform) to 2^17 is accepted."""
    for nfft, nchan in ((1024, 8), (2048, 8), (4096, 8), (1 << 17, 16)):
        assert _plan_status(2, 120.0, 0.1953125, nfft, 256, nchan, 4) == cdmt.CDMT_OK, nfft
    assert _plan_status(2, 120.0, 0.1953125, 512, 0, 8, 4) == cdmt.CDMT_E_UNSUPPORTED
    assert _plan_status(2, 120.0, 0.1953125, 1 << 18, 256, 8, 4) == cdmt.CDMT_E_UNSUPPORTED
    p = cdmt.cdmt_plan(2, 120.0, 0.1953125, 2048, 256, 8, 4)
    try:
        # one pass: no four-step split to choose
        assert cdmt.load().cdmt_plan_set(p, cdmt.CDMT_OPT_FWD_N2, 64) == cdmt.CDMT_E_ARG
    finally:
        cdmt.cdmt_destroy(p)


def test_binding_checks_out_and_workspace_before_any_launch(lib):
    """Plan.dedisperse_spectra takes an output tensor the C call cannot size:
    a wrong dtype, shape, layout or device raises ValueError before the
    library is called (CPU tensors here, so nothing can launch)."""
    import torch
    plan = cdmt.Plan(*GOOD)
    ws = torch.empty(16, dtype=torch.uint8)
    shape = plan.out_shape(2, 1)
    good_shape = torch.empty(shape, dtype=torch.float32)
    for out in (torch.empty(shape, dtype=torch.float64),
                torch.empty((2, shape[1] - 1, shape[2]), dtype=torch.float32),
                torch.empty((2, shape[2], shape[1]), dtype=torch.float32).transpose(1, 2),
                torch.empty((1,) + shape[1:], dtype=torch.float32),
                good_shape):                                     # right shape, not on the device
        with pytest.raises(ValueError):
            plan.dedisperse_spectra(1, [0.0, 1.0], out, ws)
    with pytest.raises(ValueError):
        plan._check_workspace(torch.empty(4, dtype=torch.float32))
