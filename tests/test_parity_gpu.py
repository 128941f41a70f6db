"""GPU parity: the HIP library against the FP64 oracle on the same bytes.

Bar (FP32 path): for every DM trial the normwise relative error of the
filterbank power, ||F_gpu - F_ref||_2 / ||F_ref||_2, is at most 1e-5.  The
largest elementwise error relative to the filterbank maximum is reported and
held to the same bound.  Integer decisions (where an impulse recompresses)
must agree exactly.
"""
import numpy as np
import pytest

import oracle
from conftest import allow_short_overlap
from paper_1607_00909_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _errors(gpu, ref):
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    d = gpu - ref
    per_dm = np.sqrt((d ** 2).reshape(d.shape[0], -1).sum(1) / (ref ** 2).reshape(d.shape[0], -1).sum(1))
    return float(per_dm.max()), float(np.abs(d).max() / np.abs(ref).max())


def _plan(cdmt, cfg, kind, **kw):
    return cdmt.Plan(cfg.nsub, cfg.f_centre, cfg.bw, cfg.nfft, cfg.noverlap, cfg.nchan, cfg.ndec,
                     input_kind=cdmt.INPUT_CI8 if kind == "ci8" else cdmt.INPUT_CF32,
                     chirp_ref=cfg.chirp_ref, sign=cfg.sign, **kw)


def _voltages(cfg, nblock, sigma, seed, kind, pulses=()):
    x = synth.gaussian_voltages(cfg.nsub, cfg.ntime_in(nblock), sigma, seed)
    for dm, t0, amp in pulses:
        for s in range(cfg.nsub):
            oracle.inject_impulse(cfg, x, s, dm, oracle.pulse_sample(cfg, t0), amp)
    if kind == "ci8":
        v, _ = synth.encode_ci8(x)
    else:
        v = synth.encode_cf32(x)
    return v


def _run_gpu(hip_lib, cfg, v, nblock, dms, kind, **kw):
    torch = _torch()
    plan = _plan(hip_lib, cfg, kind, **kw)
    allow_short_overlap(plan, dms)
    xd = torch.from_numpy(v).cuda()
    out = plan.dedisperse(xd, nblock, list(dms))
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _tiny_cfg(chirp_ref):
    w = synth.TINY
    return oracle.Config(w.nsub, w.f_centre, w.bw, w.nfft, w.noverlap, w.nchan, w.ndec,
                         chirp_ref=chirp_ref, sign=-1)


@pytest.mark.parametrize("lane_bins", [16, 8])
@pytest.mark.parametrize("exact", [0, 1], ids=["recurrence", "exact"])
@pytest.mark.parametrize("chirp_ref", [oracle.CHANNEL, oracle.SUBBAND], ids=["channel", "subband"])
def test_tiny_workload_parity_and_recompression(hip_lib, chirp_ref, exact, lane_bins):
    """8 subbands (120.0-121.5625 MHz), cf32 noise sigma 1 plus a 20-sigma
    impulse dispersed at DM 10, nfft 16384 / noverlap 4096, 4 blocks, DMs
    0..15, 8 channels, x4 downsampling; transfer function evaluated per DM
    (exact) or advanced through each DM tile (recurrence)."""
    w = synth.TINY
    cfg = _tiny_cfg(chirp_ref)
    _say(f"tiny workload chirp_ref={chirp_ref} exact={exact} lane_bins={lane_bins}")
    t0 = w.tblk + w.tblk // 2
    v = _voltages(cfg, w.nblock, w.sigma, w.seed, "cf32",
                  pulses=[(w.extra["pulse_dm"], t0, w.pulse_amp_sigma * w.sigma)])
    ref = oracle.dedisperse(cfg, v, w.nblock, w.dms)
    gpu = _run_gpu(hip_lib, cfg, v, w.nblock, w.dms, "cf32", chirp_exact=exact, dm_tile=16,
                   lane_bins=lane_bins)
    assert gpu.shape == ref.shape
    e_norm, e_max = _errors(gpu, ref)
    print(f"tiny chirp_ref={chirp_ref} exact={exact} bins={lane_bins}: max_d normwise {e_norm:.3e}, "
          f"max-abs/max {e_max:.3e}")
    assert e_norm <= TOL and e_max <= TOL
    # the pulse recompresses at the same (DM, t) on both sides
    sg, sr = gpu.sum(axis=2), ref.sum(axis=2)
    assert np.unravel_index(np.argmax(sg), sg.shape) == np.unravel_index(np.argmax(sr), sr.shape)
    assert np.unravel_index(np.argmax(sg), sg.shape) == (10, t0)


CASES = [
    # nsub, nfft, noverlap, nchan, ndec, nblock, kind, chirp_ref, sign, ndm, dm_tile
    (3, 4096, 1024, 64, 2, 2, "ci8", oracle.CHANNEL, -1, 5, 4),      # M = 64, 64 chunks / WG
    (2, 8192, 1024, 32, 4, 3, "cf32", oracle.SUBBAND, -1, 7, 3),     # M = 256
    (2, 8192, 2048, 16, 1, 2, "ci8", oracle.CHANNEL, 1, 4, 16),      # M = 512, sign +1
    (3, 16384, 1024, 16, 3, 2, "cf32", oracle.CHANNEL, -1, 6, 2),    # M = 1024, ndec 3
    (1, 32768, 8192, 8, 8, 2, "ci8", oracle.SUBBAND, -1, 9, 4),      # M = 4096, nfft 2^15
    (2, 65536, 15360, 16, 8, 2, "ci8", oracle.CHANNEL, -1, 9, 4),    # LOFAR chunk shape
    (1, 65536, 8192, 16, 1, 2, "cf32", oracle.CHANNEL, -1, 5, 4),    # M = 4096, ndec 1
    (1, 65536, 8192, 16, 2, 2, "ci8", oracle.SUBBAND, 1, 5, 3),      # M = 4096, ndec 2
    (1, 65536, 8192, 16, 4, 2, "cf32", oracle.CHANNEL, -1, 6, 16),   # M = 4096, ndec 4
    (2, 65536, 15360, 16, 8, 2, "ci8", oracle.SUBBAND, -1, 9, 8, 8), # same, 8 bins per lane
    (1, 32768, 4096, 16, 2, 2, "cf32", oracle.CHANNEL, 1, 5, 2, 8),  # M = 2048, 8 bins per lane
    (2, 32768, 4096, 16, 4, 2, "ci8", oracle.SUBBAND, -1, 6, 4),     # M = 2048, three passes
    (1, 32768, 4096, 16, 8, 2, "cf32", oracle.CHANNEL, 1, 5, 16),    # same, ndec 8
    (3, 2048, 512, 1, 2, 3, "cf32", oracle.CHANNEL, -1, 5, 4),       # M = 2048, 9 chunks (odd)
    (2, 16384, 2048, 16, 2, 2, "cf32", oracle.SUBBAND, 1, 5, 16),    # M = 1024, three passes
    (3, 1024, 256, 1, 8, 3, "ci8", oracle.CHANNEL, -1, 5, 4),        # M = 1024, 9 chunks
    (1, 131072, 16384, 16, 4, 2, "cf32", oracle.CHANNEL, -1, 3, 1),  # M = 8192, nfft 2^17
    (3, 1024, 256, 8, 2, 3, "ci8", oracle.CHANNEL, -1, 5, 4),        # nfft 2^10, one-pass forward
    (2, 2048, 512, 16, 4, 3, "cf32", oracle.SUBBAND, 1, 6, 3),       # nfft 2^11, M = 128
    (5, 2048, 256, 2, 4, 2, "ci8", oracle.SUBBAND, -1, 4, 16),       # nfft 2^11, M = 1024
]


@pytest.mark.parametrize("case", CASES, ids=[f"M{c[1] // c[3]}-nfft{c[1]}-ndec{c[4]}-{c[6]}"
                                             f"-b{(c + (16,))[11]}" for c in CASES])
def test_shapes_parity(hip_lib, case):
    nsub, nfft, nov, nchan, ndec, nblock, kind, ref_mode, sign, ndm, tile = case[:11]
    bins = case[11] if len(case) > 11 else 16
    cfg = oracle.Config(nsub, 138.0, synth.SUBBAND_MHZ, nfft, nov, nchan, ndec,
                        chirp_ref=ref_mode, sign=sign)
    _say(f"shapes case {case}")
    sigma = 16.0 if kind == "ci8" else 1.0
    v = _voltages(cfg, nblock, sigma, 11 + nfft, kind)
    dms = list(np.linspace(-3.0, 60.0, ndm))
    ref = oracle.dedisperse(cfg, v, nblock, dms)
    gpu = _run_gpu(hip_lib, cfg, v, nblock, dms, kind, dm_tile=tile, lane_bins=bins)
    e_norm, e_max = _errors(gpu, ref)
    print(f"case {case}: max_d normwise {e_norm:.3e}, max-abs/max {e_max:.3e}")
    assert e_norm <= TOL and e_max <= TOL


SPLITS = [  # nfft, nchan, noverlap, N2 (the non-default forward splits)
    (8192, 32, 1024, 128), (16384, 16, 2048, 64), (16384, 16, 2048, 256),
    (32768, 8, 4096, 64), (32768, 8, 4096, 256), (65536, 16, 15360, 128),
]


@pytest.mark.parametrize("case", SPLITS, ids=[f"nfft{c[0]}-N2_{c[3]}" for c in SPLITS])
def test_forward_splits_parity(hip_lib, case):
    """Every non-default four-step split of the forward FFT (CDMT_OPT_FWD_N2,
    the radix schedules the batch autotuner chooses from) against the oracle."""
    nfft, nchan, nov, n2 = case
    cfg = oracle.Config(2, 130.0, synth.SUBBAND_MHZ, nfft, nov, nchan, 4)
    _say(f"forward split case {case}")
    v = _voltages(cfg, 2, 16.0, 5 + n2, "ci8")
    dms = [0.0, 7.5, 31.0]
    ref = oracle.dedisperse(cfg, v, 2, dms)
    gpu = _run_gpu(hip_lib, cfg, v, 2, dms, "ci8", fwd_n2=n2)
    e_norm, e_max = _errors(gpu, ref)
    print(f"split {case}: max_d normwise {e_norm:.3e}, max-abs/max {e_max:.3e}")
    assert e_norm <= TOL and e_max <= TOL


LAYOUT_CASES = [  # nfft, noverlap, nchan, ndec, mode, options
    (16384, 4096, 8, 4, oracle.CHANNEL, {}),                                # M 2048, recurrence
    (16384, 4096, 8, 4, oracle.SUBBAND, {"chirp_exact": 1}),
    (65536, 15360, 16, 8, oracle.CHANNEL, {"lane_bins": 8}),                # M 4096, 8 bins/lane
    (65536, 15360, 16, 8, oracle.CHANNEL, {"precision": 2}),                # FP16x3 matrix cores
    (8192, 1024, 64, 2, oracle.CHANNEL, {}),                                # M 128, 32 chunks/WG
]


@pytest.mark.parametrize("case", LAYOUT_CASES, ids=[f"nfft{c[0]}-{'-'.join(c[5]) or 'fp32'}"
                                                    for c in LAYOUT_CASES])
def test_channel_major_layout_is_the_transpose(hip_lib, case):
    """CDMT_OPT_OUT_LAYOUT = 1 writes the same filterbank [DM][channel][time],
    bit for bit the transpose of the default layout."""
    torch = _torch()
    nfft, nov, nchan, ndec, mode, opts = case
    cfg = oracle.Config(3, 125.0, synth.SUBBAND_MHZ, nfft, nov, nchan, ndec, chirp_ref=mode)
    _say(f"layout case {case}")
    v = torch.from_numpy(_voltages(cfg, 2, 16.0, 71, "ci8")).cuda()
    dms = list(np.arange(0.0, 36.0, 2.25))
    outs = []
    for layout in (0, 1):
        kw = {k: val for k, val in opts.items() if k != "precision"}
        plan = _plan(hip_lib, cfg, "ci8", out_layout=layout, **kw)
        allow_short_overlap(plan, dms)
        if "precision" in opts:
            hip_lib.cdmt_plan_set(plan.handle, hip_lib.CDMT_OPT_PRECISION, opts["precision"])
        outs.append(plan.dedisperse(v, 2, dms))
    torch.cuda.synchronize()
    assert outs[1].shape == (len(dms), outs[0].shape[2], outs[0].shape[1])
    assert torch.equal(outs[1], outs[0].transpose(1, 2).contiguous())


def test_dm_tile_and_repeat_bitwise_identical(hip_lib):
    """With the transfer function evaluated per DM, the result of a DM does
    not depend on how DMs are tiled per workgroup, and repeated runs are
    bitwise identical (no atomics, no races).  The recurrence mode is also
    repeatable bitwise and agrees with the exact mode to the parity bar."""
    cfg = _tiny_cfg(oracle.CHANNEL)
    _say("dm tile invariance")
    v = _voltages(cfg, 2, 1.0, 3, "cf32")
    dms = list(np.arange(13) * 1.25)
    outs = [_run_gpu(hip_lib, cfg, v, 2, dms, "cf32", dm_tile=t, chirp_exact=1)
            for t in (1, 3, 4, 16, 4)]
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])
    rec = [_run_gpu(hip_lib, cfg, v, 2, dms, "cf32", dm_tile=t) for t in (16, 16, 3)]
    np.testing.assert_array_equal(rec[0], rec[1])
    for r in (rec[0], rec[2]):
        e_norm, e_max = _errors(r, outs[0])
        assert e_norm <= TOL and e_max <= TOL


def test_non_uniform_dm_list_uses_exact_path(hip_lib):
    """A DM list that is not an arithmetic progression (random, unsorted,
    negative values) is evaluated per DM and matches the oracle."""
    cfg = _tiny_cfg(oracle.SUBBAND)
    _say("random DM list")
    v = _voltages(cfg, 2, 1.0, 21, "cf32")
    dms = list(np.random.default_rng(5).uniform(-20.0, 80.0, 11))
    ref = oracle.dedisperse(cfg, v, 2, dms)
    gpu = _run_gpu(hip_lib, cfg, v, 2, dms, "cf32", dm_tile=4)
    e_norm, e_max = _errors(gpu, ref)
    print(f"random DMs: max_d normwise {e_norm:.3e}, max-abs/max {e_max:.3e}")
    assert e_norm <= TOL and e_max <= TOL


def test_more_dms_than_one_launch(hip_lib):
    """More than 256 DM trials are split over several launches."""
    cfg = oracle.Config(1, 120.0, synth.SUBBAND_MHZ, 4096, 512, 8, 2)
    _say("300 DMs")
    v = _voltages(cfg, 2, 1.0, 4, "cf32")
    dms = list(np.linspace(0.0, 30.0, 300))
    ref = oracle.dedisperse(cfg, v, 2, dms)
    gpu = _run_gpu(hip_lib, cfg, v, 2, dms, "cf32", dm_tile=16)
    e_norm, e_max = _errors(gpu, ref)
    assert e_norm <= TOL and e_max <= TOL


def test_forward_then_spectra_matches_one_call(hip_lib):
    """cdmt_forward + cdmt_dedisperse_spectra (two DM lists on one set of
    spectra) equals cdmt_dedisperse bitwise (transfer function per DM)."""
    torch = _torch()
    cfg = _tiny_cfg(oracle.SUBBAND)
    _say("forward + spectra split")
    v = _voltages(cfg, 2, 1.0, 8, "cf32")
    plan = _plan(hip_lib, cfg, "cf32", chirp_exact=1)
    xd = torch.from_numpy(v).cuda()
    whole = plan.dedisperse(xd, 2, [1.0, 2.0, 3.0]).cpu().numpy()
    ws = plan.workspace(2)
    _, ntout, nch = plan.shape(2)
    out = torch.zeros((3, ntout, nch), device="cuda")
    plan.forward(xd, 2, ws)
    plan.dedisperse_spectra(2, [1.0, 2.0], out[:2], ws)
    plan.dedisperse_spectra(2, [3.0], out[2:], ws)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), whole)


def test_errors_write_nothing(hip_lib):
    torch = _torch()
    cfg = _tiny_cfg(oracle.CHANNEL)
    _say("error paths")
    plan = _plan(hip_lib, cfg, "cf32")
    v = _voltages(cfg, 1, 1.0, 1, "cf32")
    xd = torch.from_numpy(v).cuda()
    _, ntout, nch = plan.shape(1)
    out = torch.full((2, ntout, nch), -7.0, device="cuda")
    small = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(hip_lib.CdmtError) as e:
        plan.dedisperse(xd, 1, [0.0, 1.0], out=out, workspace=small)
    assert e.value.status == hip_lib.CDMT_E_WORKSPACE
    with pytest.raises(hip_lib.CdmtError) as e:
        plan.dedisperse(xd, 1, [0.0, float("nan")], out=out)
    assert e.value.status == hip_lib.CDMT_E_ARG
    torch.cuda.synchronize()
    assert bool((out == -7.0).all())
