"""Parity of the split-precision matrix-core DM stage (BF16x3, FP16x3) with
the FP64 oracle, on M_bin = 4096 shapes (the LOFAR channel chunk).

Bars: FP16x3 (11+11 significant bits per operand) is held to the FP32
path's 1e-5 normwise bar.  BF16x3: with u = 2^-8 (BF16's unit roundoff) a
split operand x = hi + lo carries at most u^2 |x| of representation error and
the dropped lo*lo product at most u^2 |a||b|, so each product in a radix-16
stage is off by at most 3 u^2 relative, and a detected power after three
stages by at most 2 * 3 * 3 u^2 = 2.7e-4 relative: the max-abs/max bar.  The
per-product errors are rounding errors of random sign, about u^2 / sqrt(12)
each (RMS); three such sources per product, three stages and the square give
a normwise power error of at most about 2 sqrt(3) sqrt(3) u^2 / sqrt(12) =
2.6e-5 (an estimate with every source at full strength); the normwise bar is
5e-5 (measured 3.5e-6).  The measured figures are printed."""
import numpy as np
import pytest

import oracle
from paper_1607_00909_amd import synth

pytestmark = pytest.mark.gpu

BARS = {1: (5e-5, 2.7e-4), 2: (1e-5, 1e-5)}
NAMES = {1: "bf16x3", 2: "fp16x3"}


def _errors(gpu, ref):
    d = gpu.astype(np.float64) - ref
    per_dm = np.sqrt((d ** 2).reshape(d.shape[0], -1).sum(1) / (ref ** 2).reshape(d.shape[0], -1).sum(1))
    return float(per_dm.max()), float(np.abs(d).max() / np.abs(ref).max())


@pytest.mark.parametrize("prec", [2, 1], ids=["fp16x3", "bf16x3"])
@pytest.mark.parametrize("exact", [0, 1], ids=["recurrence", "exact"])
@pytest.mark.parametrize("kind,ref_mode,sigma", [("ci8", oracle.CHANNEL, 16.0),
                                                  ("cf32", oracle.SUBBAND, 1e-3)],
                         ids=["ci8-channel", "cf32-subband-small"])
def test_mixed_precision_parity(hip_lib, prec, exact, kind, ref_mode, sigma):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cfg = oracle.Config(2, 110.0, synth.SUBBAND_MHZ, 65536, 15360, 16, 8, chirp_ref=ref_mode)
    nblock = 2
    print(f"[gpu-case] mixed {NAMES[prec]} exact={exact} {kind}", flush=True)
    x = synth.gaussian_voltages(cfg.nsub, cfg.ntime_in(nblock), sigma, 77)
    t0 = cfg.tblk // 2 + cfg.tblk
    for s in range(cfg.nsub):
        oracle.inject_impulse(cfg, x, s, 30.0, oracle.pulse_sample(cfg, t0), 20.0 * sigma)
    v = synth.encode_ci8(x)[0] if kind == "ci8" else synth.encode_cf32(x)
    dms = list(np.arange(0.0, 48.0, 3.0))
    ref = oracle.dedisperse(cfg, v, nblock, dms)
    plan = hip_lib.Plan(cfg.nsub, cfg.f_centre, cfg.bw, cfg.nfft, cfg.noverlap, cfg.nchan,
                        cfg.ndec, input_kind=hip_lib.INPUT_CI8 if kind == "ci8" else hip_lib.INPUT_CF32,
                        chirp_ref=ref_mode, chirp_exact=exact)
    hip_lib.cdmt_plan_set(plan.handle, hip_lib.CDMT_OPT_PRECISION, prec)
    out = plan.dedisperse(torch.from_numpy(v).cuda(), nblock, dms)
    torch.cuda.synchronize()
    gpu = out.cpu().numpy()
    e_norm, e_max = _errors(gpu, ref)
    print(f"{NAMES[prec]} exact={exact} {kind}: max_d normwise {e_norm:.3e}, "
          f"max-abs/max {e_max:.3e}", flush=True)
    bn, bm = BARS[prec]
    assert e_norm <= bn and e_max <= bm
    sg, sr = gpu.sum(axis=2), ref.sum(axis=2)
    assert np.unravel_index(np.argmax(sg), sg.shape) == np.unravel_index(np.argmax(sr), sr.shape)


def test_mixed_precision_rejected_off_4096(hip_lib):
    plan = hip_lib.Plan(2, 120.0, synth.SUBBAND_MHZ, 16384, 4096, 8, 4)
    assert hip_lib.load().cdmt_plan_set(plan.handle, hip_lib.CDMT_OPT_PRECISION, 1) == \
        hip_lib.CDMT_E_UNSUPPORTED
