"""S/N of injected pulses after dedispersion: FP32 vector path and the two
split-precision matrix-core paths, against the FP64 oracle at the pulse DMs.

Workload: a slice of the LOFAR HBA setup (8 of its subbands around 138 MHz,
6 blocks of nfft 65536 / noverlap 15360, 16 channels, x8 downsampling, the
128-trial grid 0..63.5), complex int8 noise with sigma 16 and five impulses of
20 sigma dispersed by the oracle at trial DMs drawn from [5, 60].  S/N of a
pulse = (peak - median) / (1.4826 MAD) of the channel-summed series at the
pulse's DM, peak taken within two samples of the injection time."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_1607_00909_amd import synth

pytestmark = pytest.mark.gpu

# relative S/N change allowed against the oracle's S/N
LOSS_BAR = {0: 1e-4, 1: 1e-3, 2: 1e-4}
NAMES = {0: "fp32", 1: "bf16x3", 2: "fp16x3"}


def snr(series: np.ndarray, t0: int) -> float:
    med = np.median(series)
    mad = np.median(np.abs(series - med))
    return float((series[t0 - 2:t0 + 3].max() - med) / (1.4826 * mad))


def test_pulse_snr_by_precision(hip_lib):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    w = dataclasses.replace(synth.LOFAR, nsub=8, nblock=6)
    cfg = oracle.Config(w.nsub, w.f_centre, w.bw, w.nfft, w.noverlap, w.nchan, w.ndec)
    pulses = synth.pulse_draws(w)
    print(f"[gpu-case] pulse S/N, pulses {pulses}", flush=True)
    x = synth.gaussian_voltages(w.nsub, w.ntime_in, w.sigma, w.seed)
    for dm, t0 in pulses:
        for s in range(w.nsub):
            oracle.inject_impulse(cfg, x, s, dm, oracle.pulse_sample(cfg, t0),
                                  w.pulse_amp_sigma * w.sigma)
    v, clipped = synth.encode_ci8(x)
    print(f"clipped components: {clipped}", flush=True)   # both sides see the same bytes
    dms = list(w.dms)
    pulse_idx = sorted({dms.index(dm) for dm, _ in pulses})
    ref = oracle.dedisperse(cfg, v, w.nblock, [dms[i] for i in pulse_idx])
    ref_snr = {dm: snr(ref[pulse_idx.index(dms.index(dm))].sum(axis=1), t0) for dm, t0 in pulses}

    dev = torch.from_numpy(v).cuda()
    for prec in (0, 1, 2):
        plan = hip_lib.Plan(w.nsub, w.f_centre, w.bw, w.nfft, w.noverlap, w.nchan, w.ndec,
                            input_kind=hip_lib.INPUT_CI8)
        hip_lib.cdmt_plan_set(plan.handle, hip_lib.CDMT_OPT_PRECISION, prec)
        out = plan.dedisperse(dev, w.nblock, dms)
        torch.cuda.synchronize()
        worst = 0.0
        for dm, t0 in pulses:
            series = out[dms.index(dm)].cpu().numpy().astype(np.float64).sum(axis=1)
            got = snr(series, t0)
            loss = 1.0 - got / ref_snr[dm]
            print(f"{NAMES[prec]}: DM {dm:5.1f} t0 {t0:5d} S/N {got:9.3f} "
                  f"(oracle {ref_snr[dm]:9.3f}), loss {loss:+.2e}", flush=True)
            worst = max(worst, abs(loss))
            # the pulse re-compresses into its own output sample
            assert int(np.argmax(series[t0 - 2:t0 + 3])) == 2
        assert worst <= LOSS_BAR[prec], (NAMES[prec], worst)
