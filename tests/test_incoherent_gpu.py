"""GPU incoherent stage (cdmt_incoherent) against the oracle's incoherent
dedispersion (Eq. 2 delays, channel sums).

Bars: with integer-valued filterbanks every FP32 sum is exact, so the GPU
must equal the oracle exactly, which pins every delay.  With real-valued
power the GPU sums nch float32 terms in order, so |gpu - exact| <=
gamma_(nch-1) * sum_ch |x| with gamma_n = n u / (1 - n u), u = 2^-24."""
import numpy as np
import pytest

import oracle
from oracle import incoherent
from paper_1607_00909_amd import synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _gamma(n):
    u = 2.0 ** -24
    return n * u / (1 - n * u)


def _run(hip_lib, cfg, nblock, fb, dms, ddm0, ddm, ntrial):
    torch = _torch()
    plan = hip_lib.Plan(cfg.nsub, cfg.f_centre, cfg.bw, cfg.nfft, cfg.noverlap, cfg.nchan,
                        cfg.ndec, chirp_ref=cfg.chirp_ref)
    out = hip_lib.incoherent(plan, torch.from_numpy(fb).cuda(), nblock, dms, ddm0, ddm, ntrial)
    torch.cuda.synchronize()
    return out.cpu().numpy()


CASES = {
    # name: (chirp reference, dms, ddm0, ddm, ntrial)
    "channel-fine": (oracle.CHANNEL, [0.5, 3.0, 7.0], -0.5, 0.01, 101),
    "subband-fine": (oracle.SUBBAND, [1.0, 6.0], -0.25, 0.005, 37),
    "one-trial-dm0": (oracle.CHANNEL, [0.5, 2.0], -0.5, 0.0, 1),
    "spread-over-64": (oracle.CHANNEL, [0.0, 1.0], 0.0, 0.5, 16),
    "coarse-global": (oracle.CHANNEL, [1.0, 2.0], 0.0, 2.0, 10),
    "odd-channels": (oracle.CHANNEL, [1.0, 4.0], -0.5, 0.05, 20),
}


@pytest.mark.parametrize("kind", ["codes", "power"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_incoherent_parity(hip_lib, name, kind):
    mode, dms, ddm0, ddm, ntrial = CASES[name]
    # 4 subbands at 140 MHz, 8 channels each, 163.84 us samples; 4 blocks of
    # 384 samples: several 256-sample tiles and a ragged tail
    cfg = oracle.Config(4, 140.0, synth.SUBBAND_MHZ, 16384, 4096, 8, 4, chirp_ref=mode)
    nblock = 4
    if name == "odd-channels":
        # 3 subbands of one channel each (an odd channel count), 81.92 us samples
        cfg = oracle.Config(3, 140.0, synth.SUBBAND_MHZ, 4096, 1024, 1, 16, chirp_ref=mode)
        nblock = 2
    ntime = nblock * cfg.tblk
    nch = cfg.nsub * cfg.nchan
    print(f"[gpu-case] incoherent {name} {kind}", flush=True)
    fb = synth.filterbank(len(dms), ntime, nch, 90 + len(name), kind)
    gpu = _run(hip_lib, cfg, nblock, fb, dms, ddm0, ddm, ntrial)
    ref = incoherent.dedisperse(cfg, fb, dms, ddm0, ddm, ntrial)
    assert gpu.shape == ref.shape
    if kind == "codes":
        assert np.array_equal(gpu.astype(np.float64), ref)
    else:
        bound = _gamma(nch - 1) * ref                # positive terms: sum |x| = the sum
        err = np.abs(gpu.astype(np.float64) - ref)
        print(f"{name}: max err / bound {np.max(err / bound):.3f}", flush=True)
        assert np.all(err <= bound)


def test_incoherent_recovers_a_dispersed_spike(hip_lib):
    """A spike dispersed at DM 3 (one sample per channel on the Eq. 2 sweep)
    adds up in every channel only at trials whose delays all match DM 3's."""
    cfg = oracle.Config(4, 140.0, synth.SUBBAND_MHZ, 16384, 4096, 8, 4)
    nblock = 2
    nch = cfg.nsub * cfg.nchan
    D = incoherent.delays(cfg, 3.0)
    fb = np.zeros((1, nblock * cfg.tblk, nch), np.float32)
    t0 = 300
    fb[0, t0 + D, np.arange(nch)] = 1.0
    gpu = _run(hip_lib, cfg, nblock, fb, [3.0], -0.5, 0.01, 101)
    D_all = np.stack([incoherent.delays(cfg, 2.5 + 0.01 * k) for k in range(101)])
    same = np.all(D_all == D, axis=1)
    assert same[50] and not np.all(same)
    assert np.all(gpu[0, same, t0] == nch)
    assert np.all(gpu[0, ~same, t0] < nch)


def test_incoherent_lofar_scale_samples(hip_lib):
    """At full size: 288 subbands x 16 channels, 39 blocks (15288 samples of
    655.36 us), coherent DMs 0.5..20 and 500 fine trials -0.5..+0.498 in
    steps of 0.002 around each; sampled outputs against the oracle's sums."""
    torch = _torch()
    w = synth.LOFAR
    cfg = oracle.Config(w.nsub, w.f_centre, w.bw, w.nfft, w.noverlap, w.nchan, w.ndec)
    plan = hip_lib.Plan(w.nsub, w.f_centre, w.bw, w.nfft, w.noverlap, w.nchan, w.ndec)
    dms = [0.5 * (i + 1) for i in range(40)]
    print("[gpu-case] incoherent lofar-scale", flush=True)
    _, ntout, nch = plan.shape(w.nblock)
    fb = synth.device_filterbank(len(dms), ntout, nch, 2024, "cuda")
    out = hip_lib.incoherent(plan, fb, w.nblock, dms, -0.5, 0.002, 500)
    torch.cuda.synchronize()
    nout = out.shape[2]
    assert nout == ntout - int(incoherent.delays(cfg, 20.0 + (-0.5 + 0.002 * 499)).max())
    r = np.random.default_rng(5)
    worst = 0.0
    for d in (0, 17, 39):
        fb_d = fb[d].cpu().numpy()
        ks = list(r.integers(0, 500, 6)) + [0, 499]
        for k in ks:
            ts = list(r.integers(0, nout, 5)) + [0, nout - 1]
            dm = dms[d] + (-0.5 + 0.002 * int(k))
            ref = incoherent.sample(cfg, fb_d, dm, ts)
            got = out[d, int(k), ts].cpu().numpy().astype(np.float64)
            err = np.abs(got - ref) / (_gamma(nch - 1) * ref)
            worst = max(worst, float(err.max()))
    print(f"lofar-scale: max err / bound {worst:.3f}", flush=True)
    assert worst <= 1.0


@pytest.mark.parametrize("kind", ["codes", "power"])
def test_incoherent_edges(hip_lib, kind):
    """A largest delay that leaves exactly one output sample, and more than
    256 coherent DMs (the delay table in several launches)."""
    cfg = oracle.Config(4, 140.0, synth.SUBBAND_MHZ, 16384, 4096, 8, 4)
    nblock = 2
    nch = cfg.nsub * cfg.nchan
    ntime = nblock * cfg.tblk
    print(f"[gpu-case] incoherent edges {kind}", flush=True)
    # DM 54.87: the lowest channel's delay is 767 of 768 samples
    for dms, ddm0, ddm, ntrial in (([54.87], 0.0, 0.0, 1), ([54.0], 0.0, 0.87 / 2, 3),
                                   ([0.05 * i for i in range(300)], 0.0, 0.01, 2)):
        fb = synth.filterbank(len(dms), ntime, nch, 7 + ntrial, kind)
        ref = incoherent.dedisperse(cfg, fb, dms, ddm0, ddm, ntrial)
        gpu = _run(hip_lib, cfg, nblock, fb, dms, ddm0, ddm, ntrial)
        assert gpu.shape == ref.shape
        if kind == "codes":
            assert np.array_equal(gpu.astype(np.float64), ref)
        else:
            assert np.all(np.abs(gpu.astype(np.float64) - ref) <= _gamma(nch - 1) * ref)
    assert ref.shape[0] == 300


def test_semi_coherent_search_finds_the_pulse(hip_lib):
    """The whole semi-coherent search on the GPU (coherent stage at DMs 10.0
    and 10.5, then 251 fine trials +-0.25 around each) finds a pulse dispersed
    at DM 10.37 across the band: the same (coherent DM, fine trial, sample) as
    the oracle's chain, within 0.02 of the true DM at the injected sample,
    with about twice the peak of the coarse trials alone."""
    torch = _torch()
    print("[gpu-case] semi-coherent search", flush=True)
    nsub, fc, nfft, nov, nchan, ndec, nblock = 4, 140.0, 16384, 4096, 8, 4, 4
    cfg = oracle.Config(nsub, fc, synth.SUBBAND_MHZ, nfft, nov, nchan, ndec)
    # dispersed within each subband (inverse transfer function with nu0 at the
    # subband centre) and delayed between subbands by Eq. 2, so that every
    # channel's centre arrives at its delay behind the top channel's
    inj = oracle.Config(nsub, fc, synth.SUBBAND_MHZ, nfft, nov, nchan, ndec,
                        chirp_ref=oracle.SUBBAND)
    x = synth.gaussian_voltages(nsub, cfg.ntime_in(nblock), 1.0, 41)
    dm_true, t0 = 10.37, 600
    top = incoherent.channel_frequencies(cfg).max()
    for s in range(nsub):
        fs = cfg.sub_centre(s)
        lag = oracle.sweep_seconds(fs, top, dm_true) * cfg.bw * 1e6     # subband samples
        oracle.inject_impulse(inj, x, s, dm_true, oracle.pulse_sample(cfg, t0) + int(round(lag)),
                              40.0)
    v = synth.encode_cf32(x)
    coarse = [10.0, 10.5]
    ddm0, ddm, ntrial = -0.25, 0.002, 251
    plan = hip_lib.Plan(nsub, fc, synth.SUBBAND_MHZ, nfft, nov, nchan, ndec)
    fb = plan.dedisperse(torch.from_numpy(v).cuda(), nblock, coarse)
    gpu = hip_lib.incoherent(plan, fb, nblock, coarse, ddm0, ddm, ntrial)
    torch.cuda.synchronize()
    gpu = gpu.cpu().numpy()
    ref = incoherent.dedisperse(cfg, oracle.dedisperse(cfg, v, nblock, coarse), coarse, ddm0, ddm,
                                ntrial)
    at = np.unravel_index(np.argmax(gpu), gpu.shape)
    assert at == np.unravel_index(np.argmax(ref), ref.shape)
    d, k, t = (int(i) for i in at)
    dm = coarse[d] + (ddm0 + ddm * k)
    k0 = round(-ddm0 / ddm)                                      # fine offset 0
    print(f"found DM {dm:.3f} at sample {t} (true {dm_true}, {t0}); peak {gpu[at]:.1f}, "
          f"coarse-only peaks {gpu[0, k0].max():.1f} {gpu[1, k0].max():.1f}", flush=True)
    assert t == t0 and abs(dm - dm_true) <= 0.02
    assert gpu[at] > 1.5 * max(gpu[0, k0].max(), gpu[1, k0].max())
    assert np.all(np.abs(gpu - ref) <= 1e-5 * np.abs(ref).max())


def test_incoherent_reads_channel_major_filterbanks(hip_lib):
    """A plan with CDMT_OPT_OUT_LAYOUT = 1 has the coherent stage write
    [DM][channel][time], which the incoherent stage reads without its
    transpose: the same sums, bit for bit."""
    torch = _torch()
    cfg = oracle.Config(4, 140.0, synth.SUBBAND_MHZ, 16384, 4096, 8, 4)
    nblock = 3
    print("[gpu-case] incoherent channel-major", flush=True)
    v = torch.from_numpy(synth.encode_cf32(synth.gaussian_voltages(
        cfg.nsub, cfg.ntime_in(nblock), 1.0, 51))).cuda()
    coarse = [1.0, 2.0, 3.0]
    res = []
    for layout in (0, 1):
        plan = hip_lib.Plan(cfg.nsub, cfg.f_centre, cfg.bw, cfg.nfft, cfg.noverlap, cfg.nchan,
                            cfg.ndec, out_layout=layout)
        fb = plan.dedisperse(v, nblock, coarse)
        res.append(hip_lib.incoherent(plan, fb, nblock, coarse, -0.5, 0.01, 101))
    torch.cuda.synchronize()
    assert torch.equal(res[0], res[1])
