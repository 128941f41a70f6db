"""Parity at the full LOFAR-shaped size, in the launch configuration the
benchmark times: 288 subbands (109.875-166.125 MHz), 39 blocks of nfft 65536
with noverlap 15360, 16 channels, x8 downsampling, 128 DMs 0..63.5, ci8 noise
(sigma 16) generated in device memory exactly as the benchmark does.

The oracle recomputes sampled (subband, block) pairs with every DM; every
other output sample is checked by properties that hold at any size: the
output (pre-filled with NaN) is completely written, finite and
non-negative, the DM-tile-1 launch split (several launches to keep each
grid under 2^32 work-items) gives bitwise the same filterbank, and the
channel-major output layout is bitwise its transpose.  The split-precision
(FP16x3, BF16x3) DM stages are checked on the same sampled pairs, to the
bars their own parity tests state."""
import numpy as np
import pytest

import oracle
from paper_1607_00909_amd import synth

pytestmark = pytest.mark.gpu

PAIRS = [(0, 0), (1, 1), (143, 19), (287, 38), (200, 7), (77, 30)]


def _check_pairs(out, w, label, bar=1e-5, bar_max=1e-5):
    cols_of = lambda s: [(w.nsub - 1 - s) * w.nchan + (w.nchan - 1 - c) for c in range(w.nchan)]
    for s, b in PAIRS:
        xs = _HOST[s]
        cfg = oracle.Config(1, w.f_centre + (s - (w.nsub - 1) / 2) * w.bw, w.bw, w.nfft,
                            w.noverlap, w.nchan, w.ndec)
        key = (s, b)
        if key not in _REF:
            _REF[key] = oracle.subband_block(cfg, xs, 0, b, list(w.dms))   # [dm][t][c]
        ref = _REF[key]
        gpu = out[:, b * w.tblk:(b + 1) * w.tblk, cols_of(s)].double().cpu().numpy()
        d = gpu - ref
        e = np.sqrt((d ** 2).sum((1, 2)) / (ref ** 2).sum((1, 2))).max()
        emax = np.abs(d).max() / np.abs(ref).max()
        print(f"{label} pair s={s} b={b}: max_d normwise {e:.3e}, max-abs/max {emax:.3e}",
              flush=True)
        assert e <= bar and emax <= bar_max, (label, s, b, e, emax)


_HOST, _REF = {}, {}


def test_lofar_full_size_sampled_parity(hip_lib):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    w = synth.LOFAR
    print(f"[gpu-case] LOFAR full size {w.nsub}x{w.ntime_in}, {len(w.dms)} DMs", flush=True)
    dev = torch.device("cuda:0")
    x = synth.device_noise("ci8", w.nsub, w.ntime_in, w.sigma, w.seed, dev)
    for s, _ in PAIRS:
        _HOST[s] = x[s].cpu().numpy()[None]

    def run(precision=0, **kw):
        plan = hip_lib.Plan(w.nsub, w.f_centre, w.bw, w.nfft, w.noverlap, w.nchan, w.ndec,
                            input_kind=hip_lib.INPUT_CI8, **kw)
        if precision:
            hip_lib.cdmt_plan_set(plan.handle, hip_lib.CDMT_OPT_PRECISION, precision)
        out = torch.full(plan.out_shape(len(w.dms), w.nblock), float("nan"), device=dev)
        plan.dedisperse(x, w.nblock, list(w.dms), out=out, workspace=ws)
        torch.cuda.synchronize()
        return out

    ws = hip_lib.Plan(w.nsub, w.f_centre, w.bw, w.nfft, w.noverlap, w.nchan, w.ndec,
                      input_kind=hip_lib.INPUT_CI8).workspace(w.nblock, dev)
    # the benchmark's configuration: default DM tile, recurrence over the tile
    out_a = run()
    assert bool(torch.isfinite(out_a).all()), "some output samples were never written"
    assert float(out_a.min()) >= 0.0
    _check_pairs(out_a, w, "default")

    # transfer function evaluated per DM
    out_b = run(chirp_exact=1)
    assert bool(torch.isfinite(out_b).all())
    _check_pairs(out_b, w, "exact")
    # the two modes agree over the whole output, DM by DM
    rel = 0.0
    for d in range(out_a.shape[0]):
        a, b = out_a[d].double(), out_b[d].double()
        rel = max(rel, float(((a - b) ** 2).sum().sqrt() / (b ** 2).sum().sqrt()))
        del a, b
    print(f"recurrence vs exact, whole output: max_d normwise {rel:.3e}", flush=True)
    assert rel <= 1e-5
    del out_a

    # DM tile 1: 128 DM tiles x 179712 chunks needs two launches
    out_c = run(dm_tile=1, chirp_exact=1)
    assert bool(torch.equal(out_c, out_b))
    del out_c
    # the channel-major layout: the same filterbank, transposed, bit for bit
    out_c = run(chirp_exact=1, out_layout=1)
    assert bool(torch.isfinite(out_c).all())
    assert bool(torch.equal(out_c.transpose(1, 2), out_b))
    del out_c
    # the split-precision DM stages at full size (FP16x3 held to the FP32 bar;
    # BF16x3 to the bars derived from its split error in
    # test_parity_mixed_gpu: 5e-5 normwise, 2.7e-4 max-abs/max)
    for prec, label, bars in ((2, "fp16x3", (1e-5, 1e-5)), (1, "bf16x3", (5e-5, 2.7e-4))):
        out_c = run(precision=prec)
        assert bool(torch.isfinite(out_c).all())
        _check_pairs(out_c, w, label, *bars)
        del out_c

    # redigitisation of the full filterbank, sampled (DM, channel) series
    # against the oracle's statistics; the bytes follow from the parameters
    from oracle import redigit
    codes, mean, scale = hip_lib.redigitise(out_b, 64.0, 16.0)
    torch.cuda.synchronize()
    worst = 0
    for d, ch in [(0, 0), (5, 4607), (64, 1234), (127, 2048), (100, 17), (33, 3333)]:
        series = out_b[d, :, ch].cpu().numpy()[None, :, None]
        m_ref, k_ref = redigit.parameters(series, 16.0)
        m, k = mean[d, ch].item(), scale[d, ch].item()
        um = abs(int(np.float32(m).view(np.int32)) - int(m_ref[0, 0].view(np.int32)))
        uk = abs(int(np.float32(k).view(np.int32)) - int(k_ref[0, 0].view(np.int32)))
        worst = max(worst, um, uk)
        got = codes[d, :, ch].cpu().numpy()
        want = redigit.quantise(series, np.array([[m]], np.float32), np.array([[k]], np.float32),
                                64.0)[0, :, 0]
        assert np.array_equal(got, want), (d, ch)
    print(f"redigitise LOFAR: sampled parameters within {worst} ulp", flush=True)
    assert worst <= 1
