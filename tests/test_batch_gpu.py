"""Batches of beams (several plans, inputs, DM lists and outputs in one
persistent launch per M_bin) through the C ABI.

The batched DM stage runs the same per-item arithmetic as the single-beam
kernel, so each beam's output must be bitwise equal to cdmt_dedisperse of that
beam with the same DM tile.  Each beam is also checked against the FP64
oracle on one (subband, block) pair, and the graph form must reproduce the
eager run on every replay, with other work in between."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_1607_00909_amd import synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@dataclasses.dataclass
class BeamSpec:
    nsub: int
    f_centre: float
    nfft: int
    noverlap: int
    nchan: int
    ndec: int
    nblock: int
    dms: list
    kind: str
    chirp_ref: int = oracle.CHANNEL


# uneven subband counts, N_bin, channel counts (M_bin 4096, 4096, 2048, 1024,
# 512), DM counts (ragged tiles, more than 256) and DM ranges; one non-arithmetic
# DM list (exact transfer function, its own launch); both nu0 modes
SPECS = [
    BeamSpec(3, 150.0, 65536, 8192, 16, 8, 2, list(np.arange(0.0, 40.0, 0.5)), "ci8"),
    BeamSpec(2, 120.0, 16384, 4096, 4, 4, 3, list(np.arange(0.0, 7.0, 1.0)), "cf32",
             oracle.SUBBAND),
    BeamSpec(4, 135.0, 32768, 4096, 16, 4, 2, list(np.arange(10.0, 10.0 + 0.25 * 300, 0.25)),
             "ci8"),
    BeamSpec(1, 170.0, 16384, 2048, 16, 2, 2, [0.0, 3.0, 4.5, 11.0, 30.0], "ci8"),
    BeamSpec(2, 110.0, 131072, 16384, 256, 4, 1, list(np.arange(0.0, 200.0, 12.5)), "cf32"),
]


def _inputs(spec, seed):
    cfg = oracle.Config(spec.nsub, spec.f_centre, synth.SUBBAND_MHZ, spec.nfft, spec.noverlap,
                        spec.nchan, spec.ndec, chirp_ref=spec.chirp_ref)
    x = synth.gaussian_voltages(spec.nsub, cfg.ntime_in(spec.nblock), 16.0 if spec.kind == "ci8"
                                else 1.0, seed)
    v = synth.encode_ci8(x)[0] if spec.kind == "ci8" else synth.encode_cf32(x)
    return cfg, v


def _plan(hip_lib, spec, dm_tile=None, fwd_n2=None, fft_schedule=None, lane_bins=None):
    return hip_lib.Plan(spec.nsub, spec.f_centre, synth.SUBBAND_MHZ, spec.nfft, spec.noverlap,
                        spec.nchan, spec.ndec,
                        input_kind=hip_lib.INPUT_CI8 if spec.kind == "ci8" else hip_lib.INPUT_CF32,
                        chirp_ref=spec.chirp_ref, dm_tile=dm_tile, fwd_n2=fwd_n2,
                        fft_schedule=fft_schedule, lane_bins=lane_bins)


def _setup(hip_lib, torch, specs):
    beams, host = [], []
    for i, sp in enumerate(specs):
        cfg, v = _inputs(sp, 300 + i)
        plan = _plan(hip_lib, sp)
        _, ntout, nch = plan.shape(sp.nblock)
        x = torch.from_numpy(v).cuda()
        out = torch.full((len(sp.dms), ntout, nch), float("nan"), device="cuda")
        beams.append((plan, sp.nblock, x, sp.dms, out))
        host.append((cfg, v))
    return beams, host


def _single(hip_lib, sp, x, dm_tile, fwd_n2=None, fft_schedule=None, lane_bins=None):
    plan = _plan(hip_lib, sp, dm_tile, fwd_n2, fft_schedule, lane_bins)
    return plan.dedisperse(x, sp.nblock, sp.dms)


def test_batch_matches_single_beams_and_oracle(hip_lib):
    torch = _torch()
    print("[gpu-case] batch of 5 beams, eager", flush=True)
    beams, host = _setup(hip_lib, torch, SPECS)
    batch = hip_lib.Batch(beams)
    # M 4096 with the recurrence, ndec 8 and ndec 4 (the lane-swap item is
    # built per downsampling factor); M 2048 and 512 with the recurrence;
    # M 1024 exact
    assert batch.get(hip_lib.CDMT_BATCH_LAUNCHES) == 5
    batch.run()
    torch.cuda.synchronize()
    for i, (sp, (plan, nblock, x, dms, out)) in enumerate(zip(SPECS, beams)):
        assert bool(torch.isfinite(out).all()), f"beam {i}: output not fully written"
        ref = _single(hip_lib, sp, x, hip_lib.cdmt_plan_get(plan.handle, hip_lib.CDMT_OPT_DM_TILE))
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"beam {i} differs from its single-beam run"
        _, v = host[i]
        s, b = sp.nsub - 1, sp.nblock - 1
        cfg1 = oracle.Config(1, sp.f_centre + (s - (sp.nsub - 1) / 2) * synth.SUBBAND_MHZ,
                             synth.SUBBAND_MHZ, sp.nfft, sp.noverlap, sp.nchan, sp.ndec,
                             chirp_ref=sp.chirp_ref)
        want = oracle.subband_block(cfg1, v[s:s + 1], 0, b, sp.dms)
        cols = [(sp.nsub - 1 - s) * sp.nchan + (sp.nchan - 1 - c) for c in range(sp.nchan)]
        tb = plan.shape(1)[1]
        got = out[:, b * tb:(b + 1) * tb, cols].double().cpu().numpy()
        d = got - want
        e = float(np.sqrt((d ** 2).sum((1, 2)) / (want ** 2).sum((1, 2))).max())
        print(f"beam {i}: M {sp.nfft // sp.nchan}, {len(sp.dms)} DMs, vs oracle {e:.2e}",
              flush=True)
        assert e <= 1e-5


def test_batch_with_a_channel_major_beam(hip_lib):
    """Beams keep their plan's filterbank layout in a batch: a channel-major
    beam equals its single-beam run, and the time-major one too."""
    torch = _torch()
    print("[gpu-case] batch with a channel-major beam", flush=True)
    specs = SPECS[:2]
    beams = []
    for i, sp in enumerate(specs):
        cfg, v = _inputs(sp, 400 + i)
        plan = hip_lib.Plan(sp.nsub, sp.f_centre, synth.SUBBAND_MHZ, sp.nfft, sp.noverlap,
                            sp.nchan, sp.ndec,
                            input_kind=hip_lib.INPUT_CI8 if sp.kind == "ci8" else hip_lib.INPUT_CF32,
                            chirp_ref=sp.chirp_ref, out_layout=1 - i)
        out = torch.full(plan.out_shape(len(sp.dms), sp.nblock), float("nan"), device="cuda")
        beams.append((plan, sp.nblock, torch.from_numpy(v).cuda(), sp.dms, out))
    batch = hip_lib.Batch(beams)
    batch.run()
    torch.cuda.synchronize()
    for plan, nblock, x, dms, out in beams:
        ref = plan.dedisperse(x, nblock, dms)
        torch.cuda.synchronize()
        assert torch.equal(out, ref)


def test_batch_graph_replays_and_autotune(hip_lib):
    torch = _torch()
    print("[gpu-case] batch graph + autotune", flush=True)
    specs = SPECS[:3]
    beams, _ = _setup(hip_lib, torch, specs)
    batch = hip_lib.Batch(beams)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        batch.run(stream)
    stream.synchronize()
    eager = [b[4].clone() for b in beams]
    for rep in range(3):
        for b in beams:
            b[4].fill_(-1.0)                      # eager work between replays
        torch.cuda.synchronize()
        batch.run_graph(stream)
        stream.synchronize()
        for i, b in enumerate(beams):
            assert torch.equal(b[4], eager[i]), f"replay {rep}, beam {i}"
    # a per-beam forward split (the other radix schedule of beam 0's N_bin 65536)
    FN2 = hip_lib.CDMT_BATCH_BEAM_FWD_N2
    assert batch.beam_get(0, FN2) == 256
    batch.beam_set(0, FN2, 128)
    assert batch.beam_get(0, FN2) == 128
    batch.run_graph(stream)                       # captured again
    stream.synchronize()
    ref = _single(hip_lib, specs[0], beams[0][2], None, 128)
    torch.cuda.synchronize()
    assert torch.equal(beams[0][4], ref), "beam 0 with the 512 x 128 forward split"
    with pytest.raises(hip_lib.CdmtError):
        batch.beam_set(1, FN2, 512)               # not a split of 16384
    # a per-beam DM-stage schedule: beam 0 (M_bin 4096, ndec 8) on the
    # radix-16 Stockham stages instead of the three-pass transform
    FS = hip_lib.CDMT_BATCH_BEAM_FFT_SCHEDULE
    assert batch.beam_get(0, FS) == 0
    nl = batch.get(hip_lib.CDMT_BATCH_LAUNCHES)
    batch.beam_set(0, FS, 1)
    assert batch.beam_get(0, FS) == 1
    # beam 0 leaves the three-pass group (M_bin 4096, ndec 8) for a Stockham
    # group of its own at M_bin 4096: the launch count stays the same
    assert batch.get(hip_lib.CDMT_BATCH_LAUNCHES) == nl == 3
    batch.run_graph(stream)
    stream.synchronize()
    ref = _single(hip_lib, specs[0], beams[0][2], None, 128, 1)
    torch.cuda.synchronize()
    assert torch.equal(beams[0][4], ref), "beam 0 on the Stockham schedule"
    with pytest.raises(hip_lib.CdmtError):
        batch.beam_set(0, FS, 2)
    batch.beam_set(0, FS, -1)
    # 8 bins per lane for beam 2 (M_bin 2048, radix-8 Stockham stages)
    LB = hip_lib.CDMT_BATCH_BEAM_LANE_BINS
    assert batch.beam_get(2, LB) == 16
    batch.beam_set(2, LB, 8)
    batch.run_graph(stream)
    stream.synchronize()
    ref = _single(hip_lib, specs[2], beams[2][2], None, None, None, 8)
    torch.cuda.synchronize()
    assert torch.equal(beams[2][4], ref), "beam 2 with 8 bins per lane"
    with pytest.raises(hip_lib.CdmtError):
        batch.beam_set(2, LB, 4)
    batch.beam_set(2, LB, 0)
    best = batch.autotune(stream, reps=1)
    stream.synchronize()
    tile = batch.get(hip_lib.CDMT_BATCH_DM_TILE)
    wg = batch.get(hip_lib.CDMT_BATCH_WG_PER_CU)
    splits = [batch.beam_get(i, FN2) for i in range(len(specs))]
    scheds = [batch.beam_get(i, FS) for i in range(len(specs))]
    bins = [batch.beam_get(i, LB) for i in range(len(specs))]
    print(f"autotune: forward N2 {splits}, DM-stage schedules {scheds}, bins per lane {bins}, "
          f"dm tile {tile}, {wg} workgroups per CU, {best:.3f} ms", flush=True)
    assert best > 0 and tile in (4, 8, 16) and wg in (2, 4)
    # after tuning (graph captured again) each beam equals its single run with
    # the chosen split and tile
    batch.run_graph(stream)
    stream.synchronize()
    for i, (sp, b) in enumerate(zip(specs, beams)):
        ref = _single(hip_lib, sp, b[2], tile, splits[i], scheds[i], bins[i])
        torch.cuda.synchronize()
        assert torch.equal(b[4], ref), f"beam {i} after autotune"


def test_batch_24_beam_workload(hip_lib):
    """The benchmark's batched workload at full size (24 beams, M_bin 1024,
    2048 and 4096, 55 GB of filterbanks), in the benchmark's launch form
    (autotuned, graph replay): every output written and finite, one
    (subband, block) pair per beam against the oracle, and one beam of each
    M_bin bitwise equal to its single-beam run with the tuned settings."""
    torch = _torch()
    import math
    from concurrent.futures import ThreadPoolExecutor
    draws = synth.batch_draws()
    print(f"[gpu-case] batch workload, {len(draws)} beams", flush=True)
    beams, cfgs = [], []
    for i, d in enumerate(draws):
        # overlap from the oracle's Eq. 2 sweep over the lowest channel, rounded
        # up to a multiple of 2 n_c ndec (as the plan helper does)
        chan = synth.SUBBAND_MHZ / d.nchan
        td = oracle.sweep_seconds(d.f_lo, d.f_lo + chan, d.dm_max)
        q = 2 * d.nchan * d.ndec
        nov = int(math.ceil(td * synth.SUBBAND_MHZ * 1e6 / q)) * q
        assert nov == hip_lib.cdmt_noverlap_for(d.f_lo, synth.SUBBAND_MHZ, d.dm_max, d.nchan,
                                                d.ndec, hip_lib.CHIRP_CHANNEL)
        nblock = math.ceil(synth.SUBBAND_MHZ * 1e6 / (d.nfft - nov))
        plan = hip_lib.Plan(d.nsub, d.f_centre, synth.SUBBAND_MHZ, d.nfft, nov, d.nchan, d.ndec,
                            input_kind=hip_lib.INPUT_CI8)
        ntin, ntout, nch = plan.shape(nblock)
        x = synth.device_noise("ci8", d.nsub, ntin, 16.0, 1607 + i, "cuda")
        out = torch.full((d.ndm, ntout, nch), float("nan"), device="cuda")
        beams.append((plan, nblock, x, list(d.dms), out))
        cfgs.append((d, nov, nblock))
    batch = hip_lib.Batch(beams)
    # one persistent launch per M_bin present (every beam here takes the
    # transfer-function recurrence and ndec 8)
    assert batch.get(hip_lib.CDMT_BATCH_LAUNCHES) == len({d.nfft // d.nchan for d in draws}) > 1
    stream = torch.cuda.Stream()
    batch.autotune(stream, reps=1)
    batch.run_graph(stream)
    stream.synchronize()
    for i, b in enumerate(beams):
        assert bool(torch.isfinite(b[4]).all()), f"beam {i} not fully written"

    def check(i):
        d, nov, nblock = cfgs[i]
        s, blk = (7 * i) % d.nsub, (3 * i) % nblock
        xs = beams[i][2][s].cpu().numpy()[None]
        c1 = oracle.Config(1, d.f_centre + (s - (d.nsub - 1) / 2) * synth.SUBBAND_MHZ,
                           synth.SUBBAND_MHZ, d.nfft, nov, d.nchan, d.ndec)
        want = oracle.subband_block(c1, xs, 0, blk, list(d.dms))
        tb = want.shape[1]
        cols = [(d.nsub - 1 - s) * d.nchan + (d.nchan - 1 - c) for c in range(d.nchan)]
        got = beams[i][4][:, blk * tb:(blk + 1) * tb, cols].double().cpu().numpy()
        dd = got - want
        return float(np.sqrt((dd ** 2).sum((1, 2)) / (want ** 2).sum((1, 2))).max())

    with ThreadPoolExecutor(max_workers=16) as ex:
        errs = list(ex.map(check, range(len(beams))))
    print(f"batch workload vs oracle: worst beam {max(errs):.2e}", flush=True)
    assert max(errs) <= 1e-5
    tile = batch.get(hip_lib.CDMT_BATCH_DM_TILE)
    for i in sorted({d.nfft // d.nchan: i for i, d in enumerate(draws)}.values()):
        d, nov, nblock = cfgs[i]
        plan = hip_lib.Plan(d.nsub, d.f_centre, synth.SUBBAND_MHZ, d.nfft, nov, d.nchan, d.ndec,
                            input_kind=hip_lib.INPUT_CI8, dm_tile=tile,
                            fwd_n2=batch.beam_get(i, hip_lib.CDMT_BATCH_BEAM_FWD_N2),
                            fft_schedule=batch.beam_get(i, hip_lib.CDMT_BATCH_BEAM_FFT_SCHEDULE),
                            lane_bins=batch.beam_get(i, hip_lib.CDMT_BATCH_BEAM_LANE_BINS))
        ref = plan.dedisperse(beams[i][2], nblock, list(d.dms))
        torch.cuda.synchronize()
        assert torch.equal(ref, beams[i][4]), f"beam {i} differs from its single-beam run"
        del ref


def test_batch_with_every_launch_group_of_the_three_pass_item(hip_lib):
    """A batch whose beams fall into more launch groups than there were
    before the three-pass item ran at M_bin 2048 and 1024 (M_bin 1024, 2048
    and 4096 x ndec 1, 2, 4, 8 x recurrence / exact transfer function, plus
    four Stockham groups: 28 groups, more than the 26 sets of work counters
    the batch workspace held then): each group has its own counters, and
    every beam equals its single-beam run."""
    torch = _torch()
    print("[gpu-case] batch of 28 launch groups", flush=True)
    specs = []
    for nchan in (16, 8, 4):                         # M_bin 1024, 2048, 4096 at nfft 16384
        for ndec in (1, 2, 4, 8):
            specs.append(BeamSpec(1, 140.0, 16384, 4096, nchan, ndec, 1, [0.0, 0.5, 1.0], "cf32"))
            specs.append(BeamSpec(1, 140.0, 16384, 4096, nchan, ndec, 1, [0.0, 0.7, 1.1], "cf32"))
    for nchan in (32, 64):                           # M_bin 512, 256 (Stockham stages)
        specs.append(BeamSpec(1, 140.0, 16384, 4096, nchan, 2, 1, [0.0, 0.5, 1.0], "cf32"))
        specs.append(BeamSpec(1, 140.0, 16384, 4096, nchan, 2, 1, [0.0, 0.7, 1.1], "cf32"))
    beams, _ = _setup(hip_lib, torch, specs)
    batch = hip_lib.Batch(beams)
    assert batch.get(hip_lib.CDMT_BATCH_LAUNCHES) == 28
    batch.run()
    torch.cuda.synchronize()
    for i, (sp, (plan, nblock, x, dms, out)) in enumerate(zip(specs, beams)):
        assert bool(torch.isfinite(out).all()), f"beam {i}: output not fully written"
        ref = _single(hip_lib, sp, x, hip_lib.cdmt_plan_get(plan.handle, hip_lib.CDMT_OPT_DM_TILE))
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"beam {i} differs from its single-beam run"
