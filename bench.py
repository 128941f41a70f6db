#!/usr/bin/env python
"""Throughput of coherent dedispersion to many DM trials on one MI355X.

Workload (default): LOFAR-HBA-shaped, 288 subbands of 195.3125 kHz centred
on 138 MHz, 10.02 s of dual-polarisation complex int8 voltages (Gaussian,
sigma 16, generated in device memory from a fixed seed), nfft 65536 with
noverlap 15360, 16 channels per subband, x8 downsampling, 128 DM trials
0..63.5.  One step = the whole path for that batch: the forward FFT of every
block and subband, then every DM trial (transfer function, backward FFT,
detection, downsampling, transpose) into an FP32 filterbank
[128][15288][4608] that stays in device memory.

Metric: DM trials x seconds of data processed per second of wall time.
Prints one JSON line.  --gpus above 1 is refused: the library runs on one GPU.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "DM-trials×data-sec per sec (LOFAR-shaped), %HBM peak; mixed vs FP32 plain"
HBM_PEAK_GBS = 8000.0
# FP32 vector peak: 256 CUs x 128 FP32 lanes per clock x 2 flop (FMA) x
# 2.4 GHz = 157.3 TFLOP/s.  A SIMD retires a wave64 FP32 instruction every
# two clocks (one wave alone issues at most one every ~5), so the rate holds
# for the plain (non-packed) instructions this library emits.
VALU_FP32_PEAK_TFLOPS = 256 * 128 * 2 * 2.4e9 / 1e12


PROFILE = os.path.join(ROOT, "profiles", "fused_dedisperse_lofar_hba_288sub_128dm.md")
PROFILE_INC = os.path.join(ROOT, "profiles", "inc_sum_lofar_hba_40dm_500trials.md")
# dense FP16 / BF16 matrix-core peak of the MI355X (no sparsity)
MFMA_F16_PEAK_TFLOPS = 2500.0


def measured_traffic(kernel: str, profile: str = PROFILE,
                     sources=("cdmt.hip", "fft_core.hpp", "plan.hpp")):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when the kernel sources changed since it was taken."""
    import hashlib
    import re
    try:
        text = open(profile).read()
        blob = json.loads(re.search(r"```json\n(.*?)\n```", text, re.S).group(1))
    except (OSError, AttributeError, ValueError):
        return None
    src = b"".join(open(os.path.join(ROOT, "paper_1607_00909_amd", "csrc", f), "rb").read()
                   for f in sources)
    if hashlib.sha256(src).hexdigest()[:16] != blob.get("source_sha256_16"):
        return None
    t = blob["traffic"].get(kernel)
    return None if t is None else (t["fetch_GB"] + t["write_GB"]) * 1e9


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def mx_mfma_flops_per_chunk_dm() -> float:
    """Matrix-core flops issued by the split-precision DM stage per channel
    chunk of 4096 bins and DM: 3 radix-16 stages x 16 column tiles (256
    butterflies x 2 pols / 32) x 6 products of 32x32x16 (hi.hi, hi.lo, lo.hi
    for the real- and imaginary-input halves), 2 flops per product term."""
    return 3 * 16 * 6 * (2 * 32 * 32 * 16)


def dm_stage_kernel(w, recurrence: bool) -> str:
    """Name of the FP32 DM-stage kernel the library launches for workload w
    (default schedule, 16 bins per lane): the three-pass kernel at M_bin 4096,
    2048 or 1024 when ndec = 2^K (K <= 3) divides n_d / 2, else the radix-16
    Stockham kernel."""
    import math
    nd_half = w.noverlap // w.nchan // 2
    k = int(math.log2(w.ndec)) if w.ndec & (w.ndec - 1) == 0 else -1
    r = "true" if recurrence else "false"
    if w.m in (1024, 2048, 4096) and 0 <= k <= 3 and nd_half % w.ndec == 0:
        return f"fused_dedisperse_x3<{r}, {k}, {w.m}>"
    return f"fused_dedisperse<{w.m}, 16, {r}>"


def fused_flops_per_bin(m: int) -> float:
    """Nominal flops per spectral bin per DM of the fused kernel: for both
    polarisations, complex multiply (6), backward FFT (5 log2 M per point),
    detection (3)."""
    import math
    return 2 * (6 + 5 * math.log2(m) + 3)


def cpu_baseline(w, x_dev, npairs: int, threads: int, outputs=None, pulses=()):
    """Oracle (FP64, C) on a bounded sample of (subband, block) pairs with all
    DMs, extrapolated linearly to the whole job; the sample includes the
    block of every injected pulse (at a spread of subbands), and the GPU
    outputs are compared with the oracle on every pair."""
    import numpy as np

    import oracle
    from concurrent.futures import ThreadPoolExecutor

    cfg = oracle.Config(w.nsub, w.f_centre, w.bw, w.nfft, w.noverlap, w.nchan, w.ndec)
    pairs = []
    for i, (_, t0) in enumerate(pulses):
        pairs.append(((i * 61 + 11) % w.nsub, t0 // w.tblk))
    i = 0
    while len(pairs) < npairs:
        sb = ((i * 97) % w.nsub, (i * 7) % w.nblock)
        if sb not in pairs:
            pairs.append(sb)
        i += 1
    subs = sorted({s for s, _ in pairs})
    host = {s: x_dev[s].cpu().numpy() for s in subs}

    def one(sb):
        s, b = sb
        xs = host[s][None]
        c1 = oracle.Config(1, cfg.sub_centre(s), w.bw, w.nfft, w.noverlap, w.nchan, w.ndec)
        return oracle.subband_block(c1, xs, 0, b, list(w.dms))

    oracle._load()
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        refs = list(ex.map(one, pairs))
    dt = time.perf_counter() - t0
    errors = {}
    for name, out in (outputs or {}).items():
        worst_n = worst_m = 0.0
        for (s, b), ref in zip(pairs, refs):
            cols = [(w.nsub - 1 - s) * w.nchan + (w.nchan - 1 - c) for c in range(w.nchan)]
            gpu = out[:, b * w.tblk:(b + 1) * w.tblk, cols].double().cpu().numpy()
            d = gpu - ref
            worst_n = max(worst_n, float(np.sqrt((d ** 2).sum((1, 2)) / (ref ** 2).sum((1, 2))).max()))
            worst_m = max(worst_m, float(np.abs(d).max() / np.abs(ref).max()))
        errors[name] = {"normwise_max_over_dm": worst_n, "maxabs_over_max": worst_m}
    total_pairs = w.nsub * w.nblock
    full_seconds = dt * total_pairs / len(pairs)
    value = len(w.dms) * w.data_seconds / full_seconds
    return {"value": value, "unit": "DM-s/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(pairs)} (subband, block) pairs x {len(w.dms)} DMs of the "
                      f"{total_pairs}-pair job, {dt:.1f} s wall on {threads} threads, "
                      f"extrapolated linearly"}, errors


def batch_leg(cdmt, synth, torch, dev, steps: int, reps: int):
    """The batched workload: 24 beams, each with its own subbands, N_bin,
    channels, overlap, DM list and output, in one persistent DM-stage launch
    per M_bin (1024, 2048 and 4096 here), replayed as a hipGraph after the
    autotuner picked each beam's forward-FFT split, the DM-stage schedule of
    the M_bin 1024, 2048 and 4096 beams, the DM tile and the grid."""
    import math
    draws = synth.batch_draws()
    beams, dm_seconds = [], 0.0
    for i, d in enumerate(draws):
        nov = cdmt.cdmt_noverlap_for(d.f_lo, synth.SUBBAND_MHZ, d.dm_max, d.nchan, d.ndec,
                                     cdmt.CHIRP_CHANNEL)
        nblock = math.ceil(synth.SUBBAND_MHZ * 1e6 / (d.nfft - nov))
        plan = cdmt.Plan(d.nsub, d.f_centre, synth.SUBBAND_MHZ, d.nfft, nov, d.nchan, d.ndec,
                         input_kind=cdmt.INPUT_CI8)
        ntin, ntout, nch = plan.shape(nblock)
        x = synth.device_noise("ci8", d.nsub, ntin, 16.0, 1607 + i, dev)
        out = torch.empty((d.ndm, ntout, nch), dtype=torch.float32, device=dev)
        beams.append((plan, nblock, x, list(d.dms), out))
        dm_seconds += d.ndm * cdmt.dm_seconds(nblock, d.nfft, nov, synth.SUBBAND_MHZ)
    batch = cdmt.Batch(beams, dev)
    stream = torch.cuda.Stream()
    t0 = time.perf_counter()
    tuned_ms = batch.autotune(stream, reps=reps)
    tune_s = time.perf_counter() - t0
    batch.run_graph(stream)                      # capture and one replay
    stream.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(stream)
    for _ in range(steps):
        batch.run_graph(stream)
    ev[1].record(stream)
    stream.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / steps
    res = {"workload": f"batch-{len(draws)}beam", "beams": len(draws),
           "value": round(dm_seconds / (ms / 1e3), 2), "unit": "DM-s/s",
           "ms_per_run": round(ms, 3), "dm_seconds_per_run": round(dm_seconds, 3),
           "launches": batch.get(cdmt.CDMT_BATCH_LAUNCHES),
           "items": batch.get(cdmt.CDMT_BATCH_ITEMS),
           "dm_tile": batch.get(cdmt.CDMT_BATCH_DM_TILE),
           "wg_per_cu": batch.get(cdmt.CDMT_BATCH_WG_PER_CU),
           "forward_n2_changed": sum(
               batch.beam_get(i, cdmt.CDMT_BATCH_BEAM_FWD_N2) !=
               cdmt.cdmt_plan_get(b[0].handle, cdmt.CDMT_OPT_FWD_N2)
               for i, b in enumerate(beams)),
           "m_bins": {str(m): sum(1 for d in draws if d.nfft // d.nchan == m)
                      for m in sorted({d.nfft // d.nchan for d in draws})},
           # the DM-stage radix schedule the autotuner kept per M_bin: "x3"
           # three radix-16 passes, "s16" / "s8" radix-16 / radix-8 Stockham
           "dm_stage_radix": {str(m): sorted({
               "x3" if batch.beam_get(i, cdmt.CDMT_BATCH_BEAM_FFT_SCHEDULE) == 0 and m >= 1024
               and batch.beam_get(i, cdmt.CDMT_BATCH_BEAM_LANE_BINS) == 16
               else "s%d" % (8 if batch.beam_get(i, cdmt.CDMT_BATCH_BEAM_LANE_BINS) == 8
                             and m >= 2048 else 16)
               for i, d in enumerate(draws) if d.nfft // d.nchan == m})
               for m in sorted({d.nfft // d.nchan for d in draws})},
           "autotune_best_ms": round(tuned_ms, 3), "autotune_s": round(tune_s, 1),
           "graph": True}
    log(f"batch: {len(draws)} beams, {ms:.3f} ms per run, {res['value']} DM-s/s")
    del batch, beams
    return res


def gradient_leg(cdmt, synth, torch, dev, steps: int):
    """dL/dDM for 64 candidate DMs on a 1 s segment of the LOFAR-shaped setup
    (288 subbands, complex float32 input, N_bin 65536): the forward DM stage
    at the candidates plus the adjoint, as one refinement step costs."""
    import ctypes as ct
    import math
    w = synth.LOFAR
    nblock = math.ceil(synth.SUBBAND_MHZ * 1e6 / (w.nfft - w.noverlap))
    plan = cdmt.Plan(w.nsub, w.f_centre, w.bw, w.nfft, w.noverlap, w.nchan, w.ndec,
                     input_kind=cdmt.INPUT_CF32, chirp_exact=1)
    ntin, ntout, nch = plan.shape(nblock)
    x = synth.device_noise("cf32", w.nsub, ntin, 1.0, 4242, dev)
    ws = plan.workspace(nblock, dev)
    plan.forward(x, nblock, ws)
    dms = [5.0 + 0.73 * i for i in range(64)]           # off-grid candidates
    out = torch.empty((len(dms), ntout, nch), dtype=torch.float32, device=dev)
    g = torch.randn((len(dms), ntout, nch), dtype=torch.float32, device=dev)
    gws = torch.empty(max(1, cdmt.cdmt_gradient_workspace_size(plan.handle, nblock, len(dms))),
                      dtype=torch.uint8, device=dev)
    dldm = torch.empty(len(dms), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def grad():
        cdmt.cdmt_dm_gradient(plan.handle, ct.c_void_p(ws.data_ptr()), ws.numel(), nblock, dms,
                              ct.c_void_p(g.data_ptr()), ct.c_void_p(gws.data_ptr()), gws.numel(),
                              ct.c_void_p(dldm.data_ptr()), ct.c_void_p(stream.cuda_stream))

    plan.dedisperse_spectra(nblock, dms, out, ws)
    grad()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record(stream)
    for _ in range(steps):
        plan.dedisperse_spectra(nblock, dms, out, ws)
    ev[1].record(stream)
    for _ in range(steps):
        grad()
    ev[2].record(stream)
    torch.cuda.synchronize()
    fwd = ev[0].elapsed_time(ev[1]) / steps
    adj = ev[1].elapsed_time(ev[2]) / steps
    data_s = cdmt.dm_seconds(nblock, w.nfft, w.noverlap, w.bw)
    log(f"gradient: 64 candidates, forward {fwd:.3f} ms, adjoint {adj:.3f} ms")
    return {"workload": f"gradient-{w.nsub}sub-64dm-1s", "candidates": len(dms),
            "data_seconds": round(data_s, 4), "forward_ms": round(fwd, 3),
            "gradient_ms": round(adj, 3),
            "gradient_dm_s_per_s": round(len(dms) * data_s / (adj / 1e3), 1)}


K_DM = 1.0 / 2.41e-4          # Sec. 2, after Eq. 1


def dispersed_pulses(torch, x, cfg, chirp_ref: int, sign: int, pulses, amp: float,
                     width: float = 0.0) -> int:
    """Input synthesis for the pulse measurements (the recipe of the test
    suite's injection, on the device): for each (dm, t0), a real pulse of
    energy amp^2 per polarisation centred on output sample t0, dispersed by the
    inverse of the plan's transfer function (Eq. 1 with the plan's nu0, per
    channel or per subband), on an nfft-sample window, added to both
    polarisations of float32 voltages x [nsub][ntime][2][2] in place.  The
    pulse is an impulse (width 0) or a Gaussian of standard deviation `width`
    samples (its spectrum tapered accordingly); FP64 arithmetic, torch FFTs.
    Returns the number of samples where the window was cut at the stream ends."""
    import math
    dev = x.device
    nsub, ntime = x.shape[0], x.shape[1]
    L = cfg["nfft"]
    bw, nchan = cfg["bw"], cfg["nchan"]
    k = torch.arange(L, device=dev)
    j = (k + L // 2) % L                                   # swapped index of FFT bin k
    rel = (j.double() - L / 2) * bw / L                    # MHz from the subband centre
    freq = torch.fft.fftfreq(L, device=dev, dtype=torch.float64)      # cycles per sample
    taper = torch.exp(-0.5 * (2 * math.pi * width * freq) ** 2)
    norm = amp / math.sqrt(float((taper ** 2).sum()) / L)  # energy amp^2 whatever the width
    impulse = norm * taper * (1.0 - 2.0 * (k % 2).double())    # centred at L / 2
    cut = 0
    for dm, t0 in pulses:
        n0 = cfg["noverlap"] // 2 + t0 * nchan * cfg["ndec"] + nchan * cfg["ndec"] // 2
        w0 = n0 - L // 2
        lo, hi = max(0, -w0), min(L, ntime - w0)
        cut += L - (hi - lo)
        for s0 in range(0, nsub, 32):
            s1 = min(nsub, s0 + 32)
            fs = cfg["f_centre"] + (torch.arange(s0, s1, device=dev).double() - (nsub - 1) / 2) * bw
            if chirp_ref == 0:
                ch = torch.div(j, L // nchan, rounding_mode="floor").double()
                nu0 = fs[:, None] - bw / 2 + (ch[None, :] + 0.5) * bw / nchan
                nu = rel[None, :] - (nu0 - fs[:, None])
            else:
                nu0 = fs[:, None].expand(-1, L)
                nu = rel[None, :].expand(s1 - s0, -1)
            cyc = 1e6 * K_DM * dm * nu * nu / (nu0 * nu0 * (nu0 + nu))
            spec = impulse[None, :] * torch.exp(torch.complex(torch.zeros_like(cyc),
                                                              -sign * 2 * math.pi * cyc))
            wav = torch.fft.ifft(spec, dim=1)[:, lo:hi]
            seg = x[s0:s1, w0 + lo:w0 + hi]
            seg[..., 0] += wav.real.float()[:, :, None]
            seg[..., 1] += wav.imag.float()[:, :, None]
    return cut


def pulse_snr(torch, fb, t0: int) -> float:
    """S/N of a pulse at output sample t0 of one DM's filterbank [t][ch]:
    (series[t0] - median) / (1.4826 MAD) of the channel-summed series."""
    s = fb.double().sum(dim=1)
    med = s.median()
    mad = (s - med).abs().median()
    return float((s[t0] - med) / (1.4826 * mad))


def refine_leg(cdmt, synth, torch, dev, ncand: int = 64, max_iter: int = 40):
    """DM refinement of candidates by gradient ascent: ncand candidates, each
    its own ~1 s segment (4 blocks) of the LOFAR-shaped setup (288 subbands,
    complex float32 noise sigma 1, N_bin 65536, overlap 15360, 16 channels,
    x8, nu0 per subband) with a pulse (S/N ~30) at a random continuous DM in
    [5, 60).  From the nearest trial of the 0.5-step coarse grid, the DM moves
    along d(S/N)/dDM (the differentiable DM stage, adjoint per block, spectra
    recomputed, never stored) with a step that grows by 1.5 after a gain and
    shrinks by 0.3 otherwise, until it moves less than 1e-4 pc cm^-3.  S/N is
    (s[t] - mean) / std of the channel-summed series s at the sample t where
    the coarse trial peaks."""
    import math
    w = synth.LOFAR
    nblock = 4
    plan = cdmt.Plan(w.nsub, w.f_centre, w.bw, w.nfft, w.noverlap, w.nchan, w.ndec,
                     input_kind=cdmt.INPUT_CF32, chirp_ref=cdmt.CHIRP_SUBBAND, chirp_exact=1)
    ntin, ntout, nch = plan.shape(nblock)
    cfg = {"nfft": w.nfft, "noverlap": w.noverlap, "nchan": w.nchan, "ndec": w.ndec,
           "bw": w.bw, "f_centre": w.f_centre}
    ws = plan.workspace(nblock, dev)
    tblk = (w.m - w.nd) // w.ndec
    errs, coarse_errs, iters, ms_each, evals = [], [], [], [], []
    for i, (dm_true, r_t, seed) in enumerate(synth.candidate_draws(ncand)):
        t0 = tblk + r_t % (2 * tblk)                 # inside blocks 1-2 of 4
        x = synth.device_noise("cf32", w.nsub, ntin, 1.0, seed, dev)
        dispersed_pulses(torch, x, cfg, 1, -1, [(dm_true, t0)], 90.0)
        plan.forward(x, nblock, ws)
        del x
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        dm_c = round(dm_true * 2.0) / 2.0
        with torch.no_grad():
            f0 = cdmt.dedisperse_dm(plan, torch.tensor([dm_c], dtype=torch.float64), nblock, ws)
            tpk = int(f0[0].double().sum(dim=1).argmax())

        def snr_grad(dm):
            d = torch.tensor([dm], dtype=torch.float64, requires_grad=True)
            F = cdmt.dedisperse_dm(plan, d, nblock, ws)
            sr = F[0].double().sum(dim=1)
            snr = (sr[tpk] - sr.mean()) / sr.std(correction=0)
            snr.backward()
            return float(snr.detach()), float(d.grad[0])

        dm, S, g = dm_c, *snr_grad(dm_c)
        step = 0.25 / max(abs(g), 1e-30)
        n_eval, it = 1, 0
        for it in range(1, max_iter + 1):
            cand = dm + step * g
            Sc, gc = snr_grad(cand)
            n_eval += 1
            if Sc > S:
                dm, S, g = cand, Sc, gc
                step *= 1.5
            else:
                step *= 0.3
            if abs(step * g) < 1e-4:
                break
        torch.cuda.synchronize()
        ms_each.append((time.perf_counter() - t_start) * 1e3)
        errs.append(abs(dm - dm_true))
        coarse_errs.append(abs(dm_c - dm_true))
        iters.append(it)
        evals.append(n_eval)
    del ws
    torch.cuda.empty_cache()
    med = lambda v: sorted(v)[len(v) // 2]
    data_s = cdmt.dm_seconds(nblock, w.nfft, w.noverlap, w.bw)
    res = {"workload": f"refine-{ncand}cand-{w.nsub}sub-1s", "candidates": ncand,
           "data_seconds_each": round(data_s, 4), "chirp_ref": "subband",
           "abs_err_median": med(errs), "abs_err_max": max(errs),
           "coarse_abs_err_median": med(coarse_errs),
           "iterations_mean": round(sum(iters) / len(iters), 2),
           "evaluations_mean": round(sum(evals) / len(evals), 2),
           "ms_per_refinement_median": round(med(ms_each), 2),
           "ms_per_evaluation": round(sum(ms_each) / sum(evals), 3)}
    log(f"refine: {ncand} candidates, |DM - true| median {res['abs_err_median']:.2e} max "
        f"{res['abs_err_max']:.2e}, {res['ms_per_refinement_median']} ms each")
    return res


def copy_bandwidth(torch, dev, nbytes: int = 4 << 30, reps: int = 5) -> float:
    """Measured device-to-device copy rate (bytes read + written per second):
    the practical HBM ceiling that the kernels are also compared with."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(reps):
        dst.copy_(src)
    ev[1].record()
    torch.cuda.synchronize()
    rate = 2 * nbytes * reps / (ev[0].elapsed_time(ev[1]) / 1e3)
    del src, dst
    torch.cuda.empty_cache()
    return rate


def incoherent_leg(cdmt, torch, plan, w, out, dms, steps: int):
    """The semi-coherent search's incoherent stage on the coherent output:
    the 40 filterbanks at DM 0.5..20 (of the 128), each dedispersed
    incoherently at 500 fine trials -0.5..+0.498 in steps of 0.002 around
    its DM (the paper's fine grid), 20000 trials in all.  Times the whole
    call (delay table, transpose, channel sums); the sums are bound by FP32
    additions, one per (trial, output sample, channel)."""
    sel = [i for i, d in enumerate(dms) if 0.5 <= d <= 20.0]
    fb = out[sel[0]:sel[-1] + 1]
    dm_coh = [dms[i] for i in sel]
    ddm0, ddm, ntrial = -0.5, 0.002, 500
    nout = cdmt.cdmt_incoherent_shape(plan.handle, w.nblock, dm_coh, ddm0, ddm, ntrial)
    iws = torch.empty(max(1, cdmt.cdmt_incoherent_workspace_size(plan.handle, w.nblock,
                                                                 len(dm_coh), ntrial)),
                      dtype=torch.uint8, device=out.device)
    iout = torch.empty((len(dm_coh), ntrial, nout), dtype=torch.float32, device=out.device)
    stream = torch.cuda.current_stream()
    cdmt.incoherent(plan, fb, w.nblock, dm_coh, ddm0, ddm, ntrial, out=iout, workspace=iws)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(stream)
    for _ in range(steps):
        cdmt.incoherent(plan, fb, w.nblock, dm_coh, ddm0, ddm, ntrial, out=iout, workspace=iws)
    ev[1].record(stream)
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / steps
    # the same stage fed channel-major filterbanks (what a plan with
    # CDMT_OPT_OUT_LAYOUT = 1 writes): no transpose inside the call
    cm_plan = cdmt.Plan(w.nsub, w.f_centre, w.bw, w.nfft, w.noverlap, w.nchan, w.ndec,
                        out_layout=cdmt.LAYOUT_CHANNEL_MAJOR)
    fb_cm = fb.transpose(1, 2).contiguous()
    cm_out = torch.empty_like(iout)
    cdmt.incoherent(cm_plan, fb_cm, w.nblock, dm_coh, ddm0, ddm, ntrial, out=cm_out,
                    workspace=iws)
    torch.cuda.synchronize()
    ev[0].record(stream)
    for _ in range(steps):
        cdmt.incoherent(cm_plan, fb_cm, w.nblock, dm_coh, ddm0, ddm, ntrial, out=cm_out,
                        workspace=iws)
    ev[1].record(stream)
    torch.cuda.synchronize()
    ms_cm = ev[0].elapsed_time(ev[1]) / steps
    same = bool(torch.equal(cm_out, iout))
    del fb_cm, cm_out
    nch = fb.shape[2]
    tsamp = w.nchan * w.ndec / (w.bw * 1e6)
    adds = len(dm_coh) * ntrial * nout * nch
    adds_peak = 256 * 128 * 2.4e9                # FP32 adds per second (128 lanes per CU per clock)
    traffic = measured_traffic("inc_sum_shared", PROFILE_INC, ("incoherent.hip", "plan.hpp"))
    del iws, iout
    return {"ms": round(ms, 3), "ms_channel_major_input": round(ms_cm, 3),
            "channel_major_identical": same, "coherent_dms": len(dm_coh), "fine_trials": ntrial,
            "nout": nout,
            "trial_seconds_per_s": round(len(dm_coh) * ntrial * nout * tsamp / (ms / 1e3), 1),
            "roofline": {"bound": "alu", "achieved": round(adds / (ms / 1e3) / 1e12, 2),
                         "peak": round(adds_peak / 1e12, 2), "unit": "Tadd/s",
                         "frac": round(adds / (ms / 1e3) / adds_peak, 4),
                         "traffic": traffic,
                         "note": "whole call (delays, transpose, sums) timed; sums alone in profiles/"}}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="lofar-hba-288sub-128dm")
    ap.add_argument("--dm-tile", type=int, default=None)
    ap.add_argument("--lane-bins", type=int, default=None, choices=[8, 16])
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16x3", "fp16x3"],
                    help="backward-FFT arithmetic of the DM stage")
    ap.add_argument("--chirp-ref", choices=["channel", "subband"], default="channel")
    ap.add_argument("--cpu-pairs", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--variants", action=argparse.BooleanOptionalAction, default=True,
                    help="also time the other DM-stage arithmetics (mixed vs FP32 plain)")
    ap.add_argument("--gradient", action=argparse.BooleanOptionalAction, default=True,
                    help="also time dL/dDM for 64 candidate DMs on a 1 s segment")
    ap.add_argument("--batch", action=argparse.BooleanOptionalAction, default=True,
                    help="also time the 24-beam batched workload (persistent launch, hipGraph)")
    ap.add_argument("--redigitise", action=argparse.BooleanOptionalAction, default=True,
                    help="also time the 8-bit redigitisation of the filterbank")
    ap.add_argument("--incoherent", action=argparse.BooleanOptionalAction, default=True,
                    help="also time the incoherent stage of a semi-coherent search")
    ap.add_argument("--pulse-amp-sigma", type=float, default=62.5,
                    help="amplitude of the injected pulses in units of the noise sigma")
    ap.add_argument("--refine", action=argparse.BooleanOptionalAction, default=True,
                    help="also refine 64 pulse candidates' DMs by gradient ascent")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 1 GiB device copy first (counter calibration for profiles)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1607_00909_amd as cdmt
    from paper_1607_00909_amd import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    w = synth.WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    kind = cdmt.INPUT_CI8 if w.input_kind == "ci8" else cdmt.INPUT_CF32
    chirp_ref = cdmt.CHIRP_CHANNEL if args.chirp_ref == "channel" else cdmt.CHIRP_SUBBAND
    log(f"workload {w.name}: generating {w.nsub}x{w.ntime_in} {w.input_kind} voltages on device")
    # noise (FP32 on the device), the workload's dispersed pulses added in
    # FP32, then the 8-bit quantisation (rint, clip to +-127) where the input
    # is int8: the same bytes for every precision and for the oracle
    x = synth.device_noise("cf32", w.nsub, w.ntime_in, w.sigma, w.seed, dev)
    pulses = synth.pulse_draws(w)
    pcfg = {"nfft": w.nfft, "noverlap": w.noverlap, "nchan": w.nchan, "ndec": w.ndec,
            "bw": w.bw, "f_centre": w.f_centre}
    # Gaussian pulses of 64 input samples (half an output sample) with S/N ~15
    # in the channel sum of the 4608-channel filterbank
    pulse_amp = args.pulse_amp_sigma * w.sigma
    dispersed_pulses(torch, x, pcfg, chirp_ref, -1, pulses, pulse_amp, width=64.0)
    clipped = 0
    if w.input_kind == "ci8":
        clipped = int((x.abs() > 127.5).sum())
        x8 = torch.empty(x.shape, dtype=torch.int8, device=dev)
        for s0 in range(0, w.nsub, 16):
            x8[s0:s0 + 16] = torch.clamp(torch.round(x[s0:s0 + 16]), -127, 127).to(torch.int8)
        del x
        x = x8
        torch.cuda.empty_cache()
    log(f"{len(pulses)} pulses injected (amplitude {pulse_amp:g}), {clipped} components clipped")
    plan = cdmt.Plan(w.nsub, w.f_centre, w.bw, w.nfft, w.noverlap, w.nchan, w.ndec,
                     input_kind=kind, chirp_ref=chirp_ref, dm_tile=args.dm_tile,
                     lane_bins=args.lane_bins)
    prec_code = {"fp32": 0, "bf16x3": 1, "fp16x3": 2}[args.precision]
    cdmt.cdmt_plan_set(plan.handle, cdmt.CDMT_OPT_PRECISION, prec_code)
    dm_tile = cdmt.cdmt_plan_get(plan.handle, cdmt.CDMT_OPT_DM_TILE)
    lane_bins = cdmt.cdmt_plan_get(plan.handle, cdmt.CDMT_OPT_LANE_BINS)
    ws = plan.workspace(w.nblock, dev)
    _, ntout, nch = plan.shape(w.nblock)
    out = torch.empty((len(w.dms), ntout, nch), dtype=torch.float32, device=dev)
    dms = list(w.dms)
    stream = torch.cuda.current_stream()
    log(f"workspace {ws.numel() / 1e9:.2f} GB, output {out.numel() * 4 / 1e9:.2f} GB, "
        f"dm_tile {dm_tile}")

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        plan.forward(x, w.nblock, ws)
        if ev is not None:
            ev[1].record(stream)
        plan.dedisperse_spectra(w.nblock, dms, out, ws)
        if ev is not None:
            ev[2].record(stream)

    if args.calib_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: 1 GiB read, 1 GiB written")
        del src, dst

    copy_gbs = copy_bandwidth(torch, dev) / 1e9
    log(f"device copy: {copy_gbs:.0f} GB/s (read + write)")

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup step {i + 1}/{args.warmup} done")

    events = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(events[i])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    fwd_ms = [e[0].elapsed_time(e[1]) for e in events]
    fus_ms = [e[1].elapsed_time(e[2]) for e in events]
    log(f"timed {args.steps} steps in {elapsed:.3f} s")

    ndm = len(dms)
    value = ndm * w.data_seconds * args.steps / elapsed
    fus_avg = sum(fus_ms) / len(fus_ms) / 1e3
    fwd_avg = sum(fwd_ms) / len(fwd_ms) / 1e3
    bins = w.nblock * w.nsub * w.nfft
    flops = bins * ndm * fused_flops_per_bin(w.m)
    spec_bytes = bins * 16
    ntiles = -(-ndm // dm_tile)
    fused_bytes = spec_bytes * ntiles + out.numel() * 4
    fwd_bytes = x.numel() * x.element_size() + 3 * spec_bytes
    achieved = flops / fus_avg / 1e12
    dm_kernel = dm_stage_kernel(w, recurrence=True)
    line = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "DM-s/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "nsub": w.nsub, "f_centre_mhz": w.f_centre,
                   "bw_sub_mhz": w.bw, "nfft": w.nfft, "noverlap": w.noverlap,
                   "nchan": w.nchan, "ndec": w.ndec, "nblock": w.nblock, "ndm": ndm,
                   "data_seconds": round(w.data_seconds, 6), "input": w.input_kind,
                   "chirp_ref": args.chirp_ref, "dm_tile": dm_tile, "lane_bins": lane_bins,
                   "precision": args.precision,
                   "parallelism": "none"},
        "roofline": {"kernel": dm_kernel, "bound": "alu",
                     "achieved": round(achieved, 3), "peak": round(VALU_FP32_PEAK_TFLOPS, 1),
                     "unit": "TFLOP/s", "frac": round(achieved / VALU_FP32_PEAK_TFLOPS, 4),
                     "traffic": measured_traffic(dm_kernel),
                     "hbm_algorithmic_GBs": round(fused_bytes / fus_avg / 1e9, 1),
                     "hbm_frac": round(fused_bytes / fus_avg / 1e9 / HBM_PEAK_GBS, 4)},
        "hbm_copy_GBs": round(copy_gbs, 1),
        "kernels_ms": {"forward (fwd_col+fwd_row)": round(fwd_avg * 1e3, 3),
                       "fused_dedisperse": round(fus_avg * 1e3, 3),
                       "forward_algorithmic_GBs": round(fwd_bytes / fwd_avg / 1e9, 1),
                       "forward_frac_of_copy": round(fwd_bytes / fwd_avg / 1e9 / copy_gbs, 4)},
        "realtime_factor": round(w.data_seconds / (elapsed / args.steps), 2),
        # per-step GPU time (forward + DM stage, HIP events), median over the
        # timed steps: robust to one slow step, beside the whole-job mean above
        "step_ms_median": round(sorted(f + u for f, u in zip(fwd_ms, fus_ms))[args.steps // 2], 3),
    }
    outputs = {args.precision: out}
    o2 = None
    dm_index = {d: i for i, d in enumerate(dms)}
    snr = {args.precision: [pulse_snr(torch, out[dm_index[dm]], t0) for dm, t0 in pulses]}
    line["pulses"] = {"injected": [{"dm": dm, "t0": t0} for dm, t0 in pulses],
                      "amplitude": pulse_amp, "gaussian_width_samples": 64,
                      "clipped_components": clipped}
    if args.variants and w.m == 4096:
        # the same job with the other backward-FFT arithmetics, and with the
        # transfer function evaluated afresh for every DM, same input
        variants = {}
        for name, code in (("fp32", 0), ("bf16x3", 1), ("fp16x3", 2), ("fp32-exact", 0)):
            if name == args.precision:
                continue
            cdmt.cdmt_plan_set(plan.handle, cdmt.CDMT_OPT_PRECISION, code)
            cdmt.cdmt_plan_set(plan.handle, cdmt.CDMT_OPT_CHIRP_EXACT,
                               1 if name == "fp32-exact" else 0)
            o2 = torch.empty_like(out)
            plan.dedisperse_spectra(w.nblock, dms, o2, ws)
            torch.cuda.synchronize()
            ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
            t1 = time.perf_counter()
            for i in range(args.steps):
                ev[i][0].record(stream)
                plan.dedisperse_spectra(w.nblock, dms, o2, ws)
                ev[i][1].record(stream)
            torch.cuda.synchronize()
            el = time.perf_counter() - t1
            ms = sum(e[0].elapsed_time(e[1]) for e in ev) / args.steps
            # normwise difference from the main run, DM by DM
            rel = 0.0
            for d in range(out.shape[0]):
                a_, b_ = o2[d].double(), out[d].double()
                rel = max(rel, float(((a_ - b_) ** 2).sum().sqrt() / (b_ ** 2).sum().sqrt()))
            variants[name] = {"value": round(ndm * w.data_seconds * args.steps / (el + fwd_avg * args.steps), 2),
                              "fused_ms": round(ms, 3),
                              "normwise_vs_" + args.precision: rel}
            if code != 0:
                # the method's flops (the FP32 accounting above) against the
                # matrix-core peak, and the matrix flops the kernel issues
                # (dense 32x32 DFT blocks, three split products)
                mflops = mx_mfma_flops_per_chunk_dm() * w.nblock * w.nsub * w.nchan * ndm
                ach = flops / (ms / 1e3) / 1e12
                iss = mflops / (ms / 1e3) / 1e12
                variants[name]["roofline"] = {
                    "kernel": "fused_dedisperse_mx", "bound": "mfma", "achieved": round(ach, 2),
                    "peak": MFMA_F16_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(ach / MFMA_F16_PEAK_TFLOPS, 4),
                    "issued_achieved": round(iss, 1),
                    "issued_frac": round(iss / MFMA_F16_PEAK_TFLOPS, 4),
                    "traffic": measured_traffic("fused_dedisperse_mx<%s>" % name)}
            snr[name] = [pulse_snr(torch, o2[dm_index[dm]], t0) for dm, t0 in pulses]
            outputs[name] = o2
            log(f"variant {name}: fused {ms:.3f} ms, normwise vs {args.precision} {rel:.2e}")
        cdmt.cdmt_plan_set(plan.handle, cdmt.CDMT_OPT_PRECISION, prec_code)
        cdmt.cdmt_plan_set(plan.handle, cdmt.CDMT_OPT_CHIRP_EXACT, 0)
        line["variants"] = variants
    base = snr.get("fp32")
    line["pulses"]["snr"] = {k: [round(v, 4) for v in vals] for k, vals in snr.items()}
    if base:
        line["pulses"]["snr_loss_vs_fp32"] = {
            k: max(abs(1.0 - v / b) for v, b in zip(vals, base))
            for k, vals in snr.items() if k != "fp32"}
    if args.redigitise:
        # 8-bit redigitisation of the FP32 filterbank (the paper's step after the
        # transpose), timed on its own: two reads of the filterbank, one byte write
        rws = torch.empty(max(1, cdmt.cdmt_redigitise_workspace_size(ndm, ntout, nch)),
                          dtype=torch.uint8, device=dev)
        codes, rmean, rscale = cdmt.redigitise(out, 64.0, 16.0, workspace=rws)
        torch.cuda.synchronize()
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
        for i in range(args.steps):
            ev[i][0].record(stream)
            cdmt.cdmt_redigitise(ctypes.c_void_p(out.data_ptr()), ndm, ntout, nch, 64.0, 16.0,
                                 ctypes.c_void_p(rws.data_ptr()), rws.numel(),
                                 ctypes.c_void_p(codes.data_ptr()),
                                 ctypes.c_void_p(rmean.data_ptr()),
                                 ctypes.c_void_p(rscale.data_ptr()),
                                 ctypes.c_void_p(stream.cuda_stream))
            ev[i][1].record(stream)
        torch.cuda.synchronize()
        rms = sum(e[0].elapsed_time(e[1]) for e in ev) / args.steps
        rbytes = 2 * out.numel() * 4 + out.numel() + 2 * rws.numel()
        line["redigitise"] = {"ms": round(rms, 3), "bound": "hbm",
                              "algorithmic_GBs": round(rbytes / rms / 1e6, 1),
                              "hbm_frac": round(rbytes / rms / 1e6 / HBM_PEAK_GBS, 4),
                              "frac_of_copy": round(rbytes / rms / 1e6 / copy_gbs, 4)}
        log(f"redigitise: {rms:.3f} ms")
        del codes, rws
    if args.incoherent:
        line["incoherent"] = incoherent_leg(cdmt, torch, plan, w, out, dms, args.steps)
        log(f"incoherent: {line['incoherent']['ms']:.3f} ms")
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        # every core this process may run on, up to the GPU machine's CPU share
        # of 16 (the pool is sized to that share whatever the host shows)
        avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
        threads = min(16, avail)
        log(f"cpu baseline: oracle on {args.cpu_pairs} (subband, block) pairs, {threads} threads "
            f"(nproc {os.cpu_count()}, affinity {avail})")
        line["cpu_baseline"], errs = cpu_baseline(w, x, args.cpu_pairs, threads, outputs, pulses)
        line["cpu_baseline"]["host_nproc"] = os.cpu_count()
        line["cpu_baseline"]["affinity_cores"] = avail
        line["errors_vs_oracle"] = errs
    if args.batch:
        # free the single-job buffers first: the batch holds ~125 GB of its own
        del outputs, out, ws, x, o2
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        line["batch"] = batch_leg(cdmt, synth, torch, dev, args.steps, 1)
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    if args.gradient:
        line["gradient"] = gradient_leg(cdmt, synth, torch, dev, args.steps)
    if args.refine:
        line["refine"] = refine_leg(cdmt, synth, torch, dev)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
