"""GPU DM gradient (cdmt_dm_gradient and the autograd form) against the
oracle's gradient, and DM refinement of an off-grid pulse by gradient ascent.

Bar: dL/dDM is a sum over every bin, channel, polarisation, subband and
block of the terms t = Re(conj(g_S') dS'/dDM); the GPU forms each term in
FP32 (two M_bin-point transforms, the transfer function and products) and
accumulates in FP64.  A rounding-error bound of a sum of terms computed with
relative error e each is e * sum|t|, so per DM
    |g_gpu - g_ref| <= c u sum|t|,  u = 2^-24,  c = 2 log2(M_bin) + 8
(about log2 M roundings per transform, two transforms, plus the transfer
function and the products), with sum|t| from the oracle (measured values are
printed)."""
import math

import numpy as np
import pytest

import oracle
from conftest import allow_short_overlap
from paper_1607_00909_amd import synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


U = 2.0 ** -24


def bar(nfft, nchan):
    """c u of the module's bound for M_bin = nfft / nchan."""
    return (2 * math.log2(nfft // nchan) + 8) * U


def _oracle_gradient(cfg, v, nblock, dms, G):
    """Sum over every (subband, block) of the oracle's gradient, and the sum
    of the absolute values of its per-bin terms; G in the library's output
    layout [ndm][ntime_out][nsub*nchan] (decreasing frequency)."""
    total = np.zeros(len(dms))
    absum = np.zeros(len(dms))
    for s in range(cfg.nsub):
        c1 = oracle.Config(1, cfg.sub_centre(s), cfg.bw, cfg.nfft, cfg.noverlap, cfg.nchan,
                           cfg.ndec, chirp_ref=cfg.chirp_ref)
        cols = [(cfg.nsub - 1 - s) * cfg.nchan + (cfg.nchan - 1 - c) for c in range(cfg.nchan)]
        for b in range(nblock):
            gb = G[:, b * cfg.tblk:(b + 1) * cfg.tblk, cols]
            g, a = oracle.dm_gradient(c1, v[s:s + 1], 0, b, dms, gb, with_abs=True)
            total += g
            absum += a
    return total, absum


CASES = [  # nsub, f_centre, nfft, noverlap, nchan, ndec, nblock, mode, kind
    (4, 120.0, 16384, 4096, 8, 4, 2, oracle.CHANNEL, "cf32"),
    (4, 120.0, 16384, 4096, 8, 4, 2, oracle.SUBBAND, "cf32"),
    # M_bin 4096: blocks of 448, 896 and 1792 output samples (G rows staged
    # through LDS two or four samples per lane, or loaded directly)
    (2, 140.0, 65536, 8192, 16, 8, 2, oracle.CHANNEL, "ci8"),
    (2, 140.0, 65536, 8192, 16, 4, 2, oracle.CHANNEL, "cf32"),
    (2, 140.0, 65536, 8192, 16, 2, 2, oracle.SUBBAND, "ci8"),
    (3, 150.0, 8192, 2048, 32, 2, 3, oracle.SUBBAND, "ci8"),
]


@pytest.mark.parametrize("case", CASES, ids=[f"M{c[2] // c[4]}-ndec{c[5]}-{'sub' if c[7] else 'chan'}"
                                             f"-{c[8]}" for c in CASES])
def test_dm_gradient_matches_oracle(hip_lib, case):
    torch = _torch()
    nsub, fc, nfft, nov, nchan, ndec, nblock, mode, kind = case
    print(f"[gpu-case] dm gradient {case}", flush=True)
    cfg = oracle.Config(nsub, fc, synth.SUBBAND_MHZ, nfft, nov, nchan, ndec, chirp_ref=mode)
    sigma = 16.0 if kind == "ci8" else 1.0
    x = synth.gaussian_voltages(nsub, cfg.ntime_in(nblock), sigma, 21)
    for s in range(nsub):
        oracle.inject_impulse(cfg, x, s, 10.37, oracle.pulse_sample(cfg, cfg.tblk + 7),
                              20.0 * sigma)
    v = synth.encode_ci8(x)[0] if kind == "ci8" else synth.encode_cf32(x)
    dms = [3.3, 10.0, 10.37, 25.0]
    plan = hip_lib.Plan(nsub, fc, synth.SUBBAND_MHZ, nfft, nov, nchan, ndec,
                        input_kind=hip_lib.INPUT_CI8 if kind == "ci8" else hip_lib.INPUT_CF32,
                        chirp_ref=mode, chirp_exact=1)
    allow_short_overlap(plan, dms)
    ws = plan.workspace(nblock)
    plan.forward(torch.from_numpy(v).cuda(), nblock, ws)
    _, ntout, nch = plan.shape(nblock)
    G = np.random.default_rng(8).standard_normal((len(dms), ntout, nch)).astype(np.float32)
    gdev = torch.from_numpy(G).cuda()
    n = hip_lib.cdmt_gradient_workspace_size(plan.handle, nblock, len(dms))
    gws = torch.empty(max(1, n), dtype=torch.uint8, device="cuda")
    dldm = torch.full((len(dms),), float("nan"), dtype=torch.float64, device="cuda")
    import ctypes
    hip_lib.cdmt_dm_gradient(plan.handle, ctypes.c_void_p(ws.data_ptr()), ws.numel(), nblock, dms,
                             ctypes.c_void_p(gdev.data_ptr()), ctypes.c_void_p(gws.data_ptr()),
                             gws.numel(), ctypes.c_void_p(dldm.data_ptr()), None)
    torch.cuda.synchronize()
    got = dldm.cpu().numpy()
    ref, absum = _oracle_gradient(cfg, v, nblock, dms, G.astype(np.float64))
    err = np.abs(got - ref) / absum
    print(f"gradient {got} vs oracle {ref}: error / sum|terms| {err.max():.2e} "
          f"(bar {bar(nfft, nchan):.2e})", flush=True)
    assert np.all(err <= bar(nfft, nchan))


def test_autograd_refines_an_off_grid_dm(hip_lib):
    """Gradient ascent on the pulse's channel-summed power finds the injected
    DM from the nearest coarse trial."""
    torch = _torch()
    print("[gpu-case] autograd DM refinement", flush=True)
    nsub, fc, nfft, nov, nchan, ndec, nblock = 8, 120.78125, 16384, 4096, 8, 4, 2
    cfg = oracle.Config(nsub, fc, synth.SUBBAND_MHZ, nfft, nov, nchan, ndec,
                        chirp_ref=oracle.SUBBAND)
    x = synth.gaussian_voltages(nsub, cfg.ntime_in(nblock), 0.05, 22)
    t0 = cfg.tblk + 100
    dm_true = 10.37
    for s in range(nsub):
        oracle.inject_impulse(cfg, x, s, dm_true, oracle.pulse_sample(cfg, t0), 20.0)
    v = synth.encode_cf32(x)
    plan = hip_lib.Plan(nsub, fc, synth.SUBBAND_MHZ, nfft, nov, nchan, ndec,
                        chirp_ref=hip_lib.CHIRP_SUBBAND, chirp_exact=1)
    ws = plan.workspace(nblock)
    plan.forward(torch.from_numpy(v).cuda(), nblock, ws)

    def loss_and_grad(dm):
        d = torch.tensor([dm], dtype=torch.float64, requires_grad=True)
        F = hip_lib.dedisperse_dm(plan, d, nblock, ws)
        L = F[0, t0, :].double().sum()
        L.backward()
        return float(L.detach()), float(d.grad[0])

    # the autograd gradient is the oracle's gradient of the same loss
    L0, g0 = loss_and_grad(10.0)
    G = np.zeros((1, nblock * cfg.tblk, nsub * nchan))
    G[0, t0, :] = 1.0
    ref, absum = _oracle_gradient(cfg, v, nblock, [10.0], G)
    print(f"autograd dL/dDM {g0:.6e}, oracle {ref[0]:.6e}, error / sum|terms| "
          f"{abs(g0 - ref[0]) / absum[0]:.2e}", flush=True)
    assert abs(g0 - ref[0]) <= bar(nfft, nchan) * absum[0]

    dm, L, g = 10.0, L0, g0
    step = 0.5 / abs(g)                          # first move of 0.5 pc cm^-3 at most
    for _ in range(40):
        cand = dm + step * g
        Lc, gc = loss_and_grad(cand)
        if Lc > L:
            dm, L, g = cand, Lc, gc
            step *= 1.5
        else:
            step *= 0.3
        if abs(step * g) < 1e-4:
            break
    print(f"refined DM {dm:.4f} (true {dm_true}), L {L0:.4e} -> {L:.4e}", flush=True)
    assert L > L0 and abs(dm - dm_true) < 0.02


def _snr_np(F, t0):
    """S/N of the channel-summed series s at sample t0: (s[t0] - mean) / std
    (population std).  A median/MAD form is not smooth in DM: its order
    statistics swap every few 1e-5 pc cm^-3, so differences at 1e-4 would
    straddle kinks."""
    s = F.sum(axis=1)
    return (s[t0] - s.mean()) / s.std()


def test_snr_gradient_matches_oracle_differences(hip_lib):
    """d(S/N)/dDM through the autograd function (S/N of the channel-summed
    series at the pulse sample, formed in torch) against central differences
    at 1e-4 pc cm^-3 of the same S/N of the oracle's FP64 filterbank.  (DM
    refinement by ascent is the power test above: this S/N at one sample has
    side maxima from the intra-channel smearing, and with a bright pulse it
    saturates near sqrt(n).)"""
    torch = _torch()
    print("[gpu-case] d(S/N)/dDM", flush=True)
    nsub, fc, nfft, nov, nchan, ndec, nblock = 8, 120.78125, 16384, 4096, 8, 4, 2
    cfg = oracle.Config(nsub, fc, synth.SUBBAND_MHZ, nfft, nov, nchan, ndec,
                        chirp_ref=oracle.SUBBAND)
    x = synth.gaussian_voltages(nsub, cfg.ntime_in(nblock), 0.5, 23)
    t0 = cfg.tblk + 100
    dm_true = 10.37
    for s in range(nsub):
        oracle.inject_impulse(cfg, x, s, dm_true, oracle.pulse_sample(cfg, t0), 20.0)
    v = synth.encode_cf32(x)
    plan = hip_lib.Plan(nsub, fc, synth.SUBBAND_MHZ, nfft, nov, nchan, ndec,
                        chirp_ref=hip_lib.CHIRP_SUBBAND, chirp_exact=1)
    ws = plan.workspace(nblock)
    plan.forward(torch.from_numpy(v).cuda(), nblock, ws)

    def snr_and_grad(dm):
        d = torch.tensor([dm], dtype=torch.float64, requires_grad=True)
        F = hip_lib.dedisperse_dm(plan, d, nblock, ws)
        s = F[0].double().sum(dim=1)
        snr = (s[t0] - s.mean()) / s.std(correction=0)
        snr.backward()
        return float(snr.detach()), float(d.grad[0])

    h = 1e-4
    for dm in (10.0, 10.2):
        S, g = snr_and_grad(dm)
        Sp = _snr_np(oracle.dedisperse(cfg, v, nblock, [dm + h])[0], t0)
        Sm = _snr_np(oracle.dedisperse(cfg, v, nblock, [dm - h])[0], t0)
        S0 = _snr_np(oracle.dedisperse(cfg, v, nblock, [dm])[0], t0)
        fd = (Sp - Sm) / (2 * h)
        print(f"DM {dm}: S/N gpu {S:.6f} oracle {S0:.6f}; d(S/N)/dDM autograd {g:.6e}, "
              f"oracle differences {fd:.6e}", flush=True)
        assert abs(S - S0) <= 1e-5 * abs(S0)
        assert abs(g - fd) <= 1e-4 * abs(fd)


@pytest.mark.parametrize("mode", [oracle.CHANNEL, oracle.SUBBAND], ids=["channel", "subband"])
def test_voltage_gradient_matches_oracle(hip_lib, mode):
    """dL/dvoltage for one DM against the oracle (normwise per subband), the
    accumulate flag, and the Euler identity sum Re(conj(dL/dx) x) = 2 L of the
    quadratic loss, on the GPU's own forward."""
    torch = _torch()
    import ctypes
    nsub, fc, nfft, nov, nchan, ndec, nblock = 3, 130.0, 8192, 2048, 8, 2, 3
    print(f"[gpu-case] voltage gradient mode {mode}", flush=True)
    cfg = oracle.Config(nsub, fc, synth.SUBBAND_MHZ, nfft, nov, nchan, ndec, chirp_ref=mode)
    x = synth.gaussian_voltages(nsub, cfg.ntime_in(nblock), 1.0, 41)
    v = synth.encode_cf32(x)
    dm = 6.5
    plan = hip_lib.Plan(nsub, fc, synth.SUBBAND_MHZ, nfft, nov, nchan, ndec, chirp_ref=mode,
                        chirp_exact=1)
    ws = plan.workspace(nblock)
    xd = torch.from_numpy(v).cuda()
    plan.forward(xd, nblock, ws)
    _, ntout, nch = plan.shape(nblock)
    G = np.random.default_rng(12).standard_normal((ntout, nch)).astype(np.float32)
    gd = torch.from_numpy(G).cuda()
    gsz = hip_lib.cdmt_voltage_gradient_workspace_size(plan.handle, nblock)
    gws = torch.empty(gsz, dtype=torch.uint8, device="cuda")
    gx = torch.full(xd.shape, float("nan"), dtype=torch.float32, device="cuda")
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    hip_lib.cdmt_voltage_gradient(plan.handle, P(ws), ws.numel(), nblock, dm, P(gd), P(gws),
                                  gws.numel(), P(gx), 0, None)
    torch.cuda.synchronize()
    got = gx.cpu().numpy().astype(np.float64)
    got = got[..., 0] + 1j * got[..., 1]
    worst = 0.0
    for s in range(nsub):
        cols = [(nsub - 1 - s) * nchan + (nchan - 1 - c) for c in range(nchan)]
        ref = oracle.voltage_gradient(cfg, v, s, nblock, dm, G[:, cols].astype(np.float64))
        e = np.linalg.norm(got[s] - ref) / np.linalg.norm(ref)
        worst = max(worst, e)
    print(f"voltage gradient vs oracle: worst normwise {worst:.2e}", flush=True)
    assert worst <= 1e-5
    # accumulate: a second call adds the same gradient
    hip_lib.cdmt_voltage_gradient(plan.handle, P(ws), ws.numel(), nblock, dm, P(gd), P(gws),
                                  gws.numel(), P(gx), 1, None)
    torch.cuda.synchronize()
    twice = gx.cpu().numpy().astype(np.float64)
    both = twice[..., 0] + 1j * twice[..., 1]
    assert np.linalg.norm(both - 2 * got) <= 1e-6 * np.linalg.norm(2 * got)
    # Euler identity on the GPU's forward filterbank
    F = plan.dedisperse_spectra(nblock, [dm], torch.empty((1, ntout, nch), device="cuda"), ws)
    L = float((F[0].double() * gd.double()).sum())
    lhs = float(np.real(np.conj(got) * (v[..., 0] + 1j * v[..., 1])).sum())
    print(f"Euler: sum Re(conj(g) x) {lhs:.6e}, 2L {2 * L:.6e}", flush=True)
    assert abs(lhs - 2 * L) <= 1e-5 * abs(2 * L)


def test_autograd_voltage_and_dm_gradients(hip_lib):
    """The autograd form returns the same gradients as the direct calls."""
    torch = _torch()
    import ctypes
    print("[gpu-case] autograd voltages + DMs", flush=True)
    nsub, fc, nfft, nov, nchan, ndec, nblock = 2, 125.0, 8192, 2048, 4, 4, 2
    plan = hip_lib.Plan(nsub, fc, synth.SUBBAND_MHZ, nfft, nov, nchan, ndec, chirp_exact=1)
    ntin, ntout, nch = plan.shape(nblock)
    v = synth.encode_cf32(synth.gaussian_voltages(nsub, ntin, 1.0, 43))
    ws = plan.workspace(nblock)
    x = torch.from_numpy(v).cuda().requires_grad_(True)
    dms = torch.tensor([2.0, 9.5, 30.0], dtype=torch.float64, requires_grad=True)
    G = torch.randn((3, ntout, nch), device="cuda", generator=torch.Generator("cuda").manual_seed(5))
    F = hip_lib.dedisperse(plan, x, dms, nblock, ws)
    (F * G).sum().backward()
    torch.cuda.synchronize()
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    gsz = hip_lib.cdmt_voltage_gradient_workspace_size(plan.handle, nblock)
    gws = torch.empty(gsz, dtype=torch.uint8, device="cuda")
    gx = torch.empty_like(x.detach())
    for i, dm in enumerate(dms.tolist()):
        hip_lib.cdmt_voltage_gradient(plan.handle, P(ws), ws.numel(), nblock, dm,
                                      P(G[i].contiguous()), P(gws), gws.numel(), P(gx),
                                      1 if i else 0, None)
    n = hip_lib.cdmt_gradient_workspace_size(plan.handle, nblock, 3)
    gws2 = torch.empty(n, dtype=torch.uint8, device="cuda")
    dldm = torch.empty(3, dtype=torch.float64, device="cuda")
    hip_lib.cdmt_dm_gradient(plan.handle, P(ws), ws.numel(), nblock, dms.tolist(), P(G),
                             P(gws2), gws2.numel(), P(dldm), None)
    torch.cuda.synchronize()
    assert torch.equal(x.grad, gx)
    assert torch.equal(dms.grad, dldm.cpu())


def test_gradients_in_the_channel_major_layout(hip_lib):
    """With CDMT_OPT_OUT_LAYOUT = 1, dL/dF is read [DM][channel][time]: both
    gradients equal the default layout's, bit for bit, for the transposed G."""
    torch = _torch()
    import ctypes
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    nsub, fc, nfft, nov, nchan, ndec, nblock = 3, 130.0, 16384, 4096, 8, 4, 2
    print("[gpu-case] gradients, channel-major layout", flush=True)
    cfg = oracle.Config(nsub, fc, synth.SUBBAND_MHZ, nfft, nov, nchan, ndec)
    v = synth.encode_cf32(synth.gaussian_voltages(nsub, cfg.ntime_in(nblock), 1.0, 43))
    xd = torch.from_numpy(v).cuda()
    dms = [2.0, 7.7, 19.0]
    res = []
    for layout in (0, 1):
        plan = hip_lib.Plan(nsub, fc, synth.SUBBAND_MHZ, nfft, nov, nchan, ndec, chirp_exact=1,
                            out_layout=layout)
        ws = plan.workspace(nblock)
        plan.forward(xd, nblock, ws)
        _, ntout, nch = plan.shape(nblock)
        G = torch.from_numpy(np.random.default_rng(14).standard_normal(
            (len(dms), ntout, nch)).astype(np.float32)).cuda()
        if layout:
            G = G.transpose(1, 2).contiguous()
        n = hip_lib.cdmt_gradient_workspace_size(plan.handle, nblock, len(dms))
        gws = torch.empty(max(1, n), dtype=torch.uint8, device="cuda")
        dldm = torch.empty(len(dms), dtype=torch.float64, device="cuda")
        hip_lib.cdmt_dm_gradient(plan.handle, P(ws), ws.numel(), nblock, dms, P(G), P(gws),
                                 gws.numel(), P(dldm), None)
        vsz = hip_lib.cdmt_voltage_gradient_workspace_size(plan.handle, nblock)
        vws = torch.empty(vsz, dtype=torch.uint8, device="cuda")
        gx = torch.empty(xd.shape, dtype=torch.float32, device="cuda")
        hip_lib.cdmt_voltage_gradient(plan.handle, P(ws), ws.numel(), nblock, dms[1], P(G[1]),
                                      P(vws), vws.numel(), P(gx), 0, None)
        torch.cuda.synchronize()
        res.append((dldm.cpu(), gx.cpu()))
    assert torch.equal(res[0][0], res[1][0])
    assert torch.equal(res[0][1], res[1][1])


def test_dm_gradient_at_full_size_on_sampled_pairs(hip_lib):
    """The benchmark's gradient configuration (288 subbands, N_bin 65536, ~1 s,
    64 off-grid candidate DMs): dL/dF is non-zero on two sampled (subband,
    block) pairs only, so the GPU's dL/dDM is the sum of the oracle's gradients
    of those two pairs."""
    torch = _torch()
    import ctypes
    import math
    w = synth.LOFAR
    nblock = math.ceil(synth.SUBBAND_MHZ * 1e6 / (w.nfft - w.noverlap))
    print("[gpu-case] dm gradient, full size, sampled pairs", flush=True)
    plan = hip_lib.Plan(w.nsub, w.f_centre, w.bw, w.nfft, w.noverlap, w.nchan, w.ndec,
                        input_kind=hip_lib.INPUT_CF32, chirp_exact=1)
    ntin, ntout, nch = plan.shape(nblock)
    x = synth.device_noise("cf32", w.nsub, ntin, 1.0, 4242, "cuda")
    ws = plan.workspace(nblock)
    plan.forward(x, nblock, ws)
    dms = [5.0 + 0.73 * i for i in range(64)]
    cfg = oracle.Config(w.nsub, w.f_centre, w.bw, w.nfft, w.noverlap, w.nchan, w.ndec)
    r = np.random.default_rng(15)
    G = torch.zeros((len(dms), ntout, nch), dtype=torch.float32, device="cuda")
    total, absum = np.zeros(len(dms)), np.zeros(len(dms))
    for s, b in ((17, 1), (250, nblock - 1)):
        cols = [(w.nsub - 1 - s) * w.nchan + (w.nchan - 1 - c) for c in range(w.nchan)]
        gb = r.standard_normal((len(dms), cfg.tblk, w.nchan)).astype(np.float32)
        G[:, b * cfg.tblk:(b + 1) * cfg.tblk, cols] = torch.from_numpy(gb).cuda()
        c1 = oracle.Config(1, cfg.sub_centre(s), cfg.bw, cfg.nfft, cfg.noverlap, cfg.nchan,
                           cfg.ndec)
        g, a = oracle.dm_gradient(c1, x[s:s + 1].cpu().numpy(), 0, b, dms,
                                  gb.astype(np.float64), with_abs=True)
        total += g
        absum += a
    n = hip_lib.cdmt_gradient_workspace_size(plan.handle, nblock, len(dms))
    gws = torch.empty(max(1, n), dtype=torch.uint8, device="cuda")
    dldm = torch.empty(len(dms), dtype=torch.float64, device="cuda")
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    hip_lib.cdmt_dm_gradient(plan.handle, P(ws), ws.numel(), nblock, dms, P(G), P(gws),
                             gws.numel(), P(dldm), None)
    torch.cuda.synchronize()
    # each DM's gradient is a sum of random-signed terms that can nearly
    # cancel: the error is bounded by the terms' absolute sum (module bar)
    err = np.abs(dldm.cpu().numpy() - total)
    print(f"full-size gradient vs oracle (2 pairs x 64 DMs): worst error / sum|terms| "
          f"{(err / absum).max():.2e} (bar {bar(w.nfft, w.nchan):.2e})", flush=True)
    assert np.all(err <= bar(w.nfft, w.nchan) * absum)


@pytest.mark.parametrize("cand", [0, 1])
def test_refinement_of_a_candidate_at_full_size(hip_lib, cand):
    """A candidate of the refinement workload at full size: its own ~1 s
    segment (4 blocks of N_bin 65536) of 288 subbands, complex float32 noise
    sigma 1, a pulse injected by the oracle (inverse transfer function, nu0 per
    subband) at a random continuous DM.  From the nearest trial of the 0.5-step
    coarse grid, gradient ascent on the S/N of the channel-summed series finds
    the DM to within 0.02 pc cm^-3; at the coarse trial, d(S/N)/dDM from the
    autograd function matches central differences (step 1e-4 pc cm^-3) of the
    oracle's FP64 S/N over the whole segment; and the DM gradient of a loss on
    two sampled (subband, block) pairs, one holding the pulse, matches the
    oracle's within the module's rounding bound."""
    torch = _torch()
    import ctypes
    w = synth.LOFAR
    nblock = 4
    dm_true, r_t, seed = synth.candidate_draws(64)[cand]
    cfg = oracle.Config(w.nsub, w.f_centre, w.bw, w.nfft, w.noverlap, w.nchan, w.ndec,
                        chirp_ref=oracle.SUBBAND)
    t0 = cfg.tblk + r_t % (2 * cfg.tblk)
    print(f"[gpu-case] full-size refinement, candidate {cand}: DM {dm_true:.4f}, t0 {t0}",
          flush=True)
    x = synth.gaussian_voltages(w.nsub, cfg.ntime_in(nblock), 1.0, seed)
    for s in range(w.nsub):
        oracle.inject_impulse(cfg, x, s, dm_true, oracle.pulse_sample(cfg, t0), 90.0)
    v = synth.encode_cf32(x)
    del x
    plan = hip_lib.Plan(w.nsub, w.f_centre, w.bw, w.nfft, w.noverlap, w.nchan, w.ndec,
                        chirp_ref=hip_lib.CHIRP_SUBBAND, chirp_exact=1)
    ws = plan.workspace(nblock)
    xd = torch.from_numpy(v).cuda()
    plan.forward(xd, nblock, ws)
    dm_c = round(dm_true * 2.0) / 2.0
    with torch.no_grad():
        f0 = hip_lib.dedisperse_dm(plan, torch.tensor([dm_c], dtype=torch.float64), nblock, ws)
        tpk = int(f0[0].double().sum(dim=1).argmax())
    assert tpk == t0

    def snr_grad(dm):
        d = torch.tensor([dm], dtype=torch.float64, requires_grad=True)
        F = hip_lib.dedisperse_dm(plan, d, nblock, ws)
        sr = F[0].double().sum(dim=1)
        snr = (sr[tpk] - sr.mean()) / sr.std(correction=0)
        snr.backward()
        return float(snr.detach()), float(d.grad[0])

    # d(S/N)/dDM at the coarse trial against the oracle's central differences
    h = 1e-4
    S0, g0 = snr_grad(dm_c)
    Sp = _snr_np(oracle.dedisperse(cfg, v, nblock, [dm_c + h])[0], tpk)
    Sm = _snr_np(oracle.dedisperse(cfg, v, nblock, [dm_c - h])[0], tpk)
    fd = (Sp - Sm) / (2 * h)
    print(f"coarse DM {dm_c}: S/N {S0:.5f}, d(S/N)/dDM autograd {g0:.6e}, oracle differences "
          f"{fd:.6e}", flush=True)
    assert abs(g0 - fd) <= 1e-3 * abs(fd)

    # gradient ascent from the coarse trial
    dm, S, g = dm_c, S0, g0
    step = 0.25 / abs(g)
    for it in range(40):
        cand_dm = dm + step * g
        Sc, gc = snr_grad(cand_dm)
        if Sc > S:
            dm, S, g = cand_dm, Sc, gc
            step *= 1.5
        else:
            step *= 0.3
        if abs(step * g) < 1e-4:
            break
    print(f"refined DM {dm:.5f} (true {dm_true:.5f}, coarse {dm_c}) after {it + 1} steps, "
          f"S/N {S0:.3f} -> {S:.3f}", flush=True)
    assert abs(dm - dm_true) <= 0.02
    assert S > S0 or abs(dm_c - dm_true) < 0.02

    # the DM gradient on two sampled pairs (the pulse's block and another)
    r = np.random.default_rng(31 + cand)
    _, ntout, nch = plan.shape(nblock)
    G = torch.zeros((1, ntout, nch), dtype=torch.float32, device="cuda")
    total, absum = np.zeros(1), np.zeros(1)
    for s, b in ((41, t0 // cfg.tblk), (250, 3)):
        cols = [(w.nsub - 1 - s) * w.nchan + (w.nchan - 1 - c) for c in range(w.nchan)]
        gb = r.standard_normal((1, cfg.tblk, w.nchan)).astype(np.float32)
        G[:, b * cfg.tblk:(b + 1) * cfg.tblk, cols] = torch.from_numpy(gb).cuda()
        c1 = oracle.Config(1, cfg.sub_centre(s), cfg.bw, cfg.nfft, cfg.noverlap, cfg.nchan,
                           cfg.ndec, chirp_ref=oracle.SUBBAND)
        gg, a = oracle.dm_gradient(c1, v[s:s + 1], 0, b, [dm], gb.astype(np.float64),
                                   with_abs=True)
        total += gg
        absum += a
    n = hip_lib.cdmt_gradient_workspace_size(plan.handle, nblock, 1)
    gws = torch.empty(max(1, n), dtype=torch.uint8, device="cuda")
    dldm = torch.empty(1, dtype=torch.float64, device="cuda")
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    hip_lib.cdmt_dm_gradient(plan.handle, P(ws), ws.numel(), nblock, [dm], P(G), P(gws),
                             gws.numel(), P(dldm), None)
    torch.cuda.synchronize()
    err = abs(float(dldm.cpu()[0]) - total[0])
    print(f"sampled-pair gradient at the refined DM: error / sum|terms| {err / absum[0]:.2e} "
          f"(bar {bar(w.nfft, w.nchan):.2e})", flush=True)
    assert err <= bar(w.nfft, w.nchan) * absum[0]
