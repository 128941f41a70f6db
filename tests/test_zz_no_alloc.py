"""cdmt_dm_gradient_noalloc (partial sums in the library's per-GPU scratch
array instead of a caller workspace) against cdmt_dm_gradient, through the
C ABI: two calls in a row, the second on a smaller input, each bitwise equal
to the workspace form (same kernels, same summation order) and within the
gradient bound of the oracle; a size beyond the scratch array is rejected
before anything is written."""
import ctypes
import math

import numpy as np
import pytest

import oracle
from conftest import allow_short_overlap
from paper_1607_00909_amd import synth

pytestmark = pytest.mark.gpu

U = 2.0 ** -24

CASES = [  # nsub, f_centre, nfft, noverlap, nchan, ndec, nblock, mode, kind, dms
    (2, 140.0, 65536, 8192, 16, 8, 3, oracle.CHANNEL, "ci8", [3.3, 10.0, 10.37, 25.0, 31.5]),
    (2, 120.0, 16384, 4096, 8, 4, 2, oracle.SUBBAND, "cf32", [2.0, 10.37, 12.5]),
]


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _oracle_gradient(cfg, v, nblock, dms, G):
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


def _run(hip_lib, torch, case, seed):
    nsub, fc, nfft, nov, nchan, ndec, nblock, mode, kind, dms = case
    print(f"[gpu-case] no-alloc dm gradient {case[:9]}", flush=True)
    cfg = oracle.Config(nsub, fc, synth.SUBBAND_MHZ, nfft, nov, nchan, ndec, chirp_ref=mode)
    sigma = 16.0 if kind == "ci8" else 1.0
    x = synth.gaussian_voltages(nsub, cfg.ntime_in(nblock), sigma, seed)
    for s in range(nsub):
        oracle.inject_impulse(cfg, x, s, 10.37, oracle.pulse_sample(cfg, cfg.tblk + 7),
                              20.0 * sigma)
    v = synth.encode_ci8(x)[0] if kind == "ci8" else synth.encode_cf32(x)
    plan = hip_lib.Plan(nsub, fc, synth.SUBBAND_MHZ, nfft, nov, nchan, ndec,
                        input_kind=hip_lib.INPUT_CI8 if kind == "ci8" else hip_lib.INPUT_CF32,
                        chirp_ref=mode, chirp_exact=1)
    allow_short_overlap(plan, dms)
    ws = plan.workspace(nblock)
    plan.forward(torch.from_numpy(v).cuda(), nblock, ws)
    _, ntout, nch = plan.shape(nblock)
    G = np.random.default_rng(seed).standard_normal((len(dms), ntout, nch)).astype(np.float32)
    gdev = torch.from_numpy(G).cuda()
    n = hip_lib.cdmt_gradient_workspace_size(plan.handle, nblock, len(dms))
    assert n <= hip_lib.cdmt_noalloc_scratch_bytes()
    gws = torch.empty(max(1, n), dtype=torch.uint8, device="cuda")
    ref_ws = torch.full((len(dms),), float("nan"), dtype=torch.float64, device="cuda")
    got = torch.full((len(dms),), float("nan"), dtype=torch.float64, device="cuda")
    wsp = ctypes.c_void_p(ws.data_ptr())
    gp = ctypes.c_void_p(gdev.data_ptr())
    hip_lib.cdmt_dm_gradient(plan.handle, wsp, ws.numel(), nblock, dms, gp,
                             ctypes.c_void_p(gws.data_ptr()), gws.numel(),
                             ctypes.c_void_p(ref_ws.data_ptr()), None)
    hip_lib.cdmt_dm_gradient_noalloc(plan.handle, wsp, ws.numel(), nblock, dms, gp,
                                     ctypes.c_void_p(got.data_ptr()), None)
    torch.cuda.synchronize()
    a = got.cpu().numpy()
    b = ref_ws.cpu().numpy()
    ref, absum = _oracle_gradient(cfg, v, nblock, dms, G.astype(np.float64))
    c = (2 * math.log2(nfft // nchan) + 8) * U
    err = np.abs(a - ref) / absum
    print(f"no-alloc {a} workspace {b} oracle {ref}: error / sum|terms| {err.max():.2e} "
          f"(bar {c:.2e})", flush=True)
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
    assert np.all(err <= c)


def test_noalloc_gradient_two_calls(hip_lib):
    torch = _torch()
    _run(hip_lib, torch, CASES[0], 31)
    _run(hip_lib, torch, CASES[1], 32)   # smaller: fewer subband blocks and DMs


def test_noalloc_gradient_rejects_oversize(hip_lib):
    torch = _torch()
    print("[gpu-case] no-alloc dm gradient oversize", flush=True)
    # ndec 64 keeps dL/dF small (24 samples per block) against the partials
    nsub, fc, nfft, nov, nchan, ndec, nblock = 2, 120.0, 16384, 4096, 8, 64, 1
    plan = hip_lib.Plan(nsub, fc, synth.SUBBAND_MHZ, nfft, nov, nchan, ndec, chirp_exact=1)
    ws = plan.workspace(nblock)
    cap = hip_lib.cdmt_noalloc_scratch_bytes()
    per_dm = hip_lib.cdmt_gradient_workspace_size(plan.handle, nblock, 1)
    ndm = cap // per_dm + 1
    dms = np.linspace(0.0, 1.0, ndm)
    _, ntout, nch = plan.shape(nblock)
    gdev = torch.zeros((ndm, ntout, nch), dtype=torch.float32, device="cuda")
    dldm = torch.full((ndm,), float("nan"), dtype=torch.float64, device="cuda")
    with pytest.raises(hip_lib.CdmtError) as e:
        hip_lib.cdmt_dm_gradient_noalloc(plan.handle, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                         nblock, dms, ctypes.c_void_p(gdev.data_ptr()),
                                         ctypes.c_void_p(dldm.data_ptr()), None)
    assert e.value.status == hip_lib.CDMT_E_WORKSPACE
    torch.cuda.synchronize()
    assert torch.isnan(dldm).all()
