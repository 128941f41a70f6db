"""GPU parity of the redigitisation (Sec. 3, after the transpose) with the
oracle, through the C ABI.

Both sides take the byte decision in FP32 from the same FP32 parameters, so
the codes are compared bit for bit against the oracle's quantiser fed the
library's (mean, scale).  The parameters themselves come from FP64 moments
summed in different orders (segments and pairwise merges here, two passes in
the oracle); they must agree with the oracle's to one FP32 unit in the last
place, and where they agree exactly the oracle's own codes must match too."""
import numpy as np
import pytest

import oracle
from oracle import redigit
from paper_1607_00909_amd import synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _ulps(a, b):
    a = np.asarray(a, np.float32)
    b = np.asarray(b, np.float32)
    return np.abs(a.view(np.int32).astype(np.int64) - b.view(np.int32).astype(np.int64))


def _compare(fb_host, codes, mean, scale, zero, cps, label):
    m_ref, k_ref = redigit.parameters(fb_host, cps)
    um, uk = _ulps(mean, m_ref), _ulps(scale, k_ref)
    print(f"{label}: parameters max ulp mean {um.max()}, scale {uk.max()}; "
          f"exact {np.mean((um == 0) & (uk == 0)):.6f}", flush=True)
    assert um.max() <= 1 and uk.max() <= 1
    # the bytes follow from the library's parameters exactly
    assert np.array_equal(codes, redigit.quantise(fb_host, mean, scale, zero))
    same = (um == 0) & (uk == 0)
    ref_codes = redigit.quantise(fb_host, m_ref, k_ref, zero)
    assert np.array_equal(codes.transpose(0, 2, 1)[same], ref_codes.transpose(0, 2, 1)[same])


def test_redigitise_tiny_workload_output(hip_lib):
    torch = _torch()
    w = synth.TINY
    cfg = oracle.Config(w.nsub, w.f_centre, w.bw, w.nfft, w.noverlap, w.nchan, w.ndec)
    x = synth.gaussian_voltages(w.nsub, w.ntime_in, w.sigma, w.seed)
    oracle.inject_impulse(cfg, x, 3, 10.0, oracle.pulse_sample(cfg, 700), 20.0 * w.sigma)
    v = synth.encode_cf32(x)
    print("[gpu-case] redigitise tiny workload", flush=True)
    plan = hip_lib.Plan(w.nsub, w.f_centre, w.bw, w.nfft, w.noverlap, w.nchan, w.ndec)
    fb = plan.dedisperse(torch.from_numpy(v).cuda(), w.nblock, list(w.dms))
    codes, mean, scale = hip_lib.redigitise(fb, 64.0, 16.0)
    torch.cuda.synchronize()
    _compare(fb.cpu().numpy(), codes.cpu().numpy(), mean.cpu().numpy(), scale.cpu().numpy(),
             64.0, 16.0, "tiny")
    # the impulse stays the brightest byte of its DM after redigitisation
    c = codes.cpu().numpy().astype(np.int64)
    assert np.unravel_index(np.argmax(c[10].sum(axis=1)), c[10].sum(axis=1).shape)[0] == 700


# (ndm, ntime, nchan, zero, counts_per_sigma, misalign): ragged segments (1, 1023,
# 1025, 2049 samples), channel counts off the 4-wide and 64-wide paths, a
# misaligned view (scalar path), parameters that clip at both ends
CASES = [
    (3, 2049, 64, 64.0, 16.0, False),
    (2, 1, 8, 64.0, 16.0, False),
    (1, 1023, 5, 128.0, 20.0, False),
    (4, 1025, 130, 10.0, 40.0, False),
    (2, 3000, 12, 250.0, 8.0, True),
]


@pytest.mark.parametrize("case", CASES, ids=[f"d{c[0]}-t{c[1]}-c{c[2]}" + ("-off" if c[5] else "")
                                             for c in CASES])
def test_redigitise_shapes(hip_lib, case):
    torch = _torch()
    ndm, nt, nch, zero, cps, off = case
    print(f"[gpu-case] redigitise {case}", flush=True)
    g = np.random.default_rng(ndm * 1000 + nt + nch)
    fb = g.gamma(6.0, 50.0, size=(ndm, nt, nch)).astype(np.float32)
    fb[:, :, 0] = 7.0                       # a constant channel: sigma 0, every byte at zero
    fb[0, nt // 2, -1] = 1e6                # a spike that clips
    if off:
        base = torch.zeros(fb.size + 1, dtype=torch.float32, device="cuda")
        dev = base[1:].view(ndm, nt, nch)
        dev.copy_(torch.from_numpy(fb))
    else:
        dev = torch.from_numpy(fb).cuda()
    codes, mean, scale = hip_lib.redigitise(dev, zero, cps)
    torch.cuda.synchronize()
    c = codes.cpu().numpy()
    _compare(fb, c, mean.cpu().numpy(), scale.cpu().numpy(), zero, cps, str(case))
    assert np.all(c[:, :, 0] == np.uint8(min(255, max(0, round(zero)))))
    assert scale.cpu().numpy()[:, 0].max() == 0.0


def test_redigitise_errors_write_nothing(hip_lib):
    torch = _torch()
    fb = torch.ones((2, 10, 4), dtype=torch.float32, device="cuda")
    codes = torch.full((2, 10, 4), 7, dtype=torch.uint8, device="cuda")
    mean = torch.full((2, 4), 3.0, device="cuda")
    scale = torch.full((2, 4), 3.0, device="cuda")
    ws = torch.empty(1, dtype=torch.uint8, device="cuda")   # too small
    import ctypes
    st = hip_lib.load().cdmt_redigitise(
        ctypes.c_void_p(fb.data_ptr()), 2, 10, 4, 64.0, 16.0, ctypes.c_void_p(ws.data_ptr()), 1,
        ctypes.c_void_p(codes.data_ptr()), ctypes.c_void_p(mean.data_ptr()),
        ctypes.c_void_p(scale.data_ptr()), None)
    torch.cuda.synchronize()
    assert st == hip_lib.CDMT_E_WORKSPACE
    assert bool((codes == 7).all()) and bool((mean == 3.0).all()) and bool((scale == 3.0).all())
