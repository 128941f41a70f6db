"""GPU checks of the library's guards: the Eq. 2 limit on the DM list (Sec. 2,
overlap-save) in a real run, and the autograd functions refusing a backward
pass whose spectra or plan changed after the forward pass."""
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


def _errors(gpu, ref):
    d = np.asarray(gpu, np.float64) - ref
    per_dm = np.sqrt((d ** 2).reshape(d.shape[0], -1).sum(1) / (ref ** 2).reshape(d.shape[0], -1).sum(1))
    return float(per_dm.max())


def test_dm_limit_in_a_run(hip_lib):
    """At |DM| = cdmt_dm_limit the run goes through and matches the oracle;
    just past it the call fails with CDMT_E_SHAPE and writes nothing; with
    CDMT_OPT_DM_CHECK = 0 the same DM runs (a circular convolution whose
    wrap-around reaches the kept samples, as the oracle computes it too)."""
    torch = _torch()
    print("[gpu-case] dm limit", flush=True)
    cfg = oracle.Config(2, 121.0, synth.SUBBAND_MHZ, 8192, 1024, 16, 4, chirp_ref=oracle.SUBBAND)
    nblock = 3
    plan = hip_lib.Plan(cfg.nsub, cfg.f_centre, cfg.bw, cfg.nfft, cfg.noverlap, cfg.nchan,
                        cfg.ndec, chirp_ref=hip_lib.CHIRP_SUBBAND)
    lim = plan.dm_limit()
    v = synth.encode_cf32(synth.gaussian_voltages(cfg.nsub, cfg.ntime_in(nblock), 1.0, 31))
    xd = torch.from_numpy(v).cuda()
    dms = [0.0, 0.5 * lim, -lim, lim]
    out = plan.dedisperse(xd, nblock, dms)
    torch.cuda.synchronize()
    assert _errors(out.cpu().numpy(), oracle.dedisperse(cfg, v, nblock, dms)) <= 1e-5
    past = [1.0, lim * 1.001]
    sentinel = torch.full(plan.out_shape(2, nblock), -3.0, device="cuda")
    with pytest.raises(hip_lib.CdmtError) as e:
        plan.dedisperse(xd, nblock, past, out=sentinel)
    assert e.value.status == hip_lib.CDMT_E_SHAPE
    torch.cuda.synchronize()
    assert bool((sentinel == -3.0).all())
    hip_lib.cdmt_plan_set(plan.handle, hip_lib.CDMT_OPT_DM_CHECK, 0)
    out = plan.dedisperse(xd, nblock, past + [3.0 * lim])
    torch.cuda.synchronize()
    ref = oracle.dedisperse(cfg, v, nblock, past + [3.0 * lim])
    assert _errors(out.cpu().numpy(), ref) <= 1e-5


def test_backward_refuses_rewritten_spectra(hip_lib):
    """A forward pass of the differentiable DM stage, then another forward
    stage on the same workspace (or a changed plan option), then backward:
    the backward pass raises instead of differentiating other spectra."""
    torch = _torch()
    print("[gpu-case] stale workspace in backward", flush=True)
    nsub, fc, nfft, nov, nchan, ndec, nblock = 2, 125.0, 8192, 2048, 4, 4, 2
    plan = hip_lib.Plan(nsub, fc, synth.SUBBAND_MHZ, nfft, nov, nchan, ndec, chirp_exact=1)
    ntin, _, _ = plan.shape(nblock)
    xa = torch.from_numpy(synth.encode_cf32(synth.gaussian_voltages(nsub, ntin, 1.0, 1))).cuda()
    xb = torch.from_numpy(synth.encode_cf32(synth.gaussian_voltages(nsub, ntin, 1.0, 2))).cuda()
    ws = plan.workspace(nblock)

    plan.forward(xa, nblock, ws)
    d = torch.tensor([3.0], dtype=torch.float64, requires_grad=True)
    F = hip_lib.dedisperse_dm(plan, d, nblock, ws)
    F.sum().backward()                                   # fresh: fine
    g_ok = float(d.grad[0])

    d = torch.tensor([3.0], dtype=torch.float64, requires_grad=True)
    F = hip_lib.dedisperse_dm(plan, d, nblock, ws)
    plan.forward(xb, nblock, ws)                         # the workspace now holds xb's spectra
    with pytest.raises(RuntimeError, match="rewritten"):
        F.sum().backward()

    plan.forward(xa, nblock, ws)
    d = torch.tensor([3.0], dtype=torch.float64, requires_grad=True)
    F = hip_lib.dedisperse_dm(plan, d, nblock, ws)
    hip_lib.cdmt_plan_set(plan.handle, hip_lib.CDMT_OPT_SIGN, 1)
    with pytest.raises(RuntimeError, match="option"):
        F.sum().backward()
    hip_lib.cdmt_plan_set(plan.handle, hip_lib.CDMT_OPT_SIGN, -1)

    # the whole-path function: two forwards on one workspace, then backward
    x = xa.clone().requires_grad_(True)
    d = torch.tensor([3.0], dtype=torch.float64, requires_grad=True)
    F1 = hip_lib.dedisperse(plan, x, d, nblock, ws)
    F2 = hip_lib.dedisperse(plan, xb, torch.tensor([3.0], dtype=torch.float64), nblock, ws)
    with pytest.raises(RuntimeError, match="rewritten"):
        F1.sum().backward()
    # the last forward is still current: its backward works and repeats the
    # first, fresh result for the same spectra
    plan.forward(xa, nblock, ws)
    d = torch.tensor([3.0], dtype=torch.float64, requires_grad=True)
    hip_lib.dedisperse_dm(plan, d, nblock, ws).sum().backward()
    torch.cuda.synchronize()
    assert float(d.grad[0]) == g_ok
    del F2
