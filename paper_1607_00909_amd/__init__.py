"""Python binding of the MI355X coherent-dedispersion library (libcdmt.so).

Thin ctypes layer over the C ABI in include/cdmt.h: the functions below have
the C names and only marshal arguments (device pointers from torch tensors,
HIP streams from torch streams).  Every step of the computation runs in the
library's HIP kernels.  If the library has not been built, the first call
raises; there is no fallback.

Method: coherent dedispersion to many DM trials (Bassa, Pleunis & Hessels
2016, Sec. 2-3, Alg. 1).
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcdmt.so")

# enum cdmt_status
CDMT_OK, CDMT_E_ARG, CDMT_E_SHAPE, CDMT_E_WORKSPACE, CDMT_E_DEVICE, CDMT_E_UNSUPPORTED = \
    0, -1, -2, -3, -4, -5
# enum cdmt_opt
CDMT_OPT_INPUT, CDMT_OPT_CHIRP_REF, CDMT_OPT_SIGN, CDMT_OPT_PRECISION, CDMT_OPT_DM_TILE, \
    CDMT_OPT_CHIRP_EXACT, CDMT_OPT_LANE_BINS, CDMT_OPT_FWD_N2, CDMT_OPT_OUT_LAYOUT, \
    CDMT_OPT_DM_CHECK, CDMT_OPT_FFT_SCHEDULE = 0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10
LAYOUT_TIME_MAJOR, LAYOUT_CHANNEL_MAJOR = 0, 1
INPUT_CF32, INPUT_CI8 = 0, 1
CHIRP_CHANNEL, CHIRP_SUBBAND = 0, 1

# every symbol include/cdmt.h declares
EXPORTS = ("cdmt_plan", "cdmt_plan_set", "cdmt_plan_get", "cdmt_noverlap_for", "cdmt_dm_limit",
           "cdmt_output_shape", "cdmt_workspace_size", "cdmt_forward",
           "cdmt_dedisperse_spectra", "cdmt_dedisperse", "cdmt_destroy", "cdmt_status_string",
           "cdmt_redigitise_workspace_size", "cdmt_redigitise",
           "cdmt_batch_workspace_size", "cdmt_batch_create", "cdmt_batch_set", "cdmt_batch_get",
           "cdmt_batch_run", "cdmt_batch_run_graph", "cdmt_batch_autotune", "cdmt_batch_destroy",
           "cdmt_batch_beam_set", "cdmt_batch_beam_get",
           "cdmt_gradient_workspace_size", "cdmt_dm_gradient", "cdmt_dm_gradient_noalloc",
           "cdmt_noalloc_scratch_bytes",
           "cdmt_voltage_gradient_workspace_size", "cdmt_voltage_gradient",
           "cdmt_incoherent_shape", "cdmt_incoherent_workspace_size", "cdmt_incoherent")
# enum cdmt_batch_opt
CDMT_BATCH_DM_TILE, CDMT_BATCH_WG_PER_CU, CDMT_BATCH_ITEMS, CDMT_BATCH_LAUNCHES = 0, 1, 2, 3
# enum cdmt_batch_beam_opt
CDMT_BATCH_BEAM_FWD_N2 = 0
CDMT_BATCH_BEAM_FFT_SCHEDULE = 1
CDMT_BATCH_BEAM_LANE_BINS = 2


class Beam(ctypes.Structure):
    """cdmt_beam_t: one beam of a batch."""
    _fields_ = [("plan", ctypes.c_void_p), ("nblock", ctypes.c_int),
                ("voltages", ctypes.c_void_p), ("dm_list", ctypes.POINTER(ctypes.c_double)),
                ("ndm", ctypes.c_int), ("out", ctypes.c_void_p)]

_lib = None
_lock = threading.Lock()


class CdmtError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {cdmt_status_string(status)} ({status})")


def load():
    """Load libcdmt.so (after torch, so both use the same HIP runtime)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1607_00909_amd.build`")
        try:
            import torch  # noqa: F401  (load torch's HIP runtime first)
        except ImportError:
            pass
        lib = ctypes.CDLL(LIB_PATH)
        P, I, D, Z = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
        LL = ctypes.c_longlong
        lib.cdmt_plan.argtypes = [ctypes.POINTER(P), I, D, D, I, I, I, I]
        lib.cdmt_plan_set.argtypes = [P, I, I]
        lib.cdmt_plan_get.argtypes = [P, I, ctypes.POINTER(I)]
        lib.cdmt_noverlap_for.argtypes = [D, D, D, I, I, I, ctypes.POINTER(I)]
        lib.cdmt_dm_limit.argtypes = [P, ctypes.POINTER(D)]
        lib.cdmt_output_shape.argtypes = [P, I, ctypes.POINTER(LL), ctypes.POINTER(LL),
                                          ctypes.POINTER(I)]
        lib.cdmt_workspace_size.argtypes = [P, I, ctypes.POINTER(Z)]
        lib.cdmt_forward.argtypes = [P, P, Z, P, I, P]
        lib.cdmt_dedisperse_spectra.argtypes = [P, P, Z, I, ctypes.POINTER(D), I, P, P]
        lib.cdmt_dedisperse.argtypes = [P, P, Z, P, I, ctypes.POINTER(D), I, P, P]
        lib.cdmt_destroy.argtypes = [P]
        lib.cdmt_destroy.restype = None
        lib.cdmt_status_string.argtypes = [I]
        lib.cdmt_status_string.restype = ctypes.c_char_p
        F = ctypes.c_float
        lib.cdmt_redigitise_workspace_size.argtypes = [I, LL, I, ctypes.POINTER(Z)]
        lib.cdmt_redigitise.argtypes = [P, I, LL, I, F, F, P, Z, P, P, P, P]
        lib.cdmt_gradient_workspace_size.argtypes = [P, I, I, ctypes.POINTER(Z)]
        lib.cdmt_dm_gradient.argtypes = [P, P, Z, I, ctypes.POINTER(D), I, P, P, Z, P, P]
        lib.cdmt_dm_gradient_noalloc.argtypes = [P, P, Z, I, ctypes.POINTER(D), I, P, P, P]
        lib.cdmt_noalloc_scratch_bytes.argtypes = []
        lib.cdmt_noalloc_scratch_bytes.restype = Z
        lib.cdmt_voltage_gradient_workspace_size.argtypes = [P, I, ctypes.POINTER(Z)]
        lib.cdmt_voltage_gradient.argtypes = [P, P, Z, I, D, P, P, Z, P, I, P]
        lib.cdmt_incoherent_shape.argtypes = [P, I, ctypes.POINTER(D), I, D, D, I,
                                              ctypes.POINTER(LL)]
        lib.cdmt_incoherent_workspace_size.argtypes = [P, I, I, I, ctypes.POINTER(Z)]
        lib.cdmt_incoherent.argtypes = [P, I, P, ctypes.POINTER(D), I, D, D, I, P, Z, P, P]
        BP = ctypes.POINTER(Beam)
        lib.cdmt_batch_workspace_size.argtypes = [BP, I, ctypes.POINTER(Z)]
        lib.cdmt_batch_create.argtypes = [ctypes.POINTER(P), BP, I, P, Z]
        lib.cdmt_batch_set.argtypes = [P, I, I]
        lib.cdmt_batch_get.argtypes = [P, I, ctypes.POINTER(LL)]
        lib.cdmt_batch_run.argtypes = [P, P]
        lib.cdmt_batch_run_graph.argtypes = [P, P]
        lib.cdmt_batch_autotune.argtypes = [P, P, I, ctypes.POINTER(F)]
        lib.cdmt_batch_beam_set.argtypes = [P, I, I, I]
        lib.cdmt_batch_beam_get.argtypes = [P, I, I, ctypes.POINTER(I)]
        lib.cdmt_batch_destroy.argtypes = [P]
        lib.cdmt_batch_destroy.restype = None
        for name in EXPORTS:
            if not hasattr(lib, name):
                raise RuntimeError(f"{LIB_PATH} does not export {name}")
        _lib = lib
        return lib


def _check(status: int, where: str) -> None:
    if status != CDMT_OK:
        raise CdmtError(status, where)


def cdmt_status_string(status: int) -> str:
    return load().cdmt_status_string(int(status)).decode()


# -------------------------------------------------------------- C names ----

def cdmt_plan(nsub, f_centre_mhz, bw_sub_mhz, nfft, noverlap, nchan, ndec) -> int:
    h = ctypes.c_void_p()
    _check(load().cdmt_plan(ctypes.byref(h), nsub, f_centre_mhz, bw_sub_mhz, nfft, noverlap,
                            nchan, ndec), "cdmt_plan")
    return h.value


def cdmt_plan_set(plan, opt, value) -> None:
    _check(load().cdmt_plan_set(plan, opt, value), "cdmt_plan_set")


def cdmt_plan_get(plan, opt) -> int:
    v = ctypes.c_int()
    _check(load().cdmt_plan_get(plan, opt, ctypes.byref(v)), "cdmt_plan_get")
    return v.value


def cdmt_noverlap_for(f_lo_mhz, bw_sub_mhz, dm_max, nchan, ndec, chirp_ref=CHIRP_CHANNEL) -> int:
    v = ctypes.c_int()
    _check(load().cdmt_noverlap_for(f_lo_mhz, bw_sub_mhz, dm_max, nchan, ndec, chirp_ref,
                                    ctypes.byref(v)), "cdmt_noverlap_for")
    return v.value


def cdmt_dm_limit(plan) -> float:
    v = ctypes.c_double()
    _check(load().cdmt_dm_limit(plan, ctypes.byref(v)), "cdmt_dm_limit")
    return v.value


def cdmt_output_shape(plan, nblock):
    a, b, c = ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_int()
    _check(load().cdmt_output_shape(plan, nblock, ctypes.byref(a), ctypes.byref(b),
                                    ctypes.byref(c)), "cdmt_output_shape")
    return a.value, b.value, c.value


def cdmt_workspace_size(plan, nblock) -> int:
    v = ctypes.c_size_t()
    _check(load().cdmt_workspace_size(plan, nblock, ctypes.byref(v)), "cdmt_workspace_size")
    return v.value


def _dm_array(dms):
    dms = [float(d) for d in dms]
    return (ctypes.c_double * max(1, len(dms)))(*dms), len(dms)


# Spectra generation per workspace (keyed by its device address): bumped by
# every call that rewrites the spectra, so that a backward pass can tell
# whether the spectra its forward pass used are still in the workspace.
_ws_generation: dict = {}


def _ptr(v) -> int:
    return int(v.value if isinstance(v, ctypes.c_void_p) else v or 0)


def _bump(workspace) -> None:
    k = _ptr(workspace)
    _ws_generation[k] = _ws_generation.get(k, 0) + 1


def workspace_generation(workspace) -> int:
    """How many times the spectra in this workspace (tensor or address) have
    been rewritten through this binding."""
    return _ws_generation.get(_ptr(workspace.data_ptr() if hasattr(workspace, "data_ptr")
                                   else workspace), 0)


def cdmt_forward(plan, workspace, ws_bytes, voltages, nblock, stream) -> None:
    _bump(workspace)
    _check(load().cdmt_forward(plan, workspace, ws_bytes, voltages, nblock, stream),
           "cdmt_forward")


def cdmt_dedisperse_spectra(plan, workspace, ws_bytes, nblock, dms, out, stream) -> None:
    arr, n = _dm_array(dms)
    _check(load().cdmt_dedisperse_spectra(plan, workspace, ws_bytes, nblock, arr, n, out, stream),
           "cdmt_dedisperse_spectra")


def cdmt_dedisperse(plan, workspace, ws_bytes, voltages, nblock, dms, out, stream) -> None:
    arr, n = _dm_array(dms)
    _bump(workspace)
    _check(load().cdmt_dedisperse(plan, workspace, ws_bytes, voltages, nblock, arr, n, out,
                                  stream), "cdmt_dedisperse")


def cdmt_destroy(plan) -> None:
    if plan:
        load().cdmt_destroy(plan)


def cdmt_redigitise_workspace_size(ndm, ntime, nchan) -> int:
    v = ctypes.c_size_t()
    _check(load().cdmt_redigitise_workspace_size(ndm, ntime, nchan, ctypes.byref(v)),
           "cdmt_redigitise_workspace_size")
    return v.value


def cdmt_redigitise(filterbank, ndm, ntime, nchan, zero, counts_per_sigma, workspace, ws_bytes,
                    codes, mean, scale, stream) -> None:
    _check(load().cdmt_redigitise(filterbank, ndm, ntime, nchan, zero, counts_per_sigma,
                                  workspace, ws_bytes, codes, mean, scale, stream),
           "cdmt_redigitise")


def redigitise(fb, zero=64.0, counts_per_sigma=16.0, workspace=None, stream=None):
    """8-bit codes of a device filterbank fb [ndm][ntime][nchan] float32:
    returns (codes uint8, mean float32 [ndm][nchan], scale float32 [ndm][nchan])."""
    import torch
    if fb.dtype != torch.float32 or not fb.is_cuda or not fb.is_contiguous() or fb.dim() != 3:
        raise ValueError("filterbank must be a contiguous float32 [ndm][ntime][nchan] device tensor")
    ndm, ntime, nchan = (int(v) for v in fb.shape)
    codes = torch.empty(fb.shape, dtype=torch.uint8, device=fb.device)
    mean = torch.empty((ndm, nchan), dtype=torch.float32, device=fb.device)
    scale = torch.empty((ndm, nchan), dtype=torch.float32, device=fb.device)
    if ndm == 0:
        return codes, mean, scale
    if workspace is None:
        workspace = torch.empty(max(1, cdmt_redigitise_workspace_size(ndm, ntime, nchan)),
                                dtype=torch.uint8, device=fb.device)
    s = stream if stream is not None else torch.cuda.current_stream()
    cdmt_redigitise(ctypes.c_void_p(fb.data_ptr()), ndm, ntime, nchan, float(zero),
                    float(counts_per_sigma), ctypes.c_void_p(workspace.data_ptr()),
                    workspace.numel(), ctypes.c_void_p(codes.data_ptr()),
                    ctypes.c_void_p(mean.data_ptr()), ctypes.c_void_p(scale.data_ptr()),
                    ctypes.c_void_p(s.cuda_stream))
    return codes, mean, scale


def cdmt_gradient_workspace_size(plan, nblock, ndm) -> int:
    v = ctypes.c_size_t()
    _check(load().cdmt_gradient_workspace_size(plan, nblock, ndm, ctypes.byref(v)),
           "cdmt_gradient_workspace_size")
    return v.value


def cdmt_dm_gradient(plan, workspace, ws_bytes, nblock, dms, grad_out, gws, gws_bytes, dldm,
                     stream) -> None:
    arr, n = _dm_array(dms)
    _check(load().cdmt_dm_gradient(plan, workspace, ws_bytes, nblock, arr, n, grad_out, gws,
                                   gws_bytes, dldm, stream), "cdmt_dm_gradient")


def cdmt_dm_gradient_noalloc(plan, workspace, ws_bytes, nblock, dms, grad_out, dldm,
                             stream) -> None:
    arr, n = _dm_array(dms)
    _check(load().cdmt_dm_gradient_noalloc(plan, workspace, ws_bytes, nblock, arr, n, grad_out,
                                           dldm, stream), "cdmt_dm_gradient_noalloc")


def cdmt_noalloc_scratch_bytes() -> int:
    return int(load().cdmt_noalloc_scratch_bytes())


def cdmt_voltage_gradient_workspace_size(plan, nblock) -> int:
    v = ctypes.c_size_t()
    _check(load().cdmt_voltage_gradient_workspace_size(plan, nblock, ctypes.byref(v)),
           "cdmt_voltage_gradient_workspace_size")
    return v.value


def cdmt_voltage_gradient(plan, workspace, ws_bytes, nblock, dm, grad_out, gws, gws_bytes,
                          grad_v, accumulate, stream) -> None:
    _check(load().cdmt_voltage_gradient(plan, workspace, ws_bytes, nblock, float(dm), grad_out,
                                        gws, gws_bytes, grad_v, int(accumulate), stream),
           "cdmt_voltage_gradient")


def cdmt_incoherent_shape(plan, nblock, dm_coh, ddm0, ddm, ntrial) -> int:
    arr, n = _dm_array(dm_coh)
    v = ctypes.c_longlong()
    _check(load().cdmt_incoherent_shape(plan, nblock, arr, n, float(ddm0), float(ddm), ntrial,
                                        ctypes.byref(v)), "cdmt_incoherent_shape")
    return v.value


def cdmt_incoherent_workspace_size(plan, nblock, ndm, ntrial) -> int:
    v = ctypes.c_size_t()
    _check(load().cdmt_incoherent_workspace_size(plan, nblock, ndm, ntrial, ctypes.byref(v)),
           "cdmt_incoherent_workspace_size")
    return v.value


def cdmt_incoherent(plan, nblock, fb, dm_coh, ddm0, ddm, ntrial, workspace, ws_bytes, out,
                    stream) -> None:
    arr, n = _dm_array(dm_coh)
    _check(load().cdmt_incoherent(plan, nblock, fb, arr, n, float(ddm0), float(ddm), ntrial,
                                  workspace, ws_bytes, out, stream), "cdmt_incoherent")


_N_OPTIONS = 11


def _snapshot(plan, workspace):
    """What a backward pass depends on besides its inputs: the spectra in the
    workspace (their generation) and every plan option."""
    return (workspace_generation(workspace),
            tuple(cdmt_plan_get(plan.handle, o) for o in range(_N_OPTIONS)))


def _check_snapshot(ctx) -> None:
    gen, opts = _snapshot(ctx.plan, ctx.ws)
    if gen != ctx.state[0]:
        raise RuntimeError("the workspace's spectra were rewritten (another forward or "
                           "dedisperse call on it) after this graph's forward pass; run "
                           "backward first or give each forward pass its own workspace")
    if opts != ctx.state[1]:
        raise RuntimeError("a plan option changed between this graph's forward and "
                           "backward passes")


def _dm_stage_function():
    import torch

    class DMStage(torch.autograd.Function):
        """F = the DM stage of Alg. 1 at the (continuous) trial DMs in a tensor;
        backward returns dL/dDM through cdmt_dm_gradient.  The spectra must
        already be in the workspace (Plan.forward) and the plan should use the
        exact transfer function (chirp_exact=1), the form the gradient is of."""

        @staticmethod
        def forward(ctx, dms, plan, nblock, workspace):
            dm_list = [float(v) for v in dms.detach().cpu().tolist()]
            out = torch.empty(plan.out_shape(len(dm_list), nblock), dtype=torch.float32,
                              device=workspace.device)
            plan.dedisperse_spectra(nblock, dm_list, out, workspace)
            ctx.plan, ctx.nblock, ctx.ws, ctx.dm_list = plan, nblock, workspace, dm_list
            ctx.dms_device, ctx.dms_dtype = dms.device, dms.dtype
            ctx.state = _snapshot(plan, workspace)
            return out

        @staticmethod
        def backward(ctx, grad_out):
            _check_snapshot(ctx)
            g = grad_out.detach().to(torch.float32).contiguous()
            n = len(ctx.dm_list)
            dldm = torch.empty(n, dtype=torch.float64, device=g.device)
            gsz = cdmt_gradient_workspace_size(ctx.plan.handle, ctx.nblock, n)
            gws = torch.empty(max(1, gsz), dtype=torch.uint8, device=g.device)
            cdmt_dm_gradient(ctx.plan.handle, ctypes.c_void_p(ctx.ws.data_ptr()), ctx.ws.numel(),
                             ctx.nblock, ctx.dm_list, ctypes.c_void_p(g.data_ptr()),
                             ctypes.c_void_p(gws.data_ptr()), gws.numel(),
                             ctypes.c_void_p(dldm.data_ptr()),
                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
            return dldm.to(ctx.dms_device, ctx.dms_dtype), None, None, None

    class Dedisperse(torch.autograd.Function):
        """F = the whole path of Alg. 1 (forward stage and DM stage) for complex
        float32 voltages x and trial DMs dms; backward gives dL/dx (through
        cdmt_voltage_gradient, one call per DM, accumulated) and dL/dDM."""

        @staticmethod
        def forward(ctx, x, dms, plan, nblock, workspace):
            dm_list = [float(v) for v in dms.detach().cpu().tolist()]
            plan.forward(x.detach(), nblock, workspace)
            out = torch.empty(plan.out_shape(len(dm_list), nblock), dtype=torch.float32,
                              device=x.device)
            plan.dedisperse_spectra(nblock, dm_list, out, workspace)
            ctx.plan, ctx.nblock, ctx.ws, ctx.dm_list = plan, nblock, workspace, dm_list
            ctx.dms_device, ctx.dms_dtype = dms.device, dms.dtype
            ctx.x_shape = x.shape
            ctx.state = _snapshot(plan, workspace)
            return out

        @staticmethod
        def backward(ctx, grad_out):
            _check_snapshot(ctx)
            g = grad_out.detach().to(torch.float32).contiguous()
            plan, nblock, ws = ctx.plan, ctx.nblock, ctx.ws
            stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
            gx = gdm = None
            if ctx.needs_input_grad[0]:
                gx = torch.empty(ctx.x_shape, dtype=torch.float32, device=g.device)
                gsz = cdmt_voltage_gradient_workspace_size(plan.handle, nblock)
                gws = torch.empty(max(1, gsz), dtype=torch.uint8, device=g.device)
                for i, dm in enumerate(ctx.dm_list):
                    cdmt_voltage_gradient(plan.handle, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                          nblock, dm, ctypes.c_void_p(g[i].data_ptr()),
                                          ctypes.c_void_p(gws.data_ptr()), gws.numel(),
                                          ctypes.c_void_p(gx.data_ptr()), 1 if i else 0, stream)
            if ctx.needs_input_grad[1]:
                n = len(ctx.dm_list)
                dldm = torch.empty(n, dtype=torch.float64, device=g.device)
                gsz = cdmt_gradient_workspace_size(plan.handle, nblock, n)
                gws = torch.empty(max(1, gsz), dtype=torch.uint8, device=g.device)
                cdmt_dm_gradient(plan.handle, ctypes.c_void_p(ws.data_ptr()), ws.numel(), nblock,
                                 ctx.dm_list, ctypes.c_void_p(g.data_ptr()),
                                 ctypes.c_void_p(gws.data_ptr()), gws.numel(),
                                 ctypes.c_void_p(dldm.data_ptr()), stream)
                gdm = dldm.to(ctx.dms_device, ctx.dms_dtype)
            return gx, gdm, None, None, None

    return DMStage, Dedisperse


def dedisperse(plan, x, dms, nblock, workspace):
    """Differentiable path: filterbank of complex float32 voltages x
    [nsub][ntime_in][2][2] at the DMs of the tensor dms; dL/dx and dL/dDM by
    backward."""
    global _DMStage, _Dedisperse
    if _DMStage is None:
        _DMStage, _Dedisperse = _dm_stage_function()
    return _Dedisperse.apply(x, dms, plan, nblock, workspace)


def dedisperse_dm(plan, dms, nblock, workspace):
    """Differentiable DM stage: filterbank [ndm][ntime_out][nchan_out] at the DMs
    of the tensor dms (requires_grad for dL/dDM)."""
    global _DMStage, _Dedisperse
    if _DMStage is None:
        _DMStage, _Dedisperse = _dm_stage_function()
    return _DMStage.apply(dms, plan, nblock, workspace)


_DMStage = None
_Dedisperse = None


def cdmt_batch_workspace_size(beams, nbeam) -> int:
    v = ctypes.c_size_t()
    _check(load().cdmt_batch_workspace_size(beams, nbeam, ctypes.byref(v)),
           "cdmt_batch_workspace_size")
    return v.value


def cdmt_batch_create(beams, nbeam, workspace, ws_bytes) -> int:
    h = ctypes.c_void_p()
    _check(load().cdmt_batch_create(ctypes.byref(h), beams, nbeam, workspace, ws_bytes),
           "cdmt_batch_create")
    return h.value


def cdmt_batch_set(batch, opt, value) -> None:
    _check(load().cdmt_batch_set(batch, opt, value), "cdmt_batch_set")


def cdmt_batch_get(batch, opt) -> int:
    v = ctypes.c_longlong()
    _check(load().cdmt_batch_get(batch, opt, ctypes.byref(v)), "cdmt_batch_get")
    return v.value


def cdmt_batch_run(batch, stream) -> None:
    _check(load().cdmt_batch_run(batch, stream), "cdmt_batch_run")


def cdmt_batch_run_graph(batch, stream) -> None:
    _check(load().cdmt_batch_run_graph(batch, stream), "cdmt_batch_run_graph")


def cdmt_batch_autotune(batch, stream, reps) -> float:
    v = ctypes.c_float()
    _check(load().cdmt_batch_autotune(batch, stream, reps, ctypes.byref(v)),
           "cdmt_batch_autotune")
    return v.value


def cdmt_batch_destroy(batch) -> None:
    if batch:
        load().cdmt_batch_destroy(batch)


class Batch:
    """Several beams (Plan, nblock, device voltages, DM list, device output)
    run as one batch; torch supplies the workspace and the streams."""

    def __init__(self, beams, device="cuda"):
        import torch
        load()
        self._keep = []
        arr = (Beam * len(beams))()
        for i, (plan, nblock, x, dms, out) in enumerate(beams):
            plan._check_voltages(x, nblock)
            want = plan.out_shape(len(dms), nblock)
            if (out.dtype != torch.float32 or not out.is_cuda or not out.is_contiguous()
                    or tuple(out.shape) != want):
                raise ValueError(f"beam {i}: output must be a contiguous float32 "
                                 f"{want} device tensor")
            d, n = _dm_array(dms)
            arr[i] = Beam(plan.handle, nblock, x.data_ptr(), d, n, out.data_ptr())
            self._keep += [plan, x, out, d]
        n = cdmt_batch_workspace_size(arr, len(beams))
        self.workspace = torch.empty(max(1, n), dtype=torch.uint8, device=device)
        self.handle = cdmt_batch_create(arr, len(beams), ctypes.c_void_p(self.workspace.data_ptr()),
                                        self.workspace.numel())

    def __del__(self):
        try:
            cdmt_batch_destroy(self.handle)
        except Exception:
            pass

    @staticmethod
    def _stream(stream):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        return ctypes.c_void_p(s.cuda_stream)

    def set(self, opt, value):
        cdmt_batch_set(self.handle, opt, value)

    def get(self, opt):
        return cdmt_batch_get(self.handle, opt)

    def run(self, stream=None):
        cdmt_batch_run(self.handle, self._stream(stream))

    def run_graph(self, stream):
        cdmt_batch_run_graph(self.handle, self._stream(stream))

    def autotune(self, stream=None, reps=2):
        return cdmt_batch_autotune(self.handle, self._stream(stream), reps)

    def beam_set(self, beam, opt, value):
        _check(load().cdmt_batch_beam_set(self.handle, beam, opt, value), "cdmt_batch_beam_set")

    def beam_get(self, beam, opt):
        v = ctypes.c_int()
        _check(load().cdmt_batch_beam_get(self.handle, beam, opt, ctypes.byref(v)),
               "cdmt_batch_beam_get")
        return v.value


# ------------------------------------------------- torch-facing wrapper ----

class Plan:
    """Owns a cdmt plan; torch supplies the device memory and the stream."""

    def __init__(self, nsub, f_centre_mhz, bw_sub_mhz, nfft, noverlap, nchan, ndec, *,
                 input_kind=INPUT_CF32, chirp_ref=CHIRP_CHANNEL, sign=-1, dm_tile=None,
                 chirp_exact=None, lane_bins=None, fwd_n2=None, out_layout=None,
                 dm_check=None, fft_schedule=None):
        self.handle = cdmt_plan(nsub, f_centre_mhz, bw_sub_mhz, nfft, noverlap, nchan, ndec)
        self.nsub, self.nfft, self.noverlap, self.nchan, self.ndec = \
            nsub, nfft, noverlap, nchan, ndec
        cdmt_plan_set(self.handle, CDMT_OPT_INPUT, input_kind)
        cdmt_plan_set(self.handle, CDMT_OPT_CHIRP_REF, chirp_ref)
        cdmt_plan_set(self.handle, CDMT_OPT_SIGN, sign)
        if dm_tile is not None:
            cdmt_plan_set(self.handle, CDMT_OPT_DM_TILE, dm_tile)
        if chirp_exact is not None:
            cdmt_plan_set(self.handle, CDMT_OPT_CHIRP_EXACT, int(chirp_exact))
        if lane_bins is not None:
            cdmt_plan_set(self.handle, CDMT_OPT_LANE_BINS, int(lane_bins))
        if fwd_n2 is not None:
            cdmt_plan_set(self.handle, CDMT_OPT_FWD_N2, int(fwd_n2))
        if out_layout is not None:
            cdmt_plan_set(self.handle, CDMT_OPT_OUT_LAYOUT, int(out_layout))
        if dm_check is not None:
            cdmt_plan_set(self.handle, CDMT_OPT_DM_CHECK, int(dm_check))
        if fft_schedule is not None:
            cdmt_plan_set(self.handle, CDMT_OPT_FFT_SCHEDULE, int(fft_schedule))
        self.input_kind = input_kind

    def __del__(self):
        try:
            cdmt_destroy(self.handle)
        except Exception:
            pass

    def shape(self, nblock):
        return cdmt_output_shape(self.handle, nblock)

    def out_shape(self, ndm, nblock):
        """Filterbank tensor shape for ndm DMs: (ndm, ntime_out, nch) or, with
        the channel-major layout, (ndm, nch, ntime_out)."""
        _, ntout, nch = self.shape(nblock)
        layout = cdmt_plan_get(self.handle, CDMT_OPT_OUT_LAYOUT)
        return (ndm, nch, ntout) if layout == LAYOUT_CHANNEL_MAJOR else (ndm, ntout, nch)

    def dm_limit(self) -> float:
        """Largest |DM| the plan's overlap supports (Eq. 2)."""
        return cdmt_dm_limit(self.handle)

    def _check_out(self, out, ndm, nblock, device):
        """The C call takes no output size: require exactly the filterbank
        tensor it writes, before any launch."""
        import torch
        want = self.out_shape(ndm, nblock)
        if (not isinstance(out, torch.Tensor) or out.dtype != torch.float32
                or not out.is_contiguous() or tuple(out.shape) != want):
            raise ValueError(f"out must be a contiguous float32 tensor of shape {want}")
        if not out.is_cuda or (device is not None and out.device != torch.device(device)):
            raise ValueError(f"out must be on the device of the workspace ({device})")

    @staticmethod
    def _check_workspace(workspace):
        """A contiguous byte tensor on the device (its size is checked by
        the library, which reports CDMT_E_WORKSPACE)."""
        import torch
        if (not isinstance(workspace, torch.Tensor) or workspace.element_size() != 1
                or not workspace.is_contiguous()):
            raise ValueError("workspace must be a contiguous byte tensor")
        if not workspace.is_cuda:
            raise ValueError("workspace must be a device tensor")

    def workspace(self, nblock, device="cuda"):
        import torch
        n = cdmt_workspace_size(self.handle, nblock)
        return torch.empty(max(n, 1), dtype=torch.uint8, device=device)

    def _stream(self, stream):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        return ctypes.c_void_p(s.cuda_stream)

    def _check_voltages(self, x, nblock):
        import torch
        want = torch.int8 if self.input_kind == INPUT_CI8 else torch.float32
        ntin, _, _ = self.shape(nblock)
        if x.dtype != want or not x.is_cuda or not x.is_contiguous():
            raise ValueError(f"voltages must be a contiguous {want} device tensor")
        if tuple(x.shape) != (self.nsub, ntin, 2, 2):
            raise ValueError(f"voltages shape {tuple(x.shape)} != {(self.nsub, ntin, 2, 2)}")

    def dedisperse(self, x, nblock, dms, out=None, workspace=None, stream=None):
        """Filterbank [ndm][ntime_out][nsub*nchan] float32 for device voltages
        x [nsub][ntime_in][2][2] (float32 or int8)."""
        import torch
        self._check_voltages(x, nblock)
        if out is None:
            out = torch.empty(self.out_shape(len(dms), nblock), dtype=torch.float32,
                              device=x.device)
        if workspace is None:
            workspace = self.workspace(nblock, x.device)
        self._check_workspace(workspace)
        self._check_out(out, len(dms), nblock, workspace.device)
        cdmt_dedisperse(self.handle, ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                        ctypes.c_void_p(x.data_ptr()), nblock, dms,
                        ctypes.c_void_p(out.data_ptr()), self._stream(stream))
        return out

    def forward(self, x, nblock, workspace, stream=None):
        self._check_voltages(x, nblock)
        self._check_workspace(workspace)
        cdmt_forward(self.handle, ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                     ctypes.c_void_p(x.data_ptr()), nblock, self._stream(stream))

    def dedisperse_spectra(self, nblock, dms, out, workspace, stream=None):
        self._check_out(out, len(dms), nblock,
                        workspace.device if hasattr(workspace, "device") else None)
        self._check_workspace(workspace)
        cdmt_dedisperse_spectra(self.handle, ctypes.c_void_p(workspace.data_ptr()),
                                workspace.numel(), nblock, dms, ctypes.c_void_p(out.data_ptr()),
                                self._stream(stream))
        return out


def incoherent(plan, fb, nblock, dm_coh, ddm0, ddm, ntrial, out=None, workspace=None,
               stream=None):
    """Semi-coherent search's incoherent stage: the device filterbanks fb
    [ndm][ntime][nsub*nchan] float32 (one per coherent DM in dm_coh) summed
    over channels at the delays of DM dm_coh[d] + ddm0 + k ddm; returns
    out [ndm][ntrial][nout] float32."""
    import torch
    ndm = len(dm_coh)
    want = plan.out_shape(ndm, nblock)
    if (fb.dtype != torch.float32 or not fb.is_cuda or not fb.is_contiguous()
            or tuple(fb.shape) != want):
        raise ValueError(f"fb must be a contiguous float32 device tensor {want}")
    nout = cdmt_incoherent_shape(plan.handle, nblock, dm_coh, ddm0, ddm, ntrial)
    if out is None:
        out = torch.empty((ndm, ntrial, nout), dtype=torch.float32, device=fb.device)
    elif (out.dtype != torch.float32 or not out.is_cuda or not out.is_contiguous()
          or tuple(out.shape) != (ndm, ntrial, nout)):
        raise ValueError(f"out must be a contiguous float32 device tensor {(ndm, ntrial, nout)}")
    if workspace is None:
        workspace = torch.empty(max(1, cdmt_incoherent_workspace_size(plan.handle, nblock, ndm,
                                                                      ntrial)),
                                dtype=torch.uint8, device=fb.device)
    cdmt_incoherent(plan.handle, nblock, ctypes.c_void_p(fb.data_ptr()), dm_coh, ddm0, ddm,
                    ntrial, ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                    ctypes.c_void_p(out.data_ptr()), plan._stream(stream))
    return out


def dm_seconds(nblock: int, nfft: int, noverlap: int, bw_mhz: float) -> float:
    """Seconds of data covered by nblock blocks (the metric's data-seconds)."""
    return nblock * (nfft - noverlap) / (bw_mhz * 1e6)


__all__ = [n for n in dir() if n.startswith("cdmt_")] + ["Plan", "load", "CdmtError",
                                                          "dm_seconds", "redigitise", "Batch", "workspace_generation",
                                                          "Beam", "dedisperse_dm", "dedisperse",
                                                          "incoherent", "EXPORTS"]
