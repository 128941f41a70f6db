// Host side of the C ABI that needs no GPU: plan creation and options, the
// size helpers of Sec. 2-3 and the validation of calls, including the Eq. 2
// check of a DM list against the plan's overlap.  Plain C++ (no HIP headers),
// built into libcdmt.so with the kernels and, for the host sanitizers, on its
// own.
#include <cmath>
#include <new>

#include "plan.hpp"

namespace cdmt {

bool is_pow2(long long v) { return v > 0 && (v & (v - 1)) == 0; }

int ilog2(long long v) {
    int l = 0;
    while ((1LL << l) < v)
        ++l;
    return l;
}

bool fwd_split_ok(int nfft, int n2) {
    return (n2 == 64 || n2 == 128 || n2 == 256) && nfft % n2 == 0 && nfft / n2 >= 64 &&
           nfft / n2 <= 512;
}

double max_half_cycles_per_dm(const cdmt_plan_s *p) {
    // Eq. 1 at the largest offset from nu0 in the lowest subband
    const double f_lo = p->f_centre - p->nsub * p->bw / 2;
    const double half = p->chirp_ref == 0 ? p->bw / (2.0 * p->nchan) : p->bw / 2;
    const double nu0 = f_lo + half;
    return 2.0 * 1e6 * kKdm * half * half / (nu0 * nu0 * f_lo);
}

double dm_limit(const cdmt_plan_s *p) {
    // Sec. 2: sections overlap by at least n_d n_c = r t_d samples, t_d from
    // Eq. 2 over the lowest channel (the band the transfer function of one
    // channel spans) or, with nu0 per subband, over the lowest subband;
    // r = bw in samples per second.
    const double f_lo = p->f_centre - p->nsub * p->bw / 2;
    const double f_hi = f_lo + (p->chirp_ref == 0 ? p->bw / p->nchan : p->bw);
    const double samples_per_dm = p->bw * 1e6 * kKdm * (1.0 / (f_lo * f_lo) - 1.0 / (f_hi * f_hi));
    if (!(samples_per_dm > 0))
        return HUGE_VAL;          // no measurable sweep (the band is too high)
    return (double)p->noverlap / samples_per_dm;
}

int check_dms(const cdmt_plan_s *p, const double *dm, int n) {
    const double bound = max_half_cycles_per_dm(p);
    // a relative slack of 1e-12 keeps the DM that cdmt_noverlap_for sized
    // the overlap for on the accepted side
    const double lim = dm_limit(p) * (1.0 + 1e-12);
    for (int i = 0; i < n; ++i) {
        if (!std::isfinite(dm[i]) || std::fabs(dm[i]) * bound >= 1073741824.0)
            return CDMT_E_ARG;
        if (p->dm_check && std::fabs(dm[i]) > lim)
            return CDMT_E_SHAPE;
    }
    return CDMT_OK;
}

bool arithmetic(const double *dm, int n, double tol) {
    const double step = dm[1] - dm[0];
    if (step == 0.0)
        return false;
    for (int i = 2; i < n; ++i)
        if (std::fabs(dm[i] - (dm[0] + i * step)) > tol)
            return false;
    return true;
}

int workspace_bytes(const cdmt_plan_s *p, int nblock, size_t *bytes) {
    if (nblock < 0)
        return CDMT_E_ARG;
    // 16 bytes per bin (both polarisations), spectra and intermediate
    const unsigned long long n = (unsigned long long)nblock * p->nsub * p->nfft;
    *bytes = (size_t)(2ULL * n * 16ULL);
    return CDMT_OK;
}

int check_call(const cdmt_plan_s *p, void *ws, size_t ws_bytes, int nblock) {
    if (!p)
        return CDMT_E_ARG;
    if (nblock < 0)
        return CDMT_E_ARG;
    size_t need = 0;
    workspace_bytes(p, nblock, &need);
    if (nblock > 0 && (!ws || ws_bytes < need))
        return ws ? CDMT_E_WORKSPACE : CDMT_E_ARG;
    const long long chunks = (long long)nblock * p->nsub * p->nchan;
    if (chunks > 0x7fffffffLL)
        return CDMT_E_SHAPE;
    return CDMT_OK;
}

long long grad_groups(const cdmt_plan_s *p, int nblock) {
    const int C = 4096 / p->m;
    return ((long long)nblock * p->nsub * p->nchan + C - 1) / C;
}

}  // namespace cdmt

using namespace cdmt;

extern "C" {

int cdmt_plan(cdmt_plan_t *out, int nsub, double f_centre_mhz, double bw_sub_mhz, int nfft,
              int noverlap, int nchan, int ndec) {
    if (!out)
        return CDMT_E_ARG;
    *out = nullptr;
    if (!std::isfinite(f_centre_mhz) || !std::isfinite(bw_sub_mhz))
        return CDMT_E_ARG;
    if (nsub < 1 || !is_pow2(nfft) || nfft < 2 || !is_pow2(nchan) || nfft % nchan)
        return CDMT_E_SHAPE;
    if (noverlap < 0 || noverlap >= nfft || noverlap % (2LL * nchan))
        return CDMT_E_SHAPE;
    const int m = nfft / nchan, nd = noverlap / nchan;
    if (ndec < 1 || (m - nd) % ndec)
        return CDMT_E_SHAPE;
    if (!(bw_sub_mhz > 0) || !(f_centre_mhz - nsub * bw_sub_mhz / 2 > 0))
        return CDMT_E_SHAPE;
    if (nfft < 1024 || nfft > (1 << 17) || m < 64 || m > 8192)
        return CDMT_E_UNSUPPORTED;
    cdmt_plan_s *p = new (std::nothrow) cdmt_plan_s;
    if (!p)
        return CDMT_E_ARG;
    p->nsub = nsub;
    p->nfft = nfft;
    p->noverlap = noverlap;
    p->nchan = nchan;
    p->ndec = ndec;
    p->f_centre = f_centre_mhz;
    p->bw = bw_sub_mhz;
    p->m = m;
    p->nd = nd;
    p->tblk = (m - nd) / ndec;
    if (nfft >= 4096) {
        const int l = ilog2(nfft);
        p->n2 = 1 << (l / 2);
        p->n1 = nfft / p->n2;
    } else {
        p->n2 = 1;            // one pass: the whole transform in one workgroup
        p->n1 = nfft;
    }
    *out = p;
    return CDMT_OK;
}

int cdmt_plan_set(cdmt_plan_t p, int opt, int value) {
    if (!p)
        return CDMT_E_ARG;
    switch (opt) {
    case CDMT_OPT_INPUT:
        if (value != 0 && value != 1)
            return CDMT_E_ARG;
        p->input_kind = value;
        return CDMT_OK;
    case CDMT_OPT_CHIRP_REF:
        if (value != 0 && value != 1)
            return CDMT_E_ARG;
        p->chirp_ref = value;
        return CDMT_OK;
    case CDMT_OPT_SIGN:
        if (value != 1 && value != -1)
            return CDMT_E_ARG;
        p->sign = value;
        return CDMT_OK;
    case CDMT_OPT_PRECISION:
        if (value < 0 || value > 2)
            return CDMT_E_ARG;
        if (value != 0 && p->m != 4096)
            return CDMT_E_UNSUPPORTED;
        p->precision = value;
        return CDMT_OK;
    case CDMT_OPT_DM_TILE:
        if (value < 1 || value > 64)
            return CDMT_E_ARG;
        p->dm_tile = value;
        return CDMT_OK;
    case CDMT_OPT_CHIRP_EXACT:
        if (value != 0 && value != 1)
            return CDMT_E_ARG;
        p->chirp_exact = value;
        return CDMT_OK;
    case CDMT_OPT_LANE_BINS:
        if (value != 8 && value != 16)
            return CDMT_E_ARG;
        p->lane_bins = value;
        return CDMT_OK;
    case CDMT_OPT_FWD_N2:
        if (!fwd_split_ok(p->nfft, value))
            return CDMT_E_ARG;
        p->n2 = value;
        p->n1 = p->nfft / value;
        return CDMT_OK;
    case CDMT_OPT_OUT_LAYOUT:
        if (value != 0 && value != 1)
            return CDMT_E_ARG;
        p->out_layout = value;
        return CDMT_OK;
    case CDMT_OPT_DM_CHECK:
        if (value != 0 && value != 1)
            return CDMT_E_ARG;
        p->dm_check = value;
        return CDMT_OK;
    case CDMT_OPT_FFT_SCHEDULE:
        if (value != 0 && value != 1)
            return CDMT_E_ARG;
        p->fft_schedule = value;
        return CDMT_OK;
    default:
        return CDMT_E_ARG;
    }
}

int cdmt_plan_get(cdmt_plan_t p, int opt, int *value) {
    if (!p || !value)
        return CDMT_E_ARG;
    switch (opt) {
    case CDMT_OPT_INPUT: *value = p->input_kind; return CDMT_OK;
    case CDMT_OPT_CHIRP_REF: *value = p->chirp_ref; return CDMT_OK;
    case CDMT_OPT_SIGN: *value = p->sign; return CDMT_OK;
    case CDMT_OPT_PRECISION: *value = p->precision; return CDMT_OK;
    case CDMT_OPT_DM_TILE: *value = p->dm_tile; return CDMT_OK;
    case CDMT_OPT_CHIRP_EXACT: *value = p->chirp_exact; return CDMT_OK;
    case CDMT_OPT_LANE_BINS: *value = p->lane_bins; return CDMT_OK;
    case CDMT_OPT_FWD_N2: *value = p->n2; return CDMT_OK;
    case CDMT_OPT_OUT_LAYOUT: *value = p->out_layout; return CDMT_OK;
    case CDMT_OPT_DM_CHECK: *value = p->dm_check; return CDMT_OK;
    case CDMT_OPT_FFT_SCHEDULE: *value = p->fft_schedule; return CDMT_OK;
    default: return CDMT_E_ARG;
    }
}

int cdmt_noverlap_for(double f_lo_mhz, double bw_sub_mhz, double dm_max, int nchan, int ndec,
                      int chirp_ref, int *noverlap_out) {
    if (!noverlap_out || !std::isfinite(f_lo_mhz) || !std::isfinite(bw_sub_mhz) ||
        !std::isfinite(dm_max))
        return CDMT_E_ARG;
    if (!(f_lo_mhz > 0) || !(bw_sub_mhz > 0) || dm_max < 0 || !is_pow2(nchan) || ndec < 1 ||
        (chirp_ref != 0 && chirp_ref != 1))
        return CDMT_E_ARG;
    // Eq. 2 over the lowest channel (or the lowest subband), then
    // n_d n_c = r t_d subband samples (Sec. 2), r = bw in samples/s
    const double hi = f_lo_mhz + (chirp_ref == 0 ? bw_sub_mhz / nchan : bw_sub_mhz);
    const double td = kKdm * (1.0 / (f_lo_mhz * f_lo_mhz) - 1.0 / (hi * hi)) * dm_max;
    const double need = std::ceil(bw_sub_mhz * 1e6 * td - 1e-9);
    if (!(need < 4e9))
        return CDMT_E_SHAPE;
    const long long unit = 2LL * nchan * ndec;
    const long long nov = ((long long)need + unit - 1) / unit * unit;
    if (nov > 0x7fffffffLL)
        return CDMT_E_SHAPE;
    *noverlap_out = (int)nov;
    return CDMT_OK;
}

int cdmt_dm_limit(cdmt_plan_t p, double *dm_max) {
    if (!p || !dm_max)
        return CDMT_E_ARG;
    *dm_max = dm_limit(p);
    return CDMT_OK;
}

int cdmt_output_shape(cdmt_plan_t p, int nblock, long long *ntime_in, long long *ntime_out,
                      int *nchan_out) {
    if (!p || nblock < 0)
        return CDMT_E_ARG;
    if (ntime_in)
        *ntime_in = (long long)nblock * (p->nfft - p->noverlap) + p->noverlap;
    if (ntime_out)
        *ntime_out = (long long)nblock * p->tblk;
    if (nchan_out)
        *nchan_out = p->nsub * p->nchan;
    return CDMT_OK;
}

int cdmt_workspace_size(cdmt_plan_t p, int nblock, size_t *bytes) {
    if (!p || !bytes)
        return CDMT_E_ARG;
    return workspace_bytes(p, nblock, bytes);
}

int cdmt_gradient_workspace_size(cdmt_plan_t p, int nblock, int ndm, size_t *bytes) {
    if (!p || !bytes || nblock < 0 || ndm < 0)
        return CDMT_E_ARG;
    if (p->m > 4096)
        return CDMT_E_UNSUPPORTED;
    *bytes = (size_t)ndm * (size_t)grad_groups(p, nblock) * sizeof(double);
    return CDMT_OK;
}

int cdmt_voltage_gradient_workspace_size(cdmt_plan_t p, int nblock, size_t *bytes) {
    if (!p || !bytes || nblock < 0)
        return CDMT_E_ARG;
    if (p->m > 4096)
        return CDMT_E_UNSUPPORTED;
    size_t w = 0;
    workspace_bytes(p, nblock, &w);
    *bytes = w / 2 * 3;                  // spectrum gradient + the forward kernels' two buffers
    return CDMT_OK;
}

void cdmt_destroy(cdmt_plan_t p) { delete p; }

const char *cdmt_status_string(int status) {
    switch (status) {
    case CDMT_OK: return "ok";
    case CDMT_E_ARG: return "invalid argument";
    case CDMT_E_SHAPE: return "shape violates the method's constraints";
    case CDMT_E_WORKSPACE: return "workspace too small";
    case CDMT_E_DEVICE: return "HIP device error";
    case CDMT_E_UNSUPPORTED: return "configuration not supported by this library";
    default: return "unknown status";
    }
}

}  // extern "C"
