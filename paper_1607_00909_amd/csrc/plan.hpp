// Internal definitions shared by the library's translation units: the plan
// object behind cdmt_plan_t, the dispersion constant and the host-side
// validation helpers (defined in plan.cpp, which is host-only C++ so that it
// can also be built with the host sanitizers).  Not part of the C ABI.
#pragma once

#include <cstddef>

#include "../../include/cdmt.h"

struct cdmt_plan_s {
    int nsub, nfft, noverlap, nchan, ndec;
    double f_centre, bw;
    int input_kind = 0, chirp_ref = 0, sign = -1, precision = 0, dm_tile = 64, chirp_exact = 0, lane_bins = 16;
    int out_layout = 0;     // 0: filterbanks [DM][t][ch], 1: [DM][ch][t]
    int dm_check = 1;       // 1: reject DMs whose Eq. 2 sweep exceeds the overlap
    int fft_schedule = 0;   // DM-stage transform schedule (CDMT_OPT_FFT_SCHEDULE)
    int m, nd, tblk, n1, n2;
};

namespace cdmt {

// Sec. 2, text after Eq. 1: k_DM^{-1} = 2.41e-4 s MHz^2 (per unit DM).
constexpr double kKdm = 1.0 / 2.41e-4;

bool is_pow2(long long v);
int ilog2(long long v);

// The four-step splits the forward kernels are built for (N2 column
// transforms, N1 = nfft / N2 row transforms); nfft <= 2048 is one pass.
bool fwd_split_ok(int nfft, int n2);

// Upper bound of |phase| in half-cycles per unit DM over every bin of the
// plan; the kernels keep the integer part of the phase in an int.
double max_half_cycles_per_dm(const cdmt_plan_s *p);

// Largest |DM| whose Eq. 2 sweep over the lowest channel (nu0 per channel)
// or the lowest subband (nu0 per subband), in subband samples, fits in the
// plan's overlap (Sec. 2, overlap-save).
double dm_limit(const cdmt_plan_s *p);

// Validation of a DM list against a plan: CDMT_E_ARG for a non-finite value
// or one beyond the phase bound, CDMT_E_SHAPE for one beyond dm_limit (when
// the plan checks it).
int check_dms(const cdmt_plan_s *p, const double *dm, int n);

// True when dm[i] = dm[0] + i (dm[1] - dm[0]) for every i to within tol.
bool arithmetic(const double *dm, int n, double tol);

// Spectra plus the four-step intermediate for nblock blocks.
int workspace_bytes(const cdmt_plan_s *p, int nblock, size_t *bytes);

// Common argument checks of the calls that take a plan and its workspace.
int check_call(const cdmt_plan_s *p, void *ws, size_t ws_bytes, int nblock);

// Channel-chunk groups (4096 bins each) of the gradient kernels.
long long grad_groups(const cdmt_plan_s *p, int nblock);

}  // namespace cdmt
