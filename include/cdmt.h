/*
 * cdmt.h -- C ABI of the MI355X coherent-dedispersion library.
 *
 * Coherent dedispersion of channelised dual-polarisation complex voltages to
 * many dispersion-measure (DM) trials, after Bassa, Pleunis & Hessels (2016),
 * "Enabling pulsar and fast transient searches using coherent dedispersion".
 * Notation follows the paper: n_s subbands, n_c channels per subband, forward
 * transform size N_bin (nfft), backward size M_bin = N_bin / n_c, overlap of
 * n_d channel samples (noverlap = n_d * n_c subband samples).
 *
 * Ownership: the caller owns every device buffer (voltages, workspace,
 * output).  The library never allocates device memory at run time and never
 * copies between host and device; the DM list is passed to the kernels by
 * value.  A plan is a host object.
 *
 * Errors: every entry point returns CDMT_OK (0) or a negative status and, on
 * error, writes nothing to device memory.  Kernel launch failures are reported
 * as CDMT_E_DEVICE.  Calls that enqueue work are asynchronous on the given HIP
 * stream (NULL = the default stream) and return once the work is enqueued.
 * Concurrent calls with the same workspace race; distinct workspaces may run
 * concurrently on different streams.
 */
#ifndef CDMT_H
#define CDMT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cdmt_plan_s *cdmt_plan_t;

enum cdmt_status {
    CDMT_OK = 0,
    CDMT_E_ARG = -1,         /* null pointer, non-finite value, bad option      */
    CDMT_E_SHAPE = -2,       /* sizes violate the method's constraints          */
    CDMT_E_WORKSPACE = -3,   /* workspace smaller than cdmt_workspace_size      */
    CDMT_E_DEVICE = -4,      /* HIP error (no device, launch failure)           */
    CDMT_E_UNSUPPORTED = -5  /* valid for the method, not built in this library */
};

enum cdmt_opt {
    CDMT_OPT_INPUT = 0,      /* 0: complex float32 (default), 1: complex int8           */
    CDMT_OPT_CHIRP_REF = 1,  /* 0: nu0 = channel centre (default), 1: subband centre    */
    CDMT_OPT_SIGN = 2,       /* -1: dedisperse (default), +1: multiply by Eq. 1 as is   */
    CDMT_OPT_PRECISION = 3,  /* backward-FFT arithmetic of the DM stage: 0 FP32 vector
                                (default); 1 BF16x3, 2 FP16x3: radix-16 stages on the
                                matrix cores with hi/lo split operands and FP32
                                accumulation (M_bin = 4096 only, else
                                CDMT_E_UNSUPPORTED)                                     */
    CDMT_OPT_DM_TILE = 4,    /* DM trials per workgroup pass, 1..64 (default 64)        */
    CDMT_OPT_CHIRP_EXACT = 5,/* 1: evaluate the transfer function afresh for every DM;
                                0 (default): when the DM list is an arithmetic
                                progression, advance it by one complex factor per DM
                                inside a tile (both factors from FP64 sincospi)        */
    CDMT_OPT_LANE_BINS = 6,  /* performance knob of the DM stage: spectral bins held per
                                GPU lane, 16 (default) or 8 (twice the lanes per channel,
                                half the registers; used for M_bin = 2048 and 4096)      */
    CDMT_OPT_FWD_N2 = 7,     /* radix schedule of the forward FFT: the four-step split
                                N_bin = N1 * N2 with column transforms of N2 in
                                {64, 128, 256} and row transforms of N1 = N_bin / N2 in
                                [64, 512] (CDMT_E_ARG otherwise); default N2 =
                                2^floor(log2(N_bin) / 2).  Splits give the same spectra
                                up to FP32 rounding                                     */
    CDMT_OPT_OUT_LAYOUT = 8, /* filterbank layout of every call on this plan (DM stage,
                                batches, gradients' dL/dF, incoherent stage input):
                                0 (default): [DM][time][channel] (Sec. 3's transpose);
                                1: [DM][channel][time], which the incoherent stage
                                reads without its own transpose.  Same values either
                                way, bit for bit                                        */
    CDMT_OPT_DM_CHECK = 9,   /* 1 (default): every call that takes DMs rejects, with
                                CDMT_E_SHAPE, any |DM| above cdmt_dm_limit (its Eq. 2
                                sweep is longer than the overlap, so wrap-around of the
                                circular convolution would reach the kept samples,
                                Sec. 2); 0: no such check (a deliberately short overlap) */
    CDMT_OPT_FFT_SCHEDULE = 10 /* performance knob of the FP32 DM stage: 0 (default):
                                at M_bin 4096, 2048 or 1024 with ndec in
                                {1, 2, 4, 8} dividing n_d / 2, the backward FFT
                                runs as three passes (radix 16, 16 and M_bin /
                                256) with two LDS exchanges per DM (the first
                                within each wave; at 1024 both) and detection and
                                downsampling in registers; other plans as 1.
                                1: radix-16 Stockham stages with every digit
                                exchange and the detected power through LDS (all
                                M_bin).  Same results up to FP32 rounding      */
};

/*
 * Create a plan.  Sec. 3 (initialisation before Alg. 1's loops): the user
 * chooses n_c, N_bin and n_d; the frequency setup is n_s adjacent subbands of
 * width bw_sub_mhz (= complex sample rate in MHz, Nyquist sampling, Sec. 3),
 * upper sideband, in increasing frequency, centred on f_centre_mhz.  Subband s
 * is centred on f_centre + (s - (n_s-1)/2) * bw.
 *
 *   nsub       n_s >= 1
 *   nfft       N_bin, power of two in [2^10, 2^17] (other powers of two:
 *              CDMT_E_UNSUPPORTED)
 *   noverlap   n_d * n_c subband samples; multiple of 2*nchan, < nfft
 *              (Sec. 2: sections overlap by n_d n_c samples, n_d/2 channel
 *              samples discarded at each edge)
 *   nchan      n_c, power of two with M_bin = nfft/nchan in [64, 8192]
 *              (outside that range: CDMT_E_UNSUPPORTED)
 *   ndec       output samples summed per filterbank sample, >= 1, must
 *              divide M_bin - n_d
 * Requires bw_sub_mhz > 0 and f_centre - nsub*bw/2 > 0.
 * On success *out holds a new plan (free with cdmt_destroy).
 */
int cdmt_plan(cdmt_plan_t *out, int nsub, double f_centre_mhz, double bw_sub_mhz,
              int nfft, int noverlap, int nchan, int ndec);

/* Set an option (enum cdmt_opt).  CDMT_E_ARG for an unknown option or value. */
int cdmt_plan_set(cdmt_plan_t plan, int opt, int value);

/* Read an option back into *value. */
int cdmt_plan_get(cdmt_plan_t plan, int opt, int *value);

/*
 * Overlap needed for a DM range (Sec. 2: n_d = r t_d / n_c with t_d from
 * Eq. 2 for the lowest channel, or the lowest subband when chirp_ref = 1),
 * in subband samples, rounded up to a multiple of 2*nchan*ndec.
 * f_lo_mhz is the lower edge of the lowest subband; dm_max >= 0.
 */
int cdmt_noverlap_for(double f_lo_mhz, double bw_sub_mhz, double dm_max, int nchan, int ndec,
                      int chirp_ref, int *noverlap_out);

/*
 * The inverse of cdmt_noverlap_for for a plan: the largest |DM| (pc cm^-3)
 * whose Eq. 2 sweep, in subband samples r t_d with r = bw_sub in samples per
 * second, fits in the plan's noverlap (Sec. 2: sections overlap by at least
 * n_d n_c samples, t_d over the lowest channel, or over the lowest subband
 * when CDMT_OPT_CHIRP_REF = 1).  Writes *dm_max; CDMT_E_ARG for NULL.
 */
int cdmt_dm_limit(cdmt_plan_t plan, double *dm_max);

/*
 * Shapes for nblock blocks (Sec. 3, the block loop of Alg. 1):
 *   ntime_in  = nblock*(nfft - noverlap) + noverlap input samples per subband
 *   ntime_out = nblock*(M_bin - n_d)/ndec filterbank samples
 *   nchan_out = nsub*nchan
 * Output sample t covers input samples noverlap/2 + t*nchan*ndec + [0, nchan*ndec).
 * Any pointer may be NULL.
 */
int cdmt_output_shape(cdmt_plan_t plan, int nblock, long long *ntime_in, long long *ntime_out,
                      int *nchan_out);

/* Device workspace in bytes for nblock blocks (spectra of both polarisations
 * plus the four-step intermediate).  It does not depend on the number of DM
 * trials: the DM list reaches the kernels by value, so no ndm_max argument. */
int cdmt_workspace_size(cdmt_plan_t plan, int nblock, size_t *bytes);

/*
 * Forward stage of Alg. 1 for nblock blocks: unpack and segment (Sec. 3), the
 * forward FFT of N_bin per subband, block and polarisation, and the swap of
 * halves per subband.  The spectra stay in the workspace for
 * cdmt_dedisperse_spectra.
 *   voltages  device, [nsub][ntime_in][2 pol X,Y][re, im], float32 or int8
 *             (CDMT_OPT_INPUT), ntime_in from cdmt_output_shape
 */
int cdmt_forward(cdmt_plan_t plan, void *workspace, size_t ws_bytes, const void *voltages,
                 int nblock, void *hip_stream);

/*
 * DM stage of Alg. 1 on spectra left by cdmt_forward with the same nblock:
 * for every DM trial, the complex multiplication with the transfer function
 * of every channel (Sec. 2, Eq. 1), the swap of halves per channel, the
 * backward FFT of M_bin, unpadding (n_d/2 per edge), detection
 * |X|^2 + |Y|^2, the sum of ndec consecutive samples, and the transpose to
 * [time][channel] with channels in decreasing frequency.
 *   dm_list   host, ndm values in pc cm^-3, read during the call only; each
 *             must be finite with |DM| small enough that the largest phase of
 *             Eq. 1 over the plan stays below 2^29 cycles (CDMT_E_ARG
 *             otherwise; the bound is ~1e7 pc cm^-3 at LOFAR frequencies) and,
 *             unless CDMT_OPT_DM_CHECK = 0, |DM| <= cdmt_dm_limit (CDMT_E_SHAPE
 *             otherwise).  The same rules hold for every call taking DMs.
 *   out       device float32 [ndm][ntime_out][nsub*nchan] ([ndm][nsub*nchan]
 *             [ntime_out] with CDMT_OPT_OUT_LAYOUT = 1)
 * ndm = 0 is a no-op.
 */
int cdmt_dedisperse_spectra(cdmt_plan_t plan, void *workspace, size_t ws_bytes, int nblock,
                            const double *dm_list, int ndm, float *out, void *hip_stream);

/* cdmt_forward followed by cdmt_dedisperse_spectra: the whole of Alg. 1's
 * compute for nblock blocks and ndm DM trials. */
int cdmt_dedisperse(cdmt_plan_t plan, void *workspace, size_t ws_bytes, const void *voltages,
                    int nblock, const double *dm_list, int ndm, float *out, void *hip_stream);

/*
 * Derivative with respect to DM, for refining a candidate's DM by gradient
 * ascent (an extension beyond the paper: the adjoint of the DM stage of
 * Alg. 1).  For the spectra left by cdmt_forward and DM trials dm_list, with
 * the caller's upstream gradient grad_out = dL/dF of a scalar loss L of the
 * filterbank F that cdmt_dedisperse_spectra would produce with the exact
 * transfer function (CDMT_OPT_CHIRP_EXACT = 1):
 *   dldm[d] = dL/dDM_d = sum over subbands, blocks, channels and pols of
 *             Re(conj(g) i pi g2 S'), g the back-propagated gradient of the
 *             chirped spectrum S' (through detection, the downsampling sum and
 *             the backward FFT; the complex time series are recomputed, not
 *             stored), pi g2 = d(phase)/dDM of Eq. 1.
 *   grad_out  device float32 [ndm][ntime_out][nchan_out] (the plan's output
 *             layout, CDMT_OPT_OUT_LAYOUT)
 *   dldm      device float64 [ndm]
 *   gws       device, >= cdmt_gradient_workspace_size bytes (FP64 partial
 *             sums, 8 bytes per DM per 4096-bin chunk group)
 * FP32 arithmetic with FP64 accumulation; M_bin <= 4096 (CDMT_E_UNSUPPORTED
 * otherwise).  Asynchronous on hip_stream; on error nothing is written.
 */
int cdmt_gradient_workspace_size(cdmt_plan_t plan, int nblock, int ndm, size_t *bytes);
int cdmt_dm_gradient(cdmt_plan_t plan, void *workspace, size_t ws_bytes, int nblock,
                     const double *dm_list, int ndm, const float *grad_out, void *gws,
                     size_t gws_bytes, double *dldm, void *hip_stream);

/*
 * cdmt_dm_gradient for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same result, bit for bit, with the FP64 partial sums kept in a scratch
 * array the library holds on each GPU (cdmt_noalloc_scratch_bytes() =
 * 16 MiB, held from the first call on that GPU until the process ends)
 * instead of the caller's gws.  The caller still passes the spectra
 * workspace, grad_out and dldm.  Limit: cdmt_gradient_workspace_size(plan,
 * nblock, ndm) must not exceed the scratch size (CDMT_E_WORKSPACE
 * otherwise, nothing written), e.g. 64 DMs over 288 subbands x 4 blocks x
 * 16 channels at M_bin = 4096 use 9.4 MB.  Every call on a GPU shares that
 * GPU's array and overwrites the slots it uses before reading them, so
 * nothing needs clearing; calls that overlap on one GPU (other streams or
 * threads) race on it and must be serialised by the caller.  The first call
 * on a device also sets up the library's per-device tables (synchronous
 * copies, no allocation).  Other rules as cdmt_dm_gradient.
 */
int cdmt_dm_gradient_noalloc(cdmt_plan_t plan, void *workspace, size_t ws_bytes, int nblock,
                             const double *dm_list, int ndm, const float *grad_out, double *dldm,
                             void *hip_stream);
size_t cdmt_noalloc_scratch_bytes(void);

/*
 * Gradient of the same kind of loss with respect to the voltages, for one DM
 * (call once per DM with accumulate = 1 to sum over DMs): the adjoint
 * continued through the transfer function and the forward stage (forward
 * FFT, swap of halves, segmentation into overlapping blocks), i.e.
 *   grad_v[s][t][p] = dL/dRe x + i dL/dIm x  (stored re, im as float32)
 * for the voltages x that cdmt_forward turned into the spectra in workspace.
 *   grad_out  device float32 [ntime_out][nchan_out] (the plan's output
 *             layout): dL/dF of this DM
 *   grad_v    device float32 [nsub][ntime_in][2 pol][re, im] (layout of
 *             complex float32 voltages); overwritten (accumulate = 0) or
 *             added to (accumulate = 1)
 *   gws       device, >= cdmt_voltage_gradient_workspace_size bytes
 * FP32 arithmetic; M_bin <= 4096.  Asynchronous on hip_stream; on error
 * nothing is written.
 */
int cdmt_voltage_gradient_workspace_size(cdmt_plan_t plan, int nblock, size_t *bytes);
int cdmt_voltage_gradient(cdmt_plan_t plan, void *workspace, size_t ws_bytes, int nblock,
                          double dm, const float *grad_out, void *gws, size_t gws_bytes,
                          float *grad_v, int accumulate, void *hip_stream);

/*
 * Redigitisation of a filterbank to 8-bit codes (Sec. 3, the paragraph after
 * the transpose; Alg. 1 "redigitize").  Independent of any plan: it takes any
 * FP32 filterbank [ndm][ntime][nchan], e.g. the output of cdmt_dedisperse.
 * For every DM trial d and channel c, over the ntime samples of the call:
 *   mean[d][c]  = (float) mu,  mu = average of the series (FP64)
 *   scale[d][c] = (float) (counts_per_sigma / sigma), sigma = population
 *                 standard deviation (FP64); 0 when sigma = 0
 *   codes[d][t][c] = clamp(rint((x - mean) * scale + zero), 0, 255), each of
 *                 the three FP32 operations rounded separately, rint rounding
 *                 half to even.
 * zero is the code given to the mean and counts_per_sigma the codes per
 * standard deviation (finite, > 0); x ~= (code - zero) / scale + mean.
 *   filterbank  device float32 [ndm][ntime][nchan] (finite values)
 *   codes       device uint8 [ndm][ntime][nchan]
 *   mean, scale device float32 [ndm][nchan]
 *   workspace   device, at least cdmt_redigitise_workspace_size bytes
 *               (per-segment partial moments, 16 B per 1024 samples per
 *               DM and channel)
 * ndm = 0 is a no-op.  ndm and ceil(ntime / 1024) must not exceed 65535
 * (CDMT_E_SHAPE).  Asynchronous on hip_stream; on error nothing is written.
 */
int cdmt_redigitise_workspace_size(int ndm, long long ntime, int nchan, size_t *bytes);
int cdmt_redigitise(const float *filterbank, int ndm, long long ntime, int nchan, float zero,
                    float counts_per_sigma, void *workspace, size_t ws_bytes,
                    unsigned char *codes, float *mean, float *scale, void *hip_stream);

/*
 * Batches of beams.  The paper's survey processes several tied-array beams
 * per source (Sec. 4), each a separate coherent-dedispersion job.  A batch
 * runs any number of such jobs, each with its own plan (subbands, N_bin,
 * channels, overlap, ndec, nu0 mode), input, DM list (any length) and
 * output, as: the forward stage of every beam, then one persistent launch of
 * the FP32 DM stage per distinct M_bin = N_bin / n_c among the beams (one
 * launch when all share M_bin), whose workgroups take (beam, chunk group, DM
 * tile) items from per-XCD work queues until all are done.  Results are
 * bitwise equal to cdmt_dedisperse of each beam with the same DM tile.
 * Restrictions: FP32 precision, M_bin <= 4096 (CDMT_E_UNSUPPORTED
 * otherwise).
 */
typedef struct cdmt_batch_s *cdmt_batch_t;

typedef struct {
    cdmt_plan_t plan;          /* the beam's plan (used during create and runs)           */
    int nblock;                /* blocks of this beam, >= 1                               */
    const void *voltages;      /* device, as for cdmt_forward                             */
    const double *dm_list;     /* host, ndm values, read during create only; checked
                                  against the beam's plan as by cdmt_dedisperse (phase
                                  bound, and cdmt_dm_limit unless CDMT_OPT_DM_CHECK = 0) */
    int ndm;                   /* >= 1                                                    */
    float *out;                /* device [ndm][ntime_out][nchan_out] of this beam (its
                                  plan's CDMT_OPT_OUT_LAYOUT)                           */
} cdmt_beam_t;

enum cdmt_batch_opt {
    CDMT_BATCH_DM_TILE = 0,    /* DM trials per item for every beam, 1..64; 0 = each plan's */
    CDMT_BATCH_WG_PER_CU = 1,  /* persistent workgroups per compute unit, 1..8 (default 2)  */
    CDMT_BATCH_ITEMS = 2,      /* (get only) work items of the DM stage                      */
    CDMT_BATCH_LAUNCHES = 3    /* (get only) persistent launches (one per distinct M_bin)    */
};

/* Workspace for a batch: every beam's spectra (cdmt_workspace_size), the DM
 * lists, the item table and the queue counters, 256-byte aligned. */
int cdmt_batch_workspace_size(const cdmt_beam_t *beams, int nbeam, size_t *bytes);

/* Validate the beams (as cdmt_dedisperse would), copy the DM lists and the
 * item table into the caller's workspace (synchronous host-to-device copies,
 * the only ones this library makes) and return a batch.  The plans, device
 * buffers and workspace must outlive the batch. */
int cdmt_batch_create(cdmt_batch_t *out, const cdmt_beam_t *beams, int nbeam, void *workspace,
                      size_t ws_bytes);

/* Change an option (enum cdmt_batch_opt).  Rewrites the item table after a
 * device-wide synchronisation; a captured graph is captured again on its
 * next run. */
int cdmt_batch_set(cdmt_batch_t batch, int opt, int value);
int cdmt_batch_get(cdmt_batch_t batch, int opt, long long *value);

/* Per-beam settings of a batch (enum cdmt_batch_beam_opt), beam = index in
 * the creation order; the beam's plan is not modified.
 * CDMT_BATCH_BEAM_FWD_N2: the forward FFT's split for that beam (as
 * CDMT_OPT_FWD_N2; set 0 to use the beam plan's own).
 * CDMT_BATCH_BEAM_FFT_SCHEDULE: the DM stage's schedule for that beam (as
 * CDMT_OPT_FFT_SCHEDULE, 0 or 1; -1 to use the beam plan's own).
 * CDMT_BATCH_BEAM_LANE_BINS: bins per lane of its DM stage (as
 * CDMT_OPT_LANE_BINS, 8 or 16, taking effect at M_bin = 2048 and 4096 with
 * the Stockham stages; 0 to use the beam plan's own).
 * These two decide the beam's launch group, so setting one rewrites the
 * item table after a device-wide synchronisation; results are bitwise equal
 * to cdmt_dedisperse of the beam with the same settings (and the batch's DM
 * tile). */
enum cdmt_batch_beam_opt {
    CDMT_BATCH_BEAM_FWD_N2 = 0,
    CDMT_BATCH_BEAM_FFT_SCHEDULE = 1,
    CDMT_BATCH_BEAM_LANE_BINS = 2
};
int cdmt_batch_beam_set(cdmt_batch_t batch, int beam, int opt, int value);
int cdmt_batch_beam_get(cdmt_batch_t batch, int beam, int opt, int *value);

/* Enqueue the whole batch on hip_stream (NULL = default stream). */
int cdmt_batch_run(cdmt_batch_t batch, void *hip_stream);

/* The same work as a HIP graph: captured from hip_stream (which must be a
 * created stream, not NULL) on the first call or after an option changed,
 * then replayed with one hipGraphLaunch per call.  The graph holds no memset
 * nodes (the queue counters are cleared by a kernel). */
int cdmt_batch_run_graph(cdmt_batch_t batch, void *hip_stream);

/* Autotune the batch on hip_stream.  First the radix schedule of each
 * beam's forward FFT: every valid split N1 x N2 (CDMT_OPT_FWD_N2) of the
 * beam's N_bin is timed on that beam's forward stage alone and the fastest
 * kept (CDMT_BATCH_BEAM_FWD_N2).  Then the DM stage's radix schedule per
 * M_bin (beams of one M_bin share launches), each candidate timed on the
 * whole batch: at M_bin 4096 and 2048 the three-pass transform, radix-16 and
 * radix-8 Stockham stages; at 1024 the three-pass transform and radix 16
 * (CDMT_BATCH_BEAM_FFT_SCHEDULE, CDMT_BATCH_BEAM_LANE_BINS).  Then the
 * whole batch for every DM tile in {8, 16, 32, 64} and 2 or 4 workgroups per CU;
 * the fastest setting is kept and its time per run returned in *best_ms
 * (may be NULL).  reps runs per candidate after one warm-up.  Writes the
 * beams' outputs. */
int cdmt_batch_autotune(cdmt_batch_t batch, void *hip_stream, int reps, float *best_ms);

/* Free a batch and its graph (NULL is accepted). */
void cdmt_batch_destroy(cdmt_batch_t batch);

/*
 * Incoherent stage of a semi-coherent search (Sec. 1; Sec. 4, where coherent
 * trials at coarse DM steps are followed by incoherent dedispersion at fine
 * steps around each): for every coherent trial d the filterbank fb[d]
 * (typically what cdmt_dedisperse wrote for dm_coh[d]) is dedispersed at the
 * ntrial DMs  DM_dk = dm_coh[d] + (ddm0 + k ddm),  k = 0 .. ntrial-1:
 *   out[d][k][t] = sum_ch fb[d][t + D(ch, DM_dk)][ch],   t < nout,
 * D = the Eq. 2 delay of channel ch behind the highest channel, in output
 * samples of nchan*ndec/bw_sub seconds, rounded half to even, computed in
 * FP64 as  rint(((k_DM DM) u) / tsamp),  u = 1/nu^2 - 1/nu_top^2, nu the
 * frequency the plan's chirp refers channel ch to (its centre, or its
 * subband's centre with CDMT_CHIRP_SUBBAND); nout = ntime - the largest
 * delay (lowest channel, largest trial DM), ntime = nblock * tblk.  Sums in
 * FP32 over channels in increasing order.
 *   fb         device float32 [ndm][ntime][nsub*nchan], decreasing frequency
 *              ([ndm][nsub*nchan][ntime] when the plan's CDMT_OPT_OUT_LAYOUT
 *              is 1: then no transposed copy is made)
 *   dm_coh     host, ndm values;  every DM_dk must be >= 0
 *   ddm        > 0 when ntrial > 1
 *   workspace  device, >= cdmt_incoherent_workspace_size bytes (the
 *              filterbanks transposed to [ndm][nch][ntime] and the delay
 *              table, at most ndm * nch * ceil(ntrial / 12) * 12 int32)
 *   out        device float32 [ndm][ntrial][nout]
 * CDMT_E_ARG for bad DMs or steps or a NULL pointer, CDMT_E_WORKSPACE for a
 * short workspace, CDMT_E_SHAPE when nout < 1, ndm exceeds 65535, ntime
 * exceeds 2^31 - 1 or ndm * ceil(nout / 256) * ceil(ntrial / 12) exceeds
 * 2^31 - 1.  The shape call validates the same arguments and returns nout.
 * Asynchronous on hip_stream; on error nothing is written.
 */
int cdmt_incoherent_shape(cdmt_plan_t plan, int nblock, const double *dm_coh, int ndm,
                          double ddm0, double ddm, int ntrial, long long *nout);
int cdmt_incoherent_workspace_size(cdmt_plan_t plan, int nblock, int ndm, int ntrial,
                                   size_t *bytes);
int cdmt_incoherent(cdmt_plan_t plan, int nblock, const float *fb, const double *dm_coh, int ndm,
                    double ddm0, double ddm, int ntrial, void *workspace, size_t ws_bytes,
                    float *out, void *hip_stream);

/* Free a plan (NULL is accepted). */
void cdmt_destroy(cdmt_plan_t plan);

/* Static description of a status code. */
const char *cdmt_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* CDMT_H */
