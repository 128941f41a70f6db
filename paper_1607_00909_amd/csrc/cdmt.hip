// MI355X (gfx950) coherent dedispersion to many DM trials.
//
// Method: Bassa, Pleunis & Hessels (2016), Sec. 2-3 and Alg. 1.  For each
// block of N_bin samples of each subband (blocks overlap by n_d n_c samples):
// forward FFT, swap halves, then for every DM trial: multiply each channel's
// bins by the transfer function of Eq. 1, swap halves per channel, backward
// FFT of M_bin = N_bin / n_c, drop n_d/2 samples at each edge, detect
// |X|^2 + |Y|^2, sum ndec consecutive samples, and store the filterbank as
// [DM][time][channel] with channels in decreasing frequency.
//
// Kernels (all hand-written here, see fft_core.hpp for the FFT engine):
//   fwd_col  first pass of a four-step N_bin = N1 x N2 forward FFT: reads the
//            voltages (int8 or float32, widened exactly), N2-point transforms
//            over stride-N1 columns, four-step twiddle, stores [k2][n1].
//   fwd_row  second pass: N1-point transforms over rows, transposed through
//            LDS so the store is contiguous, swap of halves and the 1/N_bin
//            normalisation folded into the store; spectra are kept as
//            [block][subband][bin] pairs (both pols), so channel c of a
//            subband is the contiguous run of bins [c M, (c+1) M).
//   fused_dedisperse  one workgroup per (channel chunk(s), DM tile): loads a
//            channel's M bins once into registers and, for each DM of the
//            tile, applies the transfer function (phase in FP64, reduced to
//            [-1/2, 1/2) cycles, then FP32 sincos), runs the M-point backward
//            FFT in registers + LDS, detects, downsamples and stores.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/cdmt.h"
#include "fft_core.hpp"
#include "plan.hpp"
#include "xcd.hpp"

using cdmt::cpair;

namespace {

using cdmt::kKdm;
using namespace cdmt;

constexpr int kMaxDmPerLaunch = 256;
constexpr int kTwiddleEntries = 1 << 18;   // sizes 1 .. 2^17, table P at [P, 2P)

__device__ float2 g_twiddle[kTwiddleEntries];

__device__ __forceinline__ const float2 *twiddles(int p) { return g_twiddle + p; }

using cdmt::xcd_remap;

struct FwdArgs {
    const void *x;          // voltages [nsub][ntime_in][2][2]
    cpair *ybuf;            // four-step intermediate [block][subband][k2][n1]
    cpair *spec;            // spectra [block][subband][N]
    long long ntime_in;
    int nsub, nblock, n1, n2, n, step;   // step = N - noverlap
    float inv_n;
};

// ---------------------------------------------------------------------------
// Forward FFT, pass 1 (columns).  P = N2.  C = 4096/P columns per workgroup,
// lane t -> column f = t % C (fastest, so loads are contiguous in time),
// tt = t / C.
template <int P, bool CI8>
__global__ __launch_bounds__(256) void fwd_col(FwdArgs a) {
    constexpr int T = P / 16, C = 4096 / P;
    __shared__ cpair sh[P * C];
    const int groups = a.n1 / C;
    // neighbouring column groups share 128-byte lines of int8 input: keep
    // them on one XCD (one L2)
    const int lw = xcd_remap(blockIdx.x, gridDim.x);
    const int g = lw % groups;
    const int bs = lw / groups;                  // block * nsub + subband
    const int s = bs % a.nsub, b = bs / a.nsub;
    const int t = threadIdx.x, f = t % C, tt = t / C;
    const int n1 = g * C + f;
    const long long first = (long long)s * a.ntime_in + (long long)b * a.step + n1;

    cpair v[16];
    if constexpr (CI8) {
        // one dword = one time sample: bytes X.re, X.im, Y.re, Y.im (int8)
        const int *x = reinterpret_cast<const int *>(a.x) + first;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int w = x[(long long)a.n1 * (tt + T * q)];
            v[q] = make_float4((float)(int8_t)w, (float)(int8_t)(w >> 8),
                               (float)(int8_t)(w >> 16), (float)(int8_t)(w >> 24));
        }
    } else {
        const float4 *x = reinterpret_cast<const float4 *>(a.x) + first;
#pragma unroll
        for (int q = 0; q < 16; ++q)
            v[q] = x[(long long)a.n1 * (tt + T * q)];
    }
    cdmt::LdsInterleaved<C> lds{sh + f};
    cdmt::wg_fft<P, -1, 16>(v, tt, lds);

    // four-step twiddle exp(-2 pi i n1 k2 / N), then store row k2
    const float2 *twn = twiddles(a.n);
    cpair *y = a.ybuf + (long long)bs * a.n;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int k2 = tt + T * q;
        float2 w = twn[(n1 * k2) & (a.n - 1)];
        w.y = -w.y;
        y[(long long)k2 * a.n1 + n1] = cdmt::pmul(v[q], w);
    }
}

// Forward FFT, pass 2 (rows).  P = N1.  C = 4096/P rows per workgroup.
template <int P>
__global__ __launch_bounds__(256) void fwd_row(FwdArgs a) {
    constexpr int T = P / 16, C = 4096 / P;
    constexpr int STRIDE = P + P / 16 + 1;    // odd: conflict-free transposed reads
    __shared__ cpair sh[C * STRIDE];
    const int groups = a.n2 / C;
    const int lw = xcd_remap(blockIdx.x, gridDim.x);
    const int g = lw % groups;
    const int bs = lw / groups;
    const int t = threadIdx.x;
    const int f = t / T, tt = t % T;          // lanes along the row: contiguous loads
    const int k2 = g * C + f;

    const cpair *y = a.ybuf + (long long)bs * a.n + (long long)k2 * P;
    cpair v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q)
        v[q] = y[tt + T * q];
    cdmt::LdsPadded lds{sh + f * STRIDE};
    cdmt::wg_fft<P, -1, 16>(v, tt, lds);

    // X[k2 + N2 k1] with k1 = tt + T q.  Transpose through LDS so that
    // consecutive lanes store consecutive k2, i.e. consecutive bins.
#pragma unroll
    for (int q = 0; q < 16; ++q)
        lds.store(tt + T * q, v[q]);
    __syncthreads();
    const int f2 = t % C, tt2 = t / C;
    const cdmt::LdsPadded rd{sh + f2 * STRIDE};
    cpair *spec = a.spec + (long long)bs * a.n;
    const int half = a.n >> 1;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int k1 = tt2 + T * q;
        const int k = g * C + f2 + a.n2 * k1;
        const int j = (k + half) & (a.n - 1);     // swap halves per subband
        spec[j] = cdmt::pscale(rd.load(k1), a.inv_n);
    }
}

// Forward FFT in one pass for N_bin = P <= 2048: C = 4096/P transforms per
// workgroup, one per (block, subband), lanes along the transform so that the
// loads are contiguous in time; the swap of halves and 1/N_bin are folded
// into the store as in fwd_row.
template <int P, bool CI8>
__global__ __launch_bounds__(256) void fwd_one(FwdArgs a) {
    constexpr int T = P / 16, C = 4096 / P;
    constexpr int STRIDE = P + P / 16 + 1;
    __shared__ cpair sh[C * STRIDE];
    const int t = threadIdx.x, f = t / T, tt = t % T;
    const long long bs = (long long)blockIdx.x * C + f;     // block * nsub + subband
    const bool valid = bs < (long long)a.nblock * a.nsub;
    const int s = valid ? (int)(bs % a.nsub) : 0;
    const int b = valid ? (int)(bs / a.nsub) : 0;
    const long long first = (long long)s * a.ntime_in + (long long)b * a.step + tt;

    cpair v[16];
    if constexpr (CI8) {
        const int *x = reinterpret_cast<const int *>(a.x) + first;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int w = valid ? x[T * q] : 0;
            v[q] = make_float4((float)(int8_t)w, (float)(int8_t)(w >> 8),
                               (float)(int8_t)(w >> 16), (float)(int8_t)(w >> 24));
        }
    } else {
        const float4 *x = reinterpret_cast<const float4 *>(a.x) + first;
#pragma unroll
        for (int q = 0; q < 16; ++q)
            v[q] = valid ? x[T * q] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    cdmt::LdsPadded lds{sh + f * STRIDE};
    cdmt::wg_fft<P, -1, 16>(v, tt, lds);
    if (valid) {
        cpair *spec = a.spec + bs * P;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int k = tt + T * q;
            spec[(k + P / 2) & (P - 1)] = cdmt::pscale(v[q], a.inv_n);   // swap halves
        }
    }
}

// sin(pi r) and cos(pi r) for |r| <= 1/2.  Odd / even polynomials whose
// coefficients were fitted for this kernel by iteratively reweighted least
// squares toward the minimax error (Lawson's method) on Chebyshev nodes; the
// largest absolute error in FP32 evaluation is 2.1e-7.
__device__ __forceinline__ void sincos_pi(float r, float &s, float &c) {
    const float r2 = r * r;
    float ps = 7.722071558e-02f;
    ps = fmaf(ps, r2, -5.980455279e-01f);
    ps = fmaf(ps, r2, 2.550031424e+00f);
    ps = fmaf(ps, r2, -5.167706966e+00f);
    ps = fmaf(ps, r2, 3.141592503e+00f);
    s = ps * r;
    float pc = -2.439684793e-02f;
    pc = fmaf(pc, r2, 2.349376380e-01f);
    pc = fmaf(pc, r2, -1.335212111e+00f);
    pc = fmaf(pc, r2, 4.058709145e+00f);
    pc = fmaf(pc, r2, -4.934802055e+00f);
    c = fmaf(pc, r2, 1.0f);
}

// exp(i pi t) for a phase t in half-cycles, in double precision: t is reduced
// to n + r with |r| <= 1/2, sin(pi r) and cos(pi r) come from odd / even
// polynomials fitted for this library (Lawson's method in float64; max error
// 8e-14 and 5e-15), and (-1)^n is applied as a sign.  Rounded to float.
__device__ __forceinline__ float2 cis_pi_f64(double t) {
    const double n = rint(t);
    const double r = t - n;
    const double r2 = r * r;
    double ps = 0.000447492634787997;
    ps = fma(ps, r2, -0.007364005763000102);
    ps = fma(ps, r2, 0.08214479472358047);
    ps = fma(ps, r2, -0.5992644339392923);
    ps = fma(ps, r2, 2.5501640359072306);
    ps = fma(ps, r2, -5.167712779988032);
    ps = fma(ps, r2, 3.1415926535896257);
    double pc = -0.00010031723352996529;
    pc = fma(pc, r2, 0.0019277873522597125);
    pc = fma(pc, r2, -0.025806505139857543);
    pc = fma(pc, r2, 0.23533058404112456);
    pc = fma(pc, r2, -1.3352627658364828);
    pc = fma(pc, r2, 4.058712126320176);
    pc = fma(pc, r2, -4.934802200543524);
    pc = fma(pc, r2, 0.9999999999999983);
    const int flip = static_cast<int>(n) << 31;
    const float sn = __int_as_float(__float_as_int(static_cast<float>(ps * r)) ^ flip);
    const float cs = __int_as_float(__float_as_int(static_cast<float>(pc)) ^ flip);
    return make_float2(cs, sn);
}

// a *= w for both complex values of a pair, in place: the cross products are
// formed from the old values first, then each fused multiply-add overwrites
// its own input (tied operands), so a value carried around a loop keeps its
// registers instead of being copied back at the loop latch.
__device__ __forceinline__ void pmul_inplace(cpair &a, float2 w) {
    float xr = a.x, xi = a.y, yr = a.z, yi = a.w;
    const float tx = xi * w.y, ux = xr * w.y;
    const float ty = yi * w.y, uy = yr * w.y;
    asm("v_fma_f32 %0, %0, %1, -%2" : "+v"(xr) : "v"(w.x), "v"(tx));
    asm("v_fma_f32 %0, %0, %1, %2" : "+v"(xi) : "v"(w.x), "v"(ux));
    asm("v_fma_f32 %0, %0, %1, -%2" : "+v"(yr) : "v"(w.x), "v"(ty));
    asm("v_fma_f32 %0, %0, %1, %2" : "+v"(yi) : "v"(w.x), "v"(uy));
    a = make_float4(xr, xi, yr, yi);
}

struct FusedArgs {
    const cpair *spec;      // [block][subband][N]
    float *out;             // first DM of this launch: [ndm][ntime_out][nsub*nchan]
    long long ntime_out;
    int nsub, nchan, n, nchunks, ndm, dm_tile;
    int nd_half, ndec, tblk, nch_out;
    // filterbank element (t, col) of a DM at t * t_stride + col * col_stride:
    // (nch_out, 1) time-major [t][ch] (default), (1, ntime_out) channel-major
    int t_stride;
    long long col_stride;
    int inner, ndt;         // chunk groups per subband block; DM tiles
    int cg0;                // first chunk group of this launch
    double dm_step;         // DM spacing when the list is an arithmetic progression
    int chirp_ref;
    float sign;
    double f_centre, bw, delta, kk;   // MHz, MHz, bw/N MHz, 1e6 k_DM
    int schedule;           // CDMT_OPT_FFT_SCHEDULE
};

struct DmList {
    double dm[kMaxDmPerLaunch];
};

// Transfer function, FFT, detection and downsampling for C = WG/T channel
// chunks of M bins and a tile of DMs.
// RECUR: the launch's DM list is an arithmetic progression with step a.dm_step,
// so within a tile the chirped spectrum advances by one factor per DM:
// P(d+1) = P(d) exp(i pi dm_step g2), both factors from FP64 sincospi.
//
// R = bins per lane (16: 256-lane workgroups, radix-16 stages; 8: 512-lane
// workgroups at M = 4096, radix-8 stages, half the registers per lane).
template <int M, int R>
struct FusedShape {
    static constexpr int T = M / R;                       // lanes per chunk
    static constexpr int WG = T > 256 ? T : 256;
    static constexpr int C = WG / T;                      // chunks per workgroup
    static constexpr int STRIDE = M + M / R + 1;          // LDS per chunk (pairs)
    // minimum waves per SIMD requested from the compiler: R = 8 asks for 4
    // (two 512-lane workgroups per CU, at most 128 VGPRs per lane)
    static constexpr int MIN_WAVES = R == 8 ? 4 : 1;
};

// DM values of a launch: passed by value in the kernel arguments, or read
// from device memory (batched launches); the index is uniform over the
// workgroup, so either way the load is scalar
struct ArgDms {
    const DmList &dl;
    __device__ __forceinline__ double operator[](int i) const { return dl.dm[i]; }
};
struct MemDms {
    const double *p;
    __device__ __forceinline__ double operator[](int i) const { return p[i]; }
};

// One work item: chunk group cg (C channel chunks) and DM tile dt.
template <int M, int R, bool RECUR, class DMS>
__device__ __forceinline__ void dm_item(const FusedArgs &a, DMS dms, int dt, int cg, cpair *sh) {
    using Sh = FusedShape<M, R>;
    constexpr int T = Sh::T;
    constexpr int C = Sh::C;
    constexpr int STRIDE = Sh::STRIDE;

    const int t = threadIdx.x;
    const int f = t / T, tt = t % T;
    const int chunk = cg * C + f;
    const bool valid = chunk < a.nchunks;
    const int cc = valid ? chunk : 0;
    const int c = cc % a.nchan;
    const int bs = cc / a.nchan;
    const int s = bs % a.nsub;
    const int b = bs / a.nsub;

    // this channel's M bins, both pols, increasing frequency
    cpair raw[R];
    {
        // the chunk as a raw buffer (no records when this lane's chunk is
        // past the end: the loads return zeros), row q at a scalar offset
        const cpair *src = a.spec + (long long)bs * a.n + (long long)c * M;
        const __amdgpu_buffer_rsrc_t view = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<cpair *>(src), (short)0, valid ? M * 16 : 0, 0x00020000);
#pragma unroll
        for (int q = 0; q < R; ++q)
            raw[q] = __builtin_bit_cast(
                cpair, __builtin_amdgcn_raw_buffer_load_b128(view, 16 * tt, 16 * T * q, 0));
    }

    // DM-independent part of Eq. 1 per bin: g2 = 2 * sign * 1e6 k_DM nu^2 /
    // (nu0^2 (nu0 + nu)), nu = offset from nu0 in MHz, so that for DM d the
    // transfer function exp(sign 2 pi i DM g) = exp(i pi DM g2).
    const double fs = a.f_centre + ((double)s - 0.5 * (a.nsub - 1)) * a.bw;
    double nu0, off;
    int cofs;   // bin offset of the channel within the frequency axis of nu
    if (a.chirp_ref == 0) {
        nu0 = fs - 0.5 * a.bw + ((double)c + 0.5) * a.bw / a.nchan;
        off = -0.5 * M;
        cofs = 0;
    } else {
        nu0 = fs;
        off = -0.5 * a.n;
        cofs = c * M;
    }
    const double scale = 2.0 * a.sign * a.kk / (nu0 * nu0);
    double g2[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        // (the bin's index converted per item, not held across a batch's items)
        const double nu = ((double)(tt + T * q + cofs) + off) * a.delta;
        g2[q] = scale * nu * nu / (nu0 + nu);
    }

    const cdmt::LdsPad<R> lds{sh + f * STRIDE};
    float *inten = reinterpret_cast<float *>(sh + f * STRIDE);
    const int col = (a.nsub - 1 - s) * a.nchan + (a.nchan - 1 - c);
    const int d0 = dt * a.dm_tile;
    const int d1 = min(a.ndm, d0 + a.dm_tile);

    float2 step[R];
    if constexpr (RECUR) {
        // P(d0) = raw exp(i pi dm(d0) g2) and the per-DM step, in double
#pragma unroll
        for (int q = 0; q < R; ++q) {
            raw[q] = cdmt::pmul(raw[q], cis_pi_f64(dms[d0] * g2[q]));
            step[q] = cis_pi_f64(a.dm_step * g2[q]);
        }
    }

    for (int d = d0; d < d1; ++d) {
        cpair v[R];
        if constexpr (RECUR) {
#pragma unroll
            for (int q = 0; q < R; ++q) {
                // swap halves per channel: bin i -> transform input (i + M/2) mod M
                v[q ^ (R / 2)] = raw[q];
                raw[q] = cdmt::pmul(raw[q], step[q]);
            }
        } else {
            const double dm = dms[d];
#pragma unroll
            for (int q = 0; q < R; ++q) {
                // phase in half-cycles, reduced in FP64 to n + r with |r| <= 1/2
                const double t = dm * g2[q];
                const double n = rint(t);
                float sn, cs;
                sincos_pi(static_cast<float>(t - n), sn, cs);
                const int flip = static_cast<int>(n) << 31;      // (-1)^n
                sn = __int_as_float(__float_as_int(sn) ^ flip);
                cs = __int_as_float(__float_as_int(cs) ^ flip);
                // swap halves per channel: bin i -> transform input (i + M/2) mod M
                v[q ^ (R / 2)] = cdmt::pmul(raw[q], make_float2(cs, sn));
            }
        }
        cdmt::wg_fft<M, +1>(v, tt, lds);

        // detect; channel sample m = tt + T q
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const cpair y = v[q];
            inten[tt + T * q] = y.x * y.x + y.y * y.y + y.z * y.z + y.w * y.w;
        }
        __syncthreads();
        if (valid) {
            float *o = a.out + (long long)d * a.ntime_out * a.nch_out +
                       (long long)b * a.tblk * a.t_stride + col * a.col_stride;
            if (((a.ndec | a.nd_half) & 3) == 0) {
                // 16-byte LDS reads when the summed runs are 4-float aligned
                const int n4 = a.ndec >> 2;
                for (int tq = tt; tq < a.tblk; tq += T) {
                    const float4 *p = reinterpret_cast<const float4 *>(inten + a.nd_half) + tq * n4;
                    float acc = 0.f;
                    for (int q = 0; q < n4; ++q) {
                        const float4 x = p[q];
                        acc += (x.x + x.y) + (x.z + x.w);
                    }
                    o[(long long)tq * a.t_stride] = acc;
                }
            } else {
                for (int tq = tt; tq < a.tblk; tq += T) {
                    const float *p = inten + a.nd_half + tq * a.ndec;
                    float acc = 0.f;
                    for (int q = 0; q < a.ndec; ++q)
                        acc += p[q];
                    o[(long long)tq * a.t_stride] = acc;
                }
            }
        }
        __syncthreads();
    }
}

template <int M, int R, bool RECUR>
__global__ __launch_bounds__((FusedShape<M, R>::WG), (FusedShape<M, R>::MIN_WAVES)) void fused_dedisperse(FusedArgs a,
                                                                         DmList dl) {
    using Sh = FusedShape<M, R>;
    __shared__ cpair sh[Sh::C * Sh::STRIDE];
    const int lw = xcd_remap(blockIdx.x, gridDim.x);
    const int ci = lw % a.inner;
    const int rest = lw / a.inner;
    const int dt = rest % a.ndt;
    const int cg = a.cg0 + (rest / a.ndt) * a.inner + ci;
    dm_item<M, R, RECUR>(a, ArgDms{dl}, dt, cg, sh);
}

// ---------------------------------------------------------------------------
// DM stage at M_bin = 4096: three radix-16 passes, two LDS exchanges per DM.
//
// The 4096-point backward transform y[k] = sum_i x[i] exp(+2 pi i i k / 4096)
// with i = G0 + 16 G1 + 256 G2 and k = K0 + 16 K1 + 256 K2 (hexadecimal
// digits) factors as
//   y = sum_G0 w16^(G0 K2) w4096^(G0 (K0 + 16 K1))
//         sum_G1 w16^(G1 K1) w256^(G1 K0) sum_G2 w16^(G2 K0) x,
// i.e. a 16-point DFT over G2, the twiddle w256^(G1 K0), a 16-point DFT over
// G1, the twiddle w4096^(G0 (K0 + 16 K1)) and a 16-point DFT over G0.  Each
// of the 256 lanes of a channel chunk holds 16 bin pairs (both polarisations)
// in registers; lane L = l03 + 16 l45 + 64 w (w the wave).
//   load        registers G2, lane digits G1 = l03, G0 = l45 + 4 w
//   pass 1      DFT over G2 -> registers K0; twiddle w256^(G1 K0)
//   exchange 1  registers K0 <-> lane digit l03 (within each wave)
//   pass 2      DFT over G1 -> registers K1
//   exchange 2  registers K1 <-> lane digits (l45, w) (across the waves)
//   pass 3      twiddle w4096^(G0 L), DFT over G0 -> registers K2
// so register q of lane L ends with output sample m = L + 256 q.  Detection
// adds the two polarisations' power in registers; downsampling by ndec = 2^K
// sums over m's lowest K bits, lane bits, across lanes (DPP).
//
// LDS: each wave owns a region of 4 blocks (one per l45) of 272 slots (one
// slot = one bin pair).  Exchange 1 writes element (G1, K0) of block (w, l45)
// at row K0, column G1 of rows of 17 slots and reads it back within the wave;
// exchange 2 writes element (G0, K0, K1) into the same region (block G0 & 3
// of wave G0 >> 2, row K1, column K0, rows of 16), which no other wave touched
// since the previous barrier, so each DM needs two barriers: one before
// exchange 1's writes (every wave has read the previous DM's exchange 2) and
// one between exchange 2's writes and reads.
//
// The same item serves M_bin 2048 and 1024 with a radix-P3 last pass, P3 =
// M / 256 (16 x 16 x 8 and 16 x 16 x 4): a chunk then spans M / 1024 waves
// (two, or one with no workgroup barrier), bins G0 + (M / 256) G1 + (M / 16)
// G2 with G0 = l45 + 4 (w mod M / 1024), and register r ends with sample
// Lc + (M / 16)(r / P3) + 256 (r mod P3), Lc the lane within the chunk.

// exp(+2 pi i g k / 256) at [g][k] (pass 2's twiddles, g = G1, k = K0) and
// exp(+2 pi i r l / 4096) at [l][r] (pass 3's, r = G0, l = K0 + 16 K1, the
// lane index).  Filled once per device from double precision.
__device__ __align__(16) float2 g_tw1[16 * 16];
__device__ __align__(16) float2 g_tw2[256 * 16];
// M_bin = 2048 pass 3: row l (0..127), column r: exp(+2 pi i (r & 7)(l + 128 (r >> 3)) / 2048)
__device__ __align__(16) float2 g_tw2h[128 * 16];
// M_bin = 1024 pass 3: row l (0..63), column r: exp(+2 pi i (r & 3)(l + 64 (r >> 2)) / 1024)
__device__ __align__(16) float2 g_tw2q[64 * 16];

constexpr int kX3Region = 4 * 16 * 17;       // bin pairs of LDS per wave
constexpr int kX3Lds = 4 * kX3Region;        // per workgroup (68 KiB)
constexpr int kX3TwLds = 4 * 144;            // pass 2's twiddle table in LDS (four copies)

// The w256 twiddle table g_tw1 (row r, column c: exp(+2 pi i r c / 256)) as
// four copies in LDS, 16-byte slot 144 k + 16 h + r of copy k holding
// columns 2h, 2h + 1 of row r.  A wave whose lane L reads row L & 15 from copy
// (L >> 4) & 3 touches 64 distinct slots mod 64 per read (no bank conflicts;
// one copy with the 64 lanes' reads of 16 rows broadcast to 4 lanes each
// measured 0.112 conflict cycles per LDS-active cycle).  All 256 lanes write.
__device__ __forceinline__ void put_tw1_lds(float2 *twl) {
    const int L = threadIdx.x, r = L >> 4, c = L & 15;
    const float2 t = g_tw1[L];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        twl[2 * (144 * k + 16 * (c >> 1) + r) + (c & 1)] = t;
}

// x from lane (lane xor the DPP pattern): quad_perm [1,0,3,2] = lane ^ 1,
// [2,3,0,1] = lane ^ 2, row_half_mirror = lane ^ 7 within 8 lanes
template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, false));
}
constexpr int kDppX1 = 0xb1, kDppX2 = 0x4e, kDppX7 = 0x141;

// One halving step of the sum across a lane pair (partner lane = DPP CTRL):
// of every value pair (p[2j], p[2j+1]) this lane keeps index 2j + bit and
// adds the partner's copy of it.
template <int CTRL, int N>
__device__ __forceinline__ void fold(const float (&p)[2 * N], float (&r)[N], bool bit) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const float keep = bit ? p[2 * j + 1] : p[2 * j];
        const float send = bit ? p[2 * j] : p[2 * j + 1];
        r[j] = keep + dpp<CTRL>(send);
    }
}

// Order this wave's LDS accesses before and after (the hardware executes a
// wave's LDS instructions in order; this keeps the compiler from moving them
// across).
__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// One work item: chunk group cg (4096 / M channel chunks) and DM tile dt, at
// M_bin = M (4096, 2048 or 1024), ndec = 2^K (K <= 3) and n_d / 2 a multiple
// of ndec.  sh holds kX3Lds bin pairs (plus kX3TwLds when TWL != 0).
template <bool RECUR, int K, class DMS, int TWL = 0, int M = 4096>
__device__ __forceinline__ void dm_item_x3(const FusedArgs &a, DMS dms, int dt, int cg, cpair *sh) {
    static_assert(M == 4096 || M == 2048 || M == 1024,
                  "three-pass schedules: radix 16 x 16 x P3, P3 = M / 256 = 16, 8 or 4");
    // M = 4096: one chunk per workgroup; M = 2048: two, chunk f on waves
    // 2f, 2f + 1; M = 1024: four, one per wave (a chunk past the end runs on
    // zeros and stores nothing)
    constexpr int LC = M / 16;            // lanes per chunk
    constexpr int P3 = M / 256;           // radix of pass 3
    const int L = threadIdx.x;
    // the chunk index is uniform over a wave: kept scalar (readfirstlane)
    const int f = M == 4096 ? 0 : __builtin_amdgcn_readfirstlane(L / LC);
    const int Lc = M == 4096 ? L : L % LC;
    const int chunk = M == 4096 ? cg : cg * (4096 / M) + f;
    const bool valid = M == 4096 || chunk < a.nchunks;   // one chunk: always in range
    const int cc = valid ? chunk : 0;
    const int c = cc % a.nchan;
    const int bs = cc / a.nchan;
    const int s = bs % a.nsub;
    const int b = bs / a.nsub;
    const int w = L >> 6, l45 = (L >> 4) & 3, l03 = L & 15;
    const int wc = w % (LC / 64);         // wave within the chunk

    // bins G0 + LC/16 G1 + LC q (G0 = l45 + 4 wc, G1 = l03), both pols,
    // increasing frequency; the transform input index is bin ^ (M / 2)
    const int base = l45 + 4 * wc + (LC / 16) * l03;
    cpair raw[16];
    {
        // the chunk as a raw buffer (uniform descriptor; no records for a
        // chunk past the end), row q at a scalar offset of 16 LC q bytes from
        // this lane's 32-bit offset
        const cpair *chunk = a.spec + (long long)bs * a.n + (long long)c * M;
        const __amdgpu_buffer_rsrc_t view = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<cpair *>(chunk), (short)0, valid ? M * 16 : 0, 0x00020000);
#pragma unroll
        for (int q = 0; q < 16; ++q)
            raw[q] = __builtin_bit_cast(
                cpair, __builtin_amdgcn_raw_buffer_load_b128(view, 16 * base, 16 * LC * q, 0));
    }

    // DM-independent part of Eq. 1 per bin (as in dm_item)
    const double fs = a.f_centre + ((double)s - 0.5 * (a.nsub - 1)) * a.bw;
    double nu0, off;
    int cofs;   // bin offset of the channel within the frequency axis of nu
    if (a.chirp_ref == 0) {
        nu0 = fs - 0.5 * a.bw + ((double)c + 0.5) * a.bw / a.nchan;
        off = -0.5 * M;
        cofs = 0;
    } else {
        nu0 = fs;
        off = -0.5 * a.n;
        cofs = c * M;
    }
    const double scale = 2.0 * a.sign * a.kk / (nu0 * nu0);
    double g2[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        // (the bin's index converted per item: a per-lane constant held
        // across a batch's items would cost 32 registers)
        const double nu = ((double)(base + LC * q + cofs) + off) * a.delta;
        g2[q] = scale * nu * nu / (nu0 + nu);
    }

    // pass 3's twiddles (DM-invariant): row Lc of the M_bin's table
    float2 tw2[16];
    {
        const float2 *tab = M == 4096 ? g_tw2 : M == 2048 ? g_tw2h : g_tw2q;
        const float4 *row = reinterpret_cast<const float4 *>(tab + 16 * Lc);
#pragma unroll
        for (int h = 0; h < 8; ++h) {
            const float4 x = row[h];
            tw2[2 * h] = make_float2(x.x, x.y);
            tw2[2 * h + 1] = make_float2(x.z, x.w);
        }
    }
    // pass 2's twiddle row G1, columns 2h, 2h + 1 at row1[TWS h]: from L1
    // (TWL = 0), or from the LDS copies after sh's kX3Lds bin pairs, written
    // here (TWL = 1) or by the caller before a barrier (TWL = 2)
    const float4 *row1;
    constexpr int TWS = TWL != 0 ? 16 : 1;
    if constexpr (TWL != 0) {
        if constexpr (TWL == 1) {
            put_tw1_lds(reinterpret_cast<float2 *>(sh + kX3Lds));
            __syncthreads();
        }
        row1 = reinterpret_cast<const float4 *>(sh + kX3Lds) + 144 * l45 + l03;
    } else {
        row1 = reinterpret_cast<const float4 *>(g_tw1 + 16 * l03);
    }

    // LDS: exchange 1 writes at xw + 17 k (row k of 17 slots, column l03 of
    // block (w, l45)) and reads at x1r + r (row l03, column r); exchange 2
    // writes at xw + 16 k (rows of 16) and reads at x2r + x2off(r): block
    // G0 = r mod P3 of the chunk's regions, row K1 = (Lc >> 4) + (LC / 16)
    // (r / P3), column K0 = l03 (at M = 4096: block r of the workgroup's
    // regions, row L >> 4).  The block pitch (272 = 16 mod 64 slots) and the
    // row pitches keep all 64 lanes of a wave on distinct 16-byte slots mod
    // 64 in every access.  At M = 1024 a chunk's exchanges stay within its
    // wave, so a wave-level fence replaces the workgroup barriers.
    cpair *const xw = sh + w * kX3Region + 272 * l45 + l03;
    const cpair *const x1r = sh + w * kX3Region + 272 * l45 + 17 * l03;
    const cpair *const x2r = sh + (LC / 64) * f * kX3Region + Lc;
    auto x2off = [](int r) {
        return kX3Region * ((r % P3) >> 2) + 272 * (r & 3) + LC * (r / P3);
    };
    auto xbarrier = []() {
        if constexpr (M == 1024)
            wave_lds_fence();
        else
            __syncthreads();
    };

    // output: this lane's samples after the sum over lane bits 0..K-1; column
    // of the channel in decreasing frequency
    const int col = (a.nsub - 1 - s) * a.nchan + (a.nchan - 1 - c);
    const int d0 = dt * a.dm_tile;
    const int d1 = min(a.ndm, d0 + a.dm_tile);

    float2 step[16];
    if constexpr (RECUR) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            raw[q] = cdmt::pmul(raw[q], cis_pi_f64(dms[d0] * g2[q]));
            step[q] = cis_pi_f64(a.dm_step * g2[q]);
        }
    }

    // One DM: the transform of rin (recurrence: rout = rin times the step).
    // The loop below alternates two register sets so that the recurrence
    // needs no copies at the loop edge.
    auto one_dm = [&](int d, cpair (&rin)[16], cpair (&rout)[16]) {
        cpair v[16];
        if constexpr (RECUR) {
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                // swap halves per channel: bin i -> transform input (i + M/2) mod M
                v[q ^ 8] = rin[q];
                rout[q] = cdmt::pmul(rin[q], step[q]);
            }
        } else {
            const double dm = dms[d];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const double t = dm * g2[q];
                const double n = rint(t);
                float sn, cs;
                sincos_pi(static_cast<float>(t - n), sn, cs);
                const int flip = static_cast<int>(n) << 31;
                sn = __int_as_float(__float_as_int(sn) ^ flip);
                cs = __int_as_float(__float_as_int(cs) ^ flip);
                v[q ^ 8] = cdmt::pmul(rin[q], make_float2(cs, sn));
            }
        }
        // back to normal wave priority (raised below for the second half)
        __builtin_amdgcn_s_setprio(0);
        // pass 2's twiddles (row G1), fetched while pass 1 runs
        float2 tw1[16];
#pragma unroll
        for (int h = 0; h < 8; ++h) {
            const float4 x = row1[TWS * h];
            tw1[2 * h] = make_float2(x.x, x.y);
            tw1[2 * h + 1] = make_float2(x.z, x.w);
        }
        // pass 1
        cdmt::dft16t<+1>(v);
#pragma unroll
        for (int k = 1; k < 16; ++k)
            v[k] = cdmt::pmul(v[k], tw1[k]);
        // exchange 1 (within the wave)
        xbarrier();
#pragma unroll
        for (int k = 0; k < 16; ++k)
            xw[17 * k] = v[k];
        wave_lds_fence();
#pragma unroll
        for (int r = 0; r < 16; ++r)
            v[r] = x1r[r];
        // pass 2
        cdmt::dft16t<+1>(v);
        // exchange 2 (across the waves), into this wave's region
        wave_lds_fence();
#pragma unroll
        for (int k = 0; k < 16; ++k)
            xw[16 * k] = v[k];
        xbarrier();
        // from exchange 2's reads to the stores this wave goes before the
        // CU's other waves of normal priority (measured 1% faster than
        // leaving the order to the arbiter)
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int r = 0; r < 16; ++r)
            v[r] = x2r[x2off(r)];
        // pass 3: 16 / P3 DFTs of P3 points over registers r mod P3 (r / P3
        // fixed); tw2 is 1 where r mod P3 = 0
#pragma unroll
        for (int r = 1; r < 16; ++r)
            if (r % P3 != 0)
                v[r] = cdmt::pmul(v[r], tw2[r]);
        if constexpr (P3 == 16) {
            cdmt::dft16t<+1>(v);
        } else {
#pragma unroll
            for (int h = 0; h < 16; h += P3)
                cdmt::dft<P3, +1>(v + h);
        }

        // detection: register q holds sample Lc + LC (q / P3) + 256 (q mod P3)
        // (at M = 4096: Lc + 256 q)
        float p[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const cpair y = v[q];
            p[q] = y.x * y.x + y.y * y.y + y.z * y.z + y.w * y.w;
        }
        const bool b0 = L & 1, b1 = (L >> 1) & 1, b2 = (L >> 2) & 1;
        // sum over the lane bits 0..K-1: remaining value r is the sum of
        // register q(r) over the 2^K lanes L & ~(2^K - 1) + x
        //   K = 0: q = r; K = 1: q = 2 r + L0; K = 2: q = 4 r + 2 L1 + L0;
        //   K = 3: q = 8 r + 4 L1 + 2 L0 + L2
        constexpr int NR = 16 >> K;
        float o[NR];
        if constexpr (K == 0) {
#pragma unroll
            for (int r = 0; r < 16; ++r)
                o[r] = p[r];
        } else if constexpr (K == 1) {
            fold<kDppX1, 8>(p, o, b0);
        } else if constexpr (K == 2) {
            float p1[8];
            fold<kDppX1, 8>(p, p1, b0);
            fold<kDppX2, 4>(p1, o, b1);
        } else {
            float p1[8], p2[4];
            fold<kDppX7, 8>(p, p1, b2);
            fold<kDppX1, 4>(p1, p2, b0);
            fold<kDppX2, 2>(p2, o, b1);
        }
        // first summed sample m of value r, then the filterbank sample
        // (m - n_d / 2) / ndec if it is kept
        const int mlane = Lc & ~((1 << K) - 1);
        float *out = a.out + (long long)d * a.ntime_out * a.nch_out +
                     (long long)b * a.tblk * a.t_stride + col * a.col_stride;
        // ndec <= 4 (4 to 16 values per lane): stores through a raw buffer
        // over this block's tblk samples of the column (the launch keeps its
        // byte extent under 2^31), a discarded sample at an offset past it,
        // which the range check drops: 32-bit offsets instead of 64-bit
        // addresses keep these forms from spilling.  ndec = 8 keeps plain
        // stores (measured 1% faster there).
        const __amdgpu_buffer_rsrc_t oview = __builtin_amdgcn_make_buffer_rsrc(
            out, (short)0, valid ? a.tblk * a.t_stride * 4 : 0, 0x00020000);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            int q;
            if constexpr (K == 0) q = r;
            else if constexpr (K == 1) q = 2 * r + (L & 1);
            else if constexpr (K == 2) q = 4 * r + 2 * ((L >> 1) & 1) + (L & 1);
            else q = 8 * r + 4 * ((L >> 1) & 1) + 2 * (L & 1) + ((L >> 2) & 1);
            const int m = mlane + LC * (q / P3) + 256 * (q % P3);
            const int tq = (m - a.nd_half) >> K;
            const bool keep = m >= a.nd_half && tq < a.tblk;
            if constexpr (K <= 2) {
                __builtin_amdgcn_raw_buffer_store_b32(
                    __float_as_uint(o[r]), oview, keep ? tq * a.t_stride * 4 : (int)0x80000000, 0, 0);
            } else {
                if (valid && keep)
                    out[(long long)tq * a.t_stride] = o[r];
            }
        }
    };
    if constexpr (RECUR) {
        cpair alt[16];
        for (int d = d0; d < d1; d += 2) {
            one_dm(d, raw, alt);
            if (d + 1 < d1)
                one_dm(d + 1, alt, raw);
        }
    } else {
        for (int d = d0; d < d1; ++d)
            one_dm(d, raw, raw);
    }
}

template <bool RECUR, int K, int M = 4096>
__global__ __launch_bounds__(256, 2) void fused_dedisperse_x3(FusedArgs a, DmList dl) {
    __shared__ cpair sh[kX3Lds + kX3TwLds];
    const int lw = xcd_remap(blockIdx.x, gridDim.x);
    const int ci = lw % a.inner;
    const int rest = lw / a.inner;
    const int dt = rest % a.ndt;
    const int cg = a.cg0 + (rest / a.ndt) * a.inner + ci;
    // the LDS twiddle table at ndec = 8 (measured 2.3% faster there; at
    // smaller ndec its registers would spill)
    dm_item_x3<RECUR, K, ArgDms, K == 3 ? 1 : 0, M>(a, ArgDms{dl}, dt, cg, sh);
}

// ---------------------------------------------------------------------------
// Split-precision matrix-core variant of the DM stage, M = 4096.
//
// Each radix-16 Stockham stage is the real 32x32 matrix
//   A = [[Fr, -Fi], [Fi, Fr]] / 16,   F[r][q] = exp(+2 pi i r q / 16),
// applied to 32 butterfly columns [Re x_0..15; Im x_0..15] with
// v_mfma_f32_32x32x16_{f16,bf16} (K = 16: one instruction for the real-input
// half of A, one for the imaginary-input half).  Both operands are split
// into hi + lo parts in the 16-bit type and A_hi B_hi + A_hi B_lo + A_lo B_hi
// accumulate in FP32.  Operand layouts (one wave, lane l, t = 0..7):
//   A: lane l holds A[l % 32][8 (l / 32) + t]
//   B: lane l holds B[8 (l / 32) + t][l % 32]
//   D: lane l, element v holds D[8 (v / 4) + 4 (l / 32) + v % 4][l % 32]
// so a lane owns inputs q = 8h + t (h = l / 32) of its column; the rows of A
// are permuted so that it owns outputs r = 8h + u (u = 0..7), real and
// imaginary parts in adjacent accumulator elements 2u, 2u + 1.  The 1/16 in A keeps every stage's
// operands within the first stage's range; a per-chunk power-of-two scale
// puts that range near 2^14 (exact, removed after detection), which keeps
// FP16 operands finite and their lo parts mostly normal.
//
// Work per workgroup (256 lanes, 4 waves): one channel chunk of 4096 bins and
// a tile of DMs.  Wave w, column c = l % 32 owns butterflies j_b = 64 w +
// 32 b + c (b = 0, 1) in both polarisations: four 32-column tiles per stage.

typedef _Float16 mx_h8 __attribute__((ext_vector_type(8)));
typedef __bf16 mx_b8 __attribute__((ext_vector_type(8)));
typedef _Float16 mx_h2 __attribute__((ext_vector_type(2)));
typedef __bf16 mx_b2 __attribute__((ext_vector_type(2)));
typedef float mx_f2 __attribute__((ext_vector_type(2)));
typedef float mx_f16 __attribute__((ext_vector_type(16)));

template <bool BF>
struct MxType;
template <>
struct MxType<false> {
    typedef mx_h8 v8;
    typedef mx_h2 v2;
    __device__ __forceinline__ static mx_f16 mma(v8 a, v8 b, mx_f16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};
template <>
struct MxType<true> {
    typedef mx_b8 v8;
    typedef mx_b2 v2;
    __device__ __forceinline__ static mx_f16 mma(v8 a, v8 b, mx_f16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};

// lo = f16(x - hi) for a pair (x0, x1) whose f16 parts are packed in hi:
// FP32 fused multiply-add with an FP16 operand, result rounded into one half
// of the destination (v_fma_mixlo_f16 / v_fma_mixhi_f16); x - hi is exact.
__device__ __forceinline__ mx_h2 mx_residual_f16(mx_h2 hi, float x0, float x1) {
    unsigned r;
    const unsigned hb = __builtin_bit_cast(unsigned, hi);
    asm volatile("v_fma_mixlo_f16 %0, %1, -1.0, %2 op_sel_hi:[1,0,0]"
                 : "=v"(r) : "v"(hb), "v"(x0));
    asm volatile("v_fma_mixhi_f16 %0, %1, -1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]"
                 : "+v"(r) : "v"(hb), "v"(x1));
    return __builtin_bit_cast(mx_h2, r);
}

// x = hi + lo in the 16-bit type (lo carries the rounding residual of hi),
// converted two values at a time (packed conversions)
template <bool BF>
__device__ __forceinline__ void mx_split(const float (&x)[8], typename MxType<BF>::v8 &hi,
                                         typename MxType<BF>::v8 &lo) {
    typedef typename MxType<BF>::v2 V2;
    V2 h[4], l[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const mx_f2 v = {x[2 * p], x[2 * p + 1]};
        h[p] = __builtin_convertvector(v, V2);
        if constexpr (BF) {
            const mx_f2 hf = __builtin_convertvector(h[p], mx_f2);
            l[p] = __builtin_convertvector(v - hf, V2);
        } else {
            l[p] = mx_residual_f16(h[p], x[2 * p], x[2 * p + 1]);
        }
    }
    hi = __builtin_shufflevector(__builtin_shufflevector(h[0], h[1], 0, 1, 2, 3),
                                 __builtin_shufflevector(h[2], h[3], 0, 1, 2, 3), 0, 1, 2, 3, 4,
                                 5, 6, 7);
    lo = __builtin_shufflevector(__builtin_shufflevector(l[0], l[1], 0, 1, 2, 3),
                                 __builtin_shufflevector(l[2], l[3], 0, 1, 2, 3), 0, 1, 2, 3, 4,
                                 5, 6, 7);
}

// D = A B for one 32-column tile: re/im are the lane's 8 inputs
template <bool BF>
__device__ __forceinline__ mx_f16 mx_dft16(const float (&re)[8], const float (&im)[8],
                                           const typename MxType<BF>::v8 (&a)[4]) {
    typedef MxType<BF> X;
    typename X::v8 rh, rl, ih, il;
    mx_split<BF>(re, rh, rl);
    mx_split<BF>(im, ih, il);
    mx_f16 d = {};
    d = X::mma(a[0], rh, d);    // A_hi(real-input block) B_hi
    d = X::mma(a[0], rl, d);    // A_hi B_lo
    d = X::mma(a[1], rh, d);    // A_lo B_hi
    d = X::mma(a[2], ih, d);    // imaginary-input block
    d = X::mma(a[2], il, d);
    d = X::mma(a[3], ih, d);
    return d;
}

template <bool RECUR, bool BF>
__global__ __launch_bounds__(256, 2) void fused_dedisperse_mx(FusedArgs a, DmList dl) {
    constexpr int M = 4096;
    constexpr int PL = M + M / 16 + 1;              // LDS plane per polarisation (float2)
    __shared__ float2 sh[2 * PL];
    __shared__ float red[4];

    const int lw = xcd_remap(blockIdx.x, gridDim.x);
    const int ci = lw % a.inner;
    const int rest = lw / a.inner;
    const int dt = rest % a.ndt;
    const int chunk = a.cg0 + (rest / a.ndt) * a.inner + ci;
    const int c = chunk % a.nchan;
    const int bs = chunk / a.nchan;
    const int s = bs % a.nsub;
    const int b = bs / a.nsub;

    const int t_id = threadIdx.x;
    const int w = t_id >> 6, l = t_id & 63;
    const int col = l & 31, h = l >> 5;
    int jb[2];
    jb[0] = 64 * w + col;
    jb[1] = jb[0] + 32;

    // A = F/16 split into hi/lo: a[0..1] real-input block hi/lo, a[2..3] imaginary.
    // Row i of A is ordered so that accumulator element v of a lane in half hl
    // (row 8 (v/4) + 4 hl + v % 4) holds the real (v even) or imaginary (v odd)
    // part of output r = 8 hl + v/2: each (Re, Im) pair is two adjacent registers.
    typename MxType<BF>::v8 amat[4];
    {
        const int i = l & 31;
        const int vv = 4 * (i >> 3) + (i & 3);
        const int r = 8 * ((i >> 2) & 1) + (vv >> 1);
        const bool im_row = (vv & 1) != 0;
        float re_blk[8], im_blk[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int q = 8 * h + t;
            const float fr = cdmt::c16(r * q) * 0.0625f, fi = cdmt::s16(r * q) * 0.0625f;
            re_blk[t] = im_row ? fi : fr;
            im_blk[t] = im_row ? fr : -fi;
        }
        mx_split<BF>(re_blk, amat[0], amat[1]);
        mx_split<BF>(im_blk, amat[2], amat[3]);
    }

    // this lane's bins: transform inputs q = 8h + t of butterflies j_b, i.e.
    // spectrum bins (after the swap of halves) i = j_b + 256 ((8h + t) ^ 8)
    cpair raw[2][8];
    const cpair *src = a.spec + (long long)bs * a.n + (long long)c * M;
#pragma unroll
    for (int bb = 0; bb < 2; ++bb)
#pragma unroll
        for (int t = 0; t < 8; ++t)
            raw[bb][t] = src[jb[bb] + 256 * ((8 * h + t) ^ 8)];

    // per-chunk power-of-two scale: max component -> about 2^14
    float mx = 0.f;
#pragma unroll
    for (int bb = 0; bb < 2; ++bb)
#pragma unroll
        for (int t = 0; t < 8; ++t)
            mx = fmaxf(mx, fmaxf(fmaxf(fabsf(raw[bb][t].x), fabsf(raw[bb][t].y)),
                                 fmaxf(fabsf(raw[bb][t].z), fabsf(raw[bb][t].w))));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        mx = fmaxf(mx, __shfl_xor(mx, o));
    if (l == 0)
        red[w] = mx;
    __syncthreads();
    mx = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    int ex = 0;
    if (mx > 0.f) {
        ex = 14 - ilogbf(mx);
        ex = ex > 60 ? 60 : (ex < -60 ? -60 : ex);
    }
    const float up = ldexpf(1.0f, ex);
    // |y|^2 = |y_computed|^2 * 16^6 * 2^(-2 ex)
    const float down = ldexpf(1.0f, 24 - 2 * ex);
#pragma unroll
    for (int bb = 0; bb < 2; ++bb)
#pragma unroll
        for (int t = 0; t < 8; ++t)
            raw[bb][t] = cdmt::pscale(raw[bb][t], up);

    // DM-independent part of Eq. 1 per bin, as in fused_dedisperse
    const double fs = a.f_centre + ((double)s - 0.5 * (a.nsub - 1)) * a.bw;
    double nu0, off;
    if (a.chirp_ref == 0) {
        nu0 = fs - 0.5 * a.bw + ((double)c + 0.5) * a.bw / a.nchan;
        off = -0.5 * M;
    } else {
        nu0 = fs;
        off = (double)c * M - 0.5 * a.n;
    }
    const double scale = 2.0 * a.sign * a.kk / (nu0 * nu0);
    double g2[2][8];
#pragma unroll
    for (int bb = 0; bb < 2; ++bb)
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int bin = jb[bb] + 256 * ((8 * h + t) ^ 8);
            const double nu = ((double)bin + off) * a.delta;
            g2[bb][t] = scale * nu * nu / (nu0 + nu);
        }

    const int d0 = dt * a.dm_tile;
    const int d1 = min(a.ndm, d0 + a.dm_tile);
    float2 step[2][8];
    if constexpr (RECUR) {
#pragma unroll
        for (int bb = 0; bb < 2; ++bb)
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                raw[bb][t] = cdmt::pmul(raw[bb][t], cis_pi_f64(dl.dm[d0] * g2[bb][t]));
                step[bb][t] = cis_pi_f64(a.dm_step * g2[bb][t]);
            }
    }

    float *inten = reinterpret_cast<float *>(sh);
    const int colo = (a.nsub - 1 - s) * a.nchan + (a.nchan - 1 - c);

    // LDS addresses (float2 index, before the pol-Y plane offset PL) of this
    // lane's tile 0; tile 1 (butterfly j + 32) adds a constant.  With the
    // padding e + e/16 the Stockham indices reduce to:
    //   stage-0 outputs   e = 16 j + r                 -> 17 j + r
    //   stage-1 outputs   e = 256 (j/16) + j%16 + 16 r -> 272 (j/16) + j%16 + 17 r
    //   stage-1/2 inputs  e = j + 256 q                -> j + j/16 + 272 q
    // with r = 8h + u, q = 8h + t.
    const int j0 = jb[0];
    const int wr0 = 17 * j0 + 8 * h;                          // + u, tile 1: + 544
    const int wr1 = 272 * (j0 >> 4) + (j0 & 15) + 136 * h;    // + 17 u, tile 1: + 544
    const int rd = j0 + (j0 >> 4) + 2176 * h;                 // + 272 t, tile 1: + 34
    // stage-1 twiddle row k = j % 16 is the same for both tiles; stage 2: k = j
    const float4 *tw1p =
        reinterpret_cast<const float4 *>(cdmt::stage_table<16>(256) + (j0 & 15) * 16 + 8 * h);
    const float4 *tw2p =
        reinterpret_cast<const float4 *>(cdmt::stage_table<16>(4096) + j0 * 16 + 8 * h);

    typedef typename MxType<BF>::v8 V8;
    typedef MxType<BF> X;
    // B operands of one tile: [pol][re hi, re lo, im hi, im lo]; two sets so
    // that one tile's matrix products overlap the other tile's conversions
    V8 opa[2][4], opb[2][4];
    auto split_tile = [&](V8 (&op)[2][4], const cpair (&x)[8]) {
        float xr[8], xi[8], yr[8], yi[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            xr[t] = x[t].x;
            xi[t] = x[t].y;
            yr[t] = x[t].z;
            yi[t] = x[t].w;
        }
        mx_split<BF>(xr, op[0][0], op[0][1]);
        mx_split<BF>(xi, op[0][2], op[0][3]);
        mx_split<BF>(yr, op[1][0], op[1][1]);
        mx_split<BF>(yi, op[1][2], op[1][3]);
    };
    // both polarisations of one tile, the two accumulation chains interleaved
    // so consecutive matrix instructions are independent
    auto mma_tile = [&](const V8 (&op)[2][4], mx_f16 &dx, mx_f16 &dy) {
        dx = mx_f16{};
        dy = mx_f16{};
        dx = X::mma(amat[0], op[0][0], dx);   // A_hi B_hi, real inputs
        dy = X::mma(amat[0], op[1][0], dy);
        dx = X::mma(amat[0], op[0][1], dx);   // A_hi B_lo
        dy = X::mma(amat[0], op[1][1], dy);
        dx = X::mma(amat[1], op[0][0], dx);   // A_lo B_hi
        dy = X::mma(amat[1], op[1][0], dy);
        dx = X::mma(amat[2], op[0][2], dx);   // imaginary inputs
        dy = X::mma(amat[2], op[1][2], dy);
        dx = X::mma(amat[2], op[0][3], dx);
        dy = X::mma(amat[2], op[1][3], dy);
        dx = X::mma(amat[3], op[0][2], dx);
        dy = X::mma(amat[3], op[1][2], dy);
    };
    auto read_tile = [&](int base, cpair (&x)[8]) {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const float2 xx = sh[base + 272 * t];
            const float2 yy = sh[PL + base + 272 * t];
            x[t] = make_float4(xx.x, xx.y, yy.x, yy.y);
        }
    };
    auto twiddle_tile = [&](cpair (&x)[8], const float4 (&tw)[4]) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            x[2 * u] = cdmt::pmul(x[2 * u], make_float2(tw[u].x, tw[u].y));
            x[2 * u + 1] = cdmt::pmul(x[2 * u + 1], make_float2(tw[u].z, tw[u].w));
        }
    };
    auto load_tw = [&](const float4 *p, float4 (&tw)[4]) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
            tw[u] = p[u];
    };
    // the chirped spectrum of tile bb for DM d (exact transfer function)
    auto chirp_tile = [&](int bb, double dm, cpair (&x)[8]) {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const double tt = dm * g2[bb][t];
            const double n = rint(tt);
            float sn, cs;
            sincos_pi(static_cast<float>(tt - n), sn, cs);
            const int flip = static_cast<int>(n) << 31;
            sn = __int_as_float(__float_as_int(sn) ^ flip);
            cs = __int_as_float(__float_as_int(cs) ^ flip);
            x[t] = cdmt::pmul(raw[bb][t], make_float2(cs, sn));
        }
    };
    auto detect_tile = [&](int j, const mx_f16 &dx, const mx_f16 &dy) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const float re0 = dx[2 * u], im0 = dx[2 * u + 1];
            const float re1 = dy[2 * u], im1 = dy[2 * u + 1];
            inten[j + 256 * (8 * h + u)] = (re0 * re0 + im0 * im0 + re1 * re1 + im1 * im1) * down;
        }
    };

    for (int d = d0; d < d1; ++d) {
        mx_f16 dx, dy;
        cpair x0[8], x1[8];
        float4 tw1[4], tw2[4];
        load_tw(tw1p, tw1);               // stage 1's twiddles; latency covered by stage 0

        // stage 0: inputs are the chirped spectrum
        if constexpr (RECUR) {
            split_tile(opa, raw[0]);
        } else {
            chirp_tile(0, dl.dm[d], x0);
            split_tile(opa, x0);
        }
        mma_tile(opa, dx, dy);
        if constexpr (RECUR) {
            split_tile(opb, raw[1]);
#pragma unroll
            for (int t = 0; t < 8; ++t)
                pmul_inplace(raw[0][t], step[0][t]);
        } else {
            chirp_tile(1, dl.dm[d], x1);
            split_tile(opb, x1);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            sh[wr0 + u] = make_float2(dx[2 * u], dx[2 * u + 1]);
            sh[PL + wr0 + u] = make_float2(dy[2 * u], dy[2 * u + 1]);
        }
        mma_tile(opb, dx, dy);
        if constexpr (RECUR) {
#pragma unroll
            for (int t = 0; t < 8; ++t)
                pmul_inplace(raw[1][t], step[1][t]);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            sh[wr0 + 544 + u] = make_float2(dx[2 * u], dx[2 * u + 1]);
            sh[PL + wr0 + 544 + u] = make_float2(dy[2 * u], dy[2 * u + 1]);
        }
        __syncthreads();

        // stage 1
        read_tile(rd, x0);
        read_tile(rd + 34, x1);
        twiddle_tile(x0, tw1);
        split_tile(opa, x0);
        twiddle_tile(x1, tw1);
        split_tile(opb, x1);
        __syncthreads();
        {
            // tile 0's stores overlap tile 1's matrix products
            mx_f16 ex, ey;
            mma_tile(opa, dx, dy);
            mma_tile(opb, ex, ey);
            load_tw(tw2p, tw2);           // stage 2, tile 0: latency covered by the stores
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                sh[wr1 + 17 * u] = make_float2(dx[2 * u], dx[2 * u + 1]);
                sh[PL + wr1 + 17 * u] = make_float2(dy[2 * u], dy[2 * u + 1]);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                sh[wr1 + 544 + 17 * u] = make_float2(ex[2 * u], ex[2 * u + 1]);
                sh[PL + wr1 + 544 + 17 * u] = make_float2(ey[2 * u], ey[2 * u + 1]);
            }
        }
        __syncthreads();

        // stage 2, then detection into LDS (every lane has read its inputs)
        read_tile(rd, x0);
        read_tile(rd + 34, x1);
        twiddle_tile(x0, tw2);
        load_tw(tw2p + 32 * 8, tw2);      // tile 1: row j + 32, 8 float4 a row
        split_tile(opa, x0);
        twiddle_tile(x1, tw2);
        split_tile(opb, x1);
        __syncthreads();
        {
            // tile 0's detection overlaps tile 1's matrix products
            mx_f16 ex, ey;
            mma_tile(opa, dx, dy);
            mma_tile(opb, ex, ey);
            detect_tile(j0, dx, dy);
            detect_tile(j0 + 32, ex, ey);
        }
        __syncthreads();
        {
            float *o = a.out + (long long)d * a.ntime_out * a.nch_out +
                       (long long)b * a.tblk * a.t_stride + colo * a.col_stride;
            if (((a.ndec | a.nd_half) & 3) == 0) {
                const int n4 = a.ndec >> 2;
                for (int tq = t_id; tq < a.tblk; tq += 256) {
                    const float4 *p = reinterpret_cast<const float4 *>(inten + a.nd_half) + tq * n4;
                    float acc = 0.f;
                    for (int q = 0; q < n4; ++q) {
                        const float4 x = p[q];
                        acc += (x.x + x.y) + (x.z + x.w);
                    }
                    o[(long long)tq * a.t_stride] = acc;
                }
            } else {
                for (int tq = t_id; tq < a.tblk; tq += 256) {
                    const float *p = inten + a.nd_half + tq * a.ndec;
                    float acc = 0.f;
                    for (int q = 0; q < a.ndec; ++q)
                        acc += p[q];
                    o[(long long)tq * a.t_stride] = acc;
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Derivative with respect to DM of L = sum G * F (G = dL/dF given by the
// caller for every filterbank sample), for refining a candidate's DM: the
// adjoint of the per-DM chain, each step reversed in turn.  Per chunk and
// DM, with S' = S H the chirped spectrum (exact transfer function, H =
// exp(i pi DM g2)):
//   y = backward FFT of swap(S')            (forward pass, kept in registers)
//   g_y = 2 (dL/dI) y, dL/dI[m] = G at the output sample holding m (0 on
//         the discarded edges)              (detection and downsampling)
//   g_z = forward FFT (e^{-}) of g_y        (adjoint of the e^{+} transform)
//   dL/dDM = sum Re(conj(g_S') i pi g2 S'), g_S' = unswap(g_z), both pols.
// One workgroup per (chunk group, DM); FP64 partial sums per workgroup,
// reduced per DM in a fixed order by dm_grad_sum (deterministic).  Work is
// ordered (subband block, DM, chunk group within the subband block): the
// channels of one subband block at one DM are neighbours on one XCD, so the
// G rows they read ([t][ch], one column each) are shared in its L2, and the
// block's spectra stay there across its DMs.  a.inner = chunk groups per
// subband block (1 when a group spans several subbands).
template <int M>
__global__ __launch_bounds__(256, 2) void dm_grad(FusedArgs a, DmList dl,
                                                  const float *__restrict__ gout,
                                                  double *__restrict__ part, long long ncg_all,
                                                  int dm_first) {
    using Sh = FusedShape<M, 16>;
    constexpr int R = 16;
    constexpr int T = Sh::T;
    constexpr int C = Sh::C;
    constexpr int STRIDE = Sh::STRIDE;
    static_assert(Sh::WG == 256, "256-lane workgroups");
    __shared__ cpair sh[C * STRIDE];
    __shared__ double red[4];

    const int lw = xcd_remap(blockIdx.x, gridDim.x);
    const int gin = lw % a.inner, rest = lw / a.inner;
    const int d = rest % a.ndm;
    const int cg = a.cg0 + (rest / a.ndm) * a.inner + gin;
    const int t = threadIdx.x;
    const int f = t / T, tt = t % T;
    const int chunk = cg * C + f;
    const bool valid = chunk < a.nchunks;
    const int cc = valid ? chunk : 0;
    const int c = cc % a.nchan;
    const int bs = cc / a.nchan;
    const int s = bs % a.nsub;
    const int b = bs / a.nsub;

    const cpair *src = a.spec + (long long)bs * a.n + (long long)c * M;
    const double fs = a.f_centre + ((double)s - 0.5 * (a.nsub - 1)) * a.bw;
    double nu0, off;
    if (a.chirp_ref == 0) {
        nu0 = fs - 0.5 * a.bw + ((double)c + 0.5) * a.bw / a.nchan;
        off = -0.5 * M;
    } else {
        nu0 = fs;
        off = (double)c * M - 0.5 * a.n;
    }
    const double scale = 2.0 * a.sign * a.kk / (nu0 * nu0);
    const double dm = dl.dm[d];
    // the chirped spectrum S' is needed again after both transforms: keep the
    // transfer function (one complex float per bin) and reload the spectrum
    // then, rather than hold S' (two) through the transforms
    double g2[R];
    float2 h[R];
    cpair v[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const double nu = ((double)(tt + T * q) + off) * a.delta;
        g2[q] = scale * nu * nu / (nu0 + nu);
        const double ph = dm * g2[q];
        const double n = rint(ph);
        float sn, cs;
        sincos_pi(static_cast<float>(ph - n), sn, cs);
        const int flip = static_cast<int>(n) << 31;
        sn = __int_as_float(__float_as_int(sn) ^ flip);
        cs = __int_as_float(__float_as_int(cs) ^ flip);
        const cpair r = valid ? src[tt + T * q] : make_float4(0.f, 0.f, 0.f, 0.f);
        h[q] = make_float2(cs, sn);
        v[q ^ (R / 2)] = cdmt::pmul(r, h[q]);
    }
    const cdmt::LdsPad<R> lds{sh + f * STRIDE};
    cdmt::wg_fft<M, +1>(v, tt, lds);               // y, sample m = tt + T q

    const int col = (a.nsub - 1 - s) * a.nchan + (a.nchan - 1 - c);
    const float *g = gout + (long long)d * a.ntime_out * a.nch_out +
                     (long long)b * a.tblk * a.t_stride + col * a.col_stride;
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int m = tt + T * q;
        float gi = 0.f;
        if (valid && m >= a.nd_half && m < M - a.nd_half)
            gi = g[(long long)((m - a.nd_half) / a.ndec) * a.t_stride];
        v[q] = cdmt::pscale(v[q], 2.0f * gi);
    }
    __syncthreads();                               // the first transform's LDS reads are done
    cdmt::wg_fft<M, -1>(v, tt, lds);               // g_z, bin j = tt + T q

    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const cpair gz = v[q ^ (R / 2)];           // g_S' of this lane's bin q
        const cpair r = valid ? src[tt + T * q] : make_float4(0.f, 0.f, 0.f, 0.f);
        const cpair x = cdmt::pmul(r, h[q]);       // S', as before the transforms
        const float tx = gz.y * x.x - gz.x * x.y;  // Re(conj(g) i S'), pol X
        const float ty = gz.w * x.z - gz.z * x.w;  // pol Y
        acc = fma(g2[q], (double)tx + (double)ty, acc);
    }
    if (!valid)
        acc = 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        acc += __shfl_xor(acc, o);
    if ((t & 63) == 0)
        red[t >> 6] = acc;
    __syncthreads();
    if (t == 0)
        part[(long long)(dm_first + d) * ncg_all + cg] = (red[0] + red[1]) + (red[2] + red[3]);
}

// The DM gradient at M_bin = 4096 on the three-pass transforms (any ndec).
// Per DM of the workgroup's tile: the chirped spectrum S' (exact transfer
// function) is transformed as in dm_item_x3 (register q of lane L ends with
// sample m = L + 256 q); g_y = 2 G y on the kept samples; then the adjoint
// transform (e-) takes the passes in reverse digit order,
//   input m = M0 + 16 M1 + 256 M2 (M0 = L & 15, M1 = L >> 4, M2 = q),
//   pass 1  DFT over M2 -> registers J0; twiddle w256^-(M1 J0)
//   exchange A (across the waves, the transpose of exchange 2): registers
//           <- M1, lane digit L >> 4 <- J0
//   pass 2  DFT over M1 -> registers J1
//   exchange B (within the wave, the transpose of exchange 1): registers
//           <- M0, lane digit L & 15 <- J1
//   pass 3  twiddle w4096^-(M0 (J0 + 16 J1)), DFT over M0 -> registers J2
// so register q of lane L holds g_x at index j = (L >> 4) + 16 (L & 15) +
// 256 q, which is the bin the lane loaded into register q ^ 8 (the swap of
// halves).  The per-bin terms Re(conj(g_S') i S') g2 are summed in FP64.
// Exchange B writes into the slots its own wave read in exchange A, so the
// next DM's exchange 1 needs no barrier: three barriers per DM.  The lane's
// bins of the spectrum stay in registers for the whole DM tile (they do not
// depend on the DM); the transfer function is evaluated twice per DM, for the
// forward transform and for the final product, which costs less than
// re-reading the spectrum from L2 each DM.
constexpr int kGradTile = 64;

template <int TILE>
__global__ __launch_bounds__(256, 2) void dm_grad_x3(FusedArgs a, DmList dl,
                                                     const float *__restrict__ gout,
                                                     double *__restrict__ part, long long ncg_all,
                                                     int dm_first) {
    constexpr int M = 4096;
    __shared__ cpair sh[kX3Lds + kX3TwLds];
    __shared__ double red[4][TILE];
    const int lw = xcd_remap(blockIdx.x, gridDim.x);
    const int ci = lw % a.inner;
    const int rest = lw / a.inner;
    const int dt = rest % a.ndt;
    const int cg = a.cg0 + (rest / a.ndt) * a.inner + ci;
    const int L = threadIdx.x;
    const int c = cg % a.nchan;
    const int bs = cg / a.nchan;
    const int s = bs % a.nsub;
    const int b = bs / a.nsub;
    const int w = L >> 6, l45 = (L >> 4) & 3, l03 = L & 15;
    const int base = l45 + 4 * w + 16 * l03;
    // the chunk as a raw buffer (uniform descriptor) and this lane's byte
    // offset: the load of row q adds 4096 q bytes as a scalar offset, so no
    // per-row addresses are held
    const cpair *chunk = a.spec + (long long)bs * a.n + (long long)c * M;
    const __amdgpu_buffer_rsrc_t spec_view =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<cpair *>(chunk), (short)0, M * 16, 0x00020000);
    const int lane_off = 16 * base;

    const double fs = a.f_centre + ((double)s - 0.5 * (a.nsub - 1)) * a.bw;
    double nu0, off;
    int cofs;
    if (a.chirp_ref == 0) {
        nu0 = fs - 0.5 * a.bw + ((double)c + 0.5) * a.bw / a.nchan;
        off = -0.5 * M;
        cofs = 0;
    } else {
        nu0 = fs;
        off = -0.5 * a.n;
        cofs = c * M;
    }
    const double scale = 2.0 * a.sign * a.kk / (nu0 * nu0);
    double g2[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const double nu = ((double)(base + 256 * q + cofs) + off) * a.delta;
        g2[q] = scale * nu * nu / (nu0 + nu);
    }

    cpair *const xw = sh + w * kX3Region + 272 * l45 + l03;
    const cpair *const x1r = sh + w * kX3Region + 272 * l45 + 17 * l03;
    cpair *const x2 = sh + 16 * (L >> 4) + l03;
    // the w256 twiddle table (rows G1 forward, J0 adjoint) from its LDS copies,
    // as in dm_item_x3 (slot stride 16 between column pairs); the w4096 rows
    // are read through L1 (stride 1)
    put_tw1_lds(reinterpret_cast<float2 *>(sh + kX3Lds));
    __syncthreads();
    const float4 *const twq = reinterpret_cast<const float4 *>(sh + kX3Lds);
    const float4 *const r1 = twq + 144 * l45 + l03;
    const float4 *const r2 = reinterpret_cast<const float4 *>(g_tw2 + 16 * L);
    const float4 *const r1b = twq + 144 * (l03 & 3) + (L >> 4);
    const float4 *const r2b =
        reinterpret_cast<const float4 *>(g_tw2 + 16 * ((L >> 4) + 16 * l03));
    const int col = (a.nsub - 1 - s) * a.nchan + (a.nchan - 1 - c);
    const int d0 = dt * a.dm_tile;
    const int d1 = min(a.ndm, d0 + a.dm_tile);
    // filterbank sample of m = L + 256 q within the block, two 16-bit values
    // per register (0xffff: m is discarded, the n_d / 2 samples at either edge)
    unsigned tpk[8];
#pragma unroll
    for (int q = 0; q < 16; q += 2) {
        const int m0 = L + 256 * q, m1 = m0 + 256;
        const unsigned t0 = (m0 >= a.nd_half && m0 < M - a.nd_half) ? (m0 - a.nd_half) / a.ndec : 0xffffu;
        const unsigned t1 = (m1 >= a.nd_half && m1 < M - a.nd_half) ? (m1 - a.nd_half) / a.ndec : 0xffffu;
        tpk[q / 2] = t0 | (t1 << 16);
    }

    // twiddle multiply from a row of 8 float4 (conjugated for the adjoint)
    auto twiddle = [](cpair (&v)[16], const float4 *row, int stride, bool conj) {
#pragma unroll
        for (int h = 0; h < 8; ++h) {
            const float4 x = row[stride * h];
            const float sy = conj ? -1.f : 1.f;
            if (h > 0)
                v[2 * h] = cdmt::pmul(v[2 * h], make_float2(x.x, sy * x.y));
            v[2 * h + 1] = cdmt::pmul(v[2 * h + 1], make_float2(x.z, sy * x.w));
        }
    };

    // the lane's 16 bins of the spectrum, loaded once for the whole DM tile
    cpair xs[16];
#pragma unroll
    for (int q = 0; q < 16; ++q)
        xs[q] = __builtin_bit_cast(
            cpair, __builtin_amdgcn_raw_buffer_load_b128(spec_view, lane_off, 4096 * q, 0));
    // the exact transfer function of bin q at this DM (Eq. 1), evaluated at
    // the start of the DM and again for the final product rather than held
    auto chirp = [&](double dm, int q) {
        const double ph = dm * g2[q];
        const double n = rint(ph);
        float sn, cs;
        sincos_pi(static_cast<float>(ph - n), sn, cs);
        const int flip = static_cast<int>(n) << 31;
        return make_float2(__int_as_float(__float_as_int(cs) ^ flip),
                           __int_as_float(__float_as_int(sn) ^ flip));
    };

    for (int d = d0; d < d1; ++d) {
        const double dm = dl.dm[d];
        // the chirped spectrum S' of this DM
        cpair v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q)
            v[q ^ 8] = cdmt::pmul(xs[q], chirp(dm, q));
        // y: pass 1, exchange 1 (within the wave), pass 2, exchange 2
        cdmt::dft16t<+1>(v);
        twiddle(v, r1, 16, false);
#pragma unroll
        for (int k = 0; k < 16; ++k)
            xw[17 * k] = v[k];
        wave_lds_fence();
#pragma unroll
        for (int r = 0; r < 16; ++r)
            v[r] = x1r[r];
        cdmt::dft16t<+1>(v);
        wave_lds_fence();
#pragma unroll
        for (int k = 0; k < 16; ++k)
            xw[16 * k] = v[k];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 16; ++r)
            v[r] = x2[kX3Region * (r >> 2) + 272 * (r & 3)];
        twiddle(v, r2, 1, false);
        cdmt::dft16t<+1>(v);
        // g_y = 2 G y on the kept samples m = L + 256 q
        const float *g = gout + (long long)d * a.ntime_out * a.nch_out +
                         (long long)b * a.tblk * a.t_stride + col * a.col_stride;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const unsigned tq = (q & 1) ? tpk[q / 2] >> 16 : tpk[q / 2] & 0xffffu;
            const bool kept = tq != 0xffffu;
            const float gi = g[(kept ? tq : 0u) * a.t_stride];
            v[q] = cdmt::pscale(v[q], kept ? 2.0f * gi : 0.f);
        }
        // g_x: pass 1 (e-), exchange A (across the waves)
        cdmt::dft16t<-1>(v);
        twiddle(v, r1b, 16, true);
        __syncthreads();                   // every wave has read exchange 2
#pragma unroll
        for (int k = 0; k < 16; ++k)
            x2[kX3Region * (k >> 2) + 272 * (k & 3)] = v[k];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 16; ++r)
            v[r] = xw[16 * r];
        // pass 2, exchange B (within the wave, the slots read in exchange A)
        cdmt::dft16t<-1>(v);
        wave_lds_fence();
#pragma unroll
        for (int k = 0; k < 16; ++k)
            xw[17 * k] = v[k];
        wave_lds_fence();
#pragma unroll
        for (int r = 0; r < 16; ++r)
            v[r] = x1r[r];
        twiddle(v, r2b, 1, true);
        cdmt::dft16t<-1>(v);
        // sum over this lane's bins of g2 Re(conj(g_S') i S'), both pols; the
        // DM is passed through an empty asm so that the compiler evaluates the
        // transfer function here again instead of holding the first one
        double dmr = dm;
        asm volatile("" : "+s"(dmr));
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const cpair gz = v[q ^ 8];
            const cpair x = cdmt::pmul(xs[q], chirp(dmr, q));
            const float tx = gz.y * x.x - gz.x * x.y;
            const float ty = gz.w * x.z - gz.z * x.w;
            acc = fma(g2[q], (double)tx + (double)ty, acc);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
            acc += __shfl_xor(acc, o);
        if ((L & 63) == 0)
            red[w][d - d0] = acc;
    }
    __syncthreads();
    if (L < d1 - d0)
        part[(long long)(dm_first + d0 + L) * ncg_all + cg] =
            (red[0][L] + red[1][L]) + (red[2][L] + red[3][L]);
}

// Gradient with respect to the voltages, one DM: the adjoint continued
// through the transfer function and the forward stage.  dv_spec forms, per
// chunk, g_spec = g_S' conj(H) as dm_grad does, and stores conj(g_spec) / N
// with the subband's halves swapped back: the conjugated, unswapped
// spectrum gradient.  The forward kernels then transform it as if it were a
// stream of voltages (one block per subband-block, no overlap), which gives
// the e^{+} transform that the adjoint needs up to conjugation, the half swap
// and 1/N; dv_gather undoes those and overlap-adds the blocks.
template <int M>
__global__ __launch_bounds__(256, 2) void dv_spec(FusedArgs a, double dm,
                                                  const float *__restrict__ gout,
                                                  cpair *__restrict__ gin) {
    using Sh = FusedShape<M, 16>;
    constexpr int R = 16;
    constexpr int T = Sh::T;
    constexpr int C = Sh::C;
    constexpr int STRIDE = Sh::STRIDE;
    static_assert(Sh::WG == 256, "256-lane workgroups");
    __shared__ cpair sh[C * STRIDE];

    const int cg = a.cg0 + xcd_remap(blockIdx.x, gridDim.x);
    const int t = threadIdx.x;
    const int f = t / T, tt = t % T;
    const int chunk = cg * C + f;
    const bool valid = chunk < a.nchunks;
    const int cc = valid ? chunk : 0;
    const int c = cc % a.nchan;
    const int bs = cc / a.nchan;
    const int s = bs % a.nsub;
    const int b = bs / a.nsub;

    const cpair *src = a.spec + (long long)bs * a.n + (long long)c * M;
    const double fs = a.f_centre + ((double)s - 0.5 * (a.nsub - 1)) * a.bw;
    double nu0, off;
    if (a.chirp_ref == 0) {
        nu0 = fs - 0.5 * a.bw + ((double)c + 0.5) * a.bw / a.nchan;
        off = -0.5 * M;
    } else {
        nu0 = fs;
        off = (double)c * M - 0.5 * a.n;
    }
    const double scale = 2.0 * a.sign * a.kk / (nu0 * nu0);
    float2 hq[R];
    cpair v[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const double nu = ((double)(tt + T * q) + off) * a.delta;
        const double ph = dm * (scale * nu * nu / (nu0 + nu));
        const double n = rint(ph);
        float sn, cs;
        sincos_pi(static_cast<float>(ph - n), sn, cs);
        const int flip = static_cast<int>(n) << 31;
        hq[q] = make_float2(__int_as_float(__float_as_int(cs) ^ flip),
                            __int_as_float(__float_as_int(sn) ^ flip));
        const cpair r = valid ? src[tt + T * q] : make_float4(0.f, 0.f, 0.f, 0.f);
        v[q ^ (R / 2)] = cdmt::pmul(r, hq[q]);
    }
    const cdmt::LdsPad<R> lds{sh + f * STRIDE};
    cdmt::wg_fft<M, +1>(v, tt, lds);                         // y

    const int col = (a.nsub - 1 - s) * a.nchan + (a.nchan - 1 - c);
    const float *g = gout + (long long)b * a.tblk * a.t_stride + col * a.col_stride;
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int m = tt + T * q;
        float gi = 0.f;
        if (valid && m >= a.nd_half && m < M - a.nd_half)
            gi = g[(long long)((m - a.nd_half) / a.ndec) * a.t_stride];
        v[q] = cdmt::pscale(v[q], 2.0f * gi);
    }
    __syncthreads();
    cdmt::wg_fft<M, -1>(v, tt, lds);                         // g_z

    if (!valid)
        return;
    const float inv_n = 1.0f / (float)a.n;
    cpair *dst = gin + (long long)bs * a.n;
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const cpair gz = v[q ^ (R / 2)];                      // g_S' of bin j
        // conj(g_S' conj(H)) / N = conj(g_S') H / N, both pols
        const cpair cg_ = make_float4(gz.x, -gz.y, gz.z, -gz.w);
        const cpair val = cdmt::pscale(cdmt::pmul(cg_, hq[q]), inv_n);
        const long long j = (long long)c * M + tt + T * q;
        dst[(j + a.n / 2) & (a.n - 1)] = val;
    }
}

// gx[s][t] (both pols) = sum over the blocks covering sample t of
// N conj(out[block][s][(t - start + N/2) mod N]), added to gx if accumulate
__global__ __launch_bounds__(256) void dv_gather(const cpair *__restrict__ out, int nsub, int nfft,
                                                 int step, int nblock, long long ntime,
                                                 float4 *__restrict__ gx, int accumulate) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)nsub * ntime)
        return;
    const int s = (int)(i / ntime);
    const long long t = i - (long long)s * ntime;
    long long blo = t - nfft + 1 <= 0 ? 0 : (t - nfft + 1 + step - 1) / step;
    long long bhi = t / step;
    if (bhi > nblock - 1)
        bhi = nblock - 1;
    float4 acc = accumulate ? gx[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    const float fn = (float)nfft;
    for (long long b = blo; b <= bhi; ++b) {
        const long long n = t - b * step;
        const cpair o = out[(b * nsub + s) * (long long)nfft + ((n + nfft / 2) & (nfft - 1))];
        acc.x += fn * o.x;
        acc.y -= fn * o.y;
        acc.z += fn * o.z;
        acc.w -= fn * o.w;
    }
    gx[i] = acc;
}

// dL/dDM[d] = pi * sum over chunk groups of the partials, fixed order
__global__ __launch_bounds__(256) void dm_grad_sum(const double *__restrict__ part, long long ncg,
                                                   double *__restrict__ dldm) {
    __shared__ double red[4];
    const int d = blockIdx.x;
    double acc = 0.0;
    for (long long i = threadIdx.x; i < ncg; i += 256)
        acc += part[(long long)d * ncg + i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        acc += __shfl_xor(acc, o);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0)
        dldm[d] = M_PI * ((red[0] + red[1]) + (red[2] + red[3]));
}

// ---------------------------------------------------------------------------
// Batches: several beams, each with its own plan (subbands, N_bin, channels,
// overlap), input, DM list and output, through the FP32 DM stage in one
// persistent launch per M_bin present and per form of the transfer function
// (recurrence for arithmetic DM lists, else exact): one launch when every
// beam has the same M_bin and arithmetic DM lists.  Work items are (beam, chunk group, DM tile); items are
// numbered beam by beam, and within a beam with the DM tiles of a chunk
// group consecutive (so they share the chunk in L2).  The item range is split
// into one contiguous queue per XCD; workgroup w serves queue w % 8 (the
// dispatcher places workgroups on XCDs round-robin) and takes items from it
// with an atomic counter until the queue is exhausted, so every workgroup
// exits once its queue is drained.

struct BatchBeam {
    FusedArgs a;            // the beam's DM-stage arguments (cg0 = 0)
    long long item0;        // first work item of the beam within its launch
    const double *dms;      // the beam's DM list in device memory
};

constexpr int kBatchQueues = 8;
// launch groups: 7 M_bin x 2 transfer-function forms, plus the three-pass
// item's 4 downsampling factors x 2 forms at M_bin 1024, 2048 and 4096, plus
// the radix-8 item (8 bins per lane) x 2 forms at M_bin 2048 and 4096; each
// group has kBatchQueues counters in the batch workspace
constexpr int kBatchGroups = 7 * 2 + 3 * 4 * 2 + 2 * 2;

__global__ void batch_reset(unsigned long long *ctr, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        ctr[i] = 0;
}

// K >= 0: the three-pass item (dm_item_x3, M_bin 4096, 2048 or 1024) with ndec = 2^K
// R = 8: the radix-8 Stockham item (8 bins per lane; 512-lane workgroups at
// M_bin = 4096, 256 at 2048)
template <int M, bool RECUR, int K = -1, int R = 16>
__global__ __launch_bounds__((FusedShape<M, R>::WG), (R == 8 ? 4 : 2)) void dm_batch(
    const BatchBeam *__restrict__ beams, int nbeam, long long total,
    unsigned long long *__restrict__ ctr) {
    using Sh = FusedShape<M, R>;
    static_assert(R == 8 || Sh::WG == 256, "radix-16 batched launches use 256-lane workgroups");
    static_assert(K < 0 || ((M == 4096 || M == 2048 || M == 1024) && R == 16),
                  "the three-pass item is built for M_bin 4096, 2048 and 1024");
    __shared__ cpair sh[K >= 0 ? kX3Lds + kX3TwLds : Sh::C * Sh::STRIDE];
    // the three-pass item at ndec = 8 reads pass 2's twiddles from LDS copies
    // written once here (first read after the loop's first barrier)
    if constexpr (K == 3)
        put_tw1_lds(reinterpret_cast<float2 *>(sh + kX3Lds));
    __shared__ long long s_item;
    const int q = blockIdx.x % kBatchQueues;
    const long long lo = total * q / kBatchQueues;
    const long long hi = total * (q + 1) / kBatchQueues;
    for (;;) {
        if (threadIdx.x == 0)
            s_item = lo + (long long)atomicAdd(&ctr[q], 1ULL);
        __syncthreads();
        // the same value in every lane: keep it (and all that follows from it) scalar
        const unsigned long long raw_item = (unsigned long long)s_item;
        const long long item = (long long)(
            ((unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)(raw_item >> 32)) << 32) |
            (unsigned)__builtin_amdgcn_readfirstlane((unsigned)raw_item));
        __syncthreads();
        if (item >= hi)
            break;
        int b = 0;
        while (b + 1 < nbeam && beams[b + 1].item0 <= item)
            ++b;
        const FusedArgs a = beams[b].a;          // a copy: the fields are read once, into SGPRs
        const long long local = item - beams[b].item0;
        const int ci = (int)(local % a.inner);
        const long long rest = local / a.inner;
        const int dt = (int)(rest % a.ndt);
        const int cg = (int)((rest / a.ndt) * a.inner + ci);
        if constexpr (K >= 0)
            dm_item_x3<RECUR, K, MemDms, K == 3 ? 2 : 0, M>(a, MemDms{beams[b].dms}, dt, cg, sh);
        else
            dm_item<M, R, RECUR>(a, MemDms{beams[b].dms}, dt, cg, sh);
    }
}

// ---------------------------------------------------------------------------
// Host side.

std::mutex g_init_mu;
std::vector<char> g_init_done;   // per device

// Library-owned scratch of cdmt_dm_gradient_noalloc: the FP64 partial sums
// that cdmt_dm_gradient keeps in the caller's gradient workspace.  Each GPU
// holds its own copy until the process ends.  Host code never names the
// array itself (on the host the name is only a stand-in): it uses the device
// address fetched once per device in ensure_twiddles.
constexpr size_t kScratchBytes = size_t(16) << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];
std::vector<void *> g_scratch_ptr;   // per device, from hipGetSymbolAddress

int ensure_twiddles() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return CDMT_E_DEVICE;
    std::lock_guard<std::mutex> lk(g_init_mu);
    if ((int)g_init_done.size() <= dev) {
        g_init_done.resize(dev + 1, 0);
        g_scratch_ptr.resize(dev + 1, nullptr);
    }
    if (g_init_done[dev])
        return CDMT_OK;
    void *sp = nullptr;
    if (hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)) != hipSuccess || !sp)
        return CDMT_E_DEVICE;
    g_scratch_ptr[dev] = sp;
    std::vector<float2> h(kTwiddleEntries);
    h[0] = make_float2(1.f, 0.f);
    for (int p = 1; p < kTwiddleEntries; p <<= 1) {
        for (int n = 0; n < p; ++n) {
            // exp(+2 pi i n / p); the angle is formed from the exact fraction
            const double a = 2.0 * M_PI * ((double)n / (double)p);
            h[p + n] = make_float2((float)std::cos(a), (float)std::sin(a));
        }
    }
    if (hipMemcpyToSymbol(HIP_SYMBOL(g_twiddle), h.data(), sizeof(float2) * h.size()) !=
        hipSuccess)
        return CDMT_E_DEVICE;
    // row tables: family r, table for sub-transform length L at entry L,
    // row k = exp(+2 pi i k q / L), q < r
    std::vector<float2> st(4 * cdmt::kStageFamily, make_float2(0.f, 0.f));
    for (int fam = 0; fam < 4; ++fam) {
        const int r = 2 << fam;
        for (int len = r; len < cdmt::kStageFamily; len <<= 1) {
            for (int k = 0; k < len / r; ++k) {
                for (int q = 0; q < r; ++q) {
                    const long long e = ((long long)k * q) % len;
                    const double a = 2.0 * M_PI * ((double)e / (double)len);
                    st[fam * cdmt::kStageFamily + len + k * r + q] =
                        make_float2((float)std::cos(a), (float)std::sin(a));
                }
            }
        }
    }
    if (hipMemcpyToSymbol(HIP_SYMBOL(cdmt::g_stage_tw), st.data(),
                          sizeof(float2) * st.size()) != hipSuccess)
        return CDMT_E_DEVICE;
    // the three-pass schedules: pass 2 [g][k] = exp(+2 pi i g k / 256); pass 3
    // at M_bin 4096 [l][r] = exp(+2 pi i r l / 4096), at M_bin 2048 [l][r] =
    // exp(+2 pi i (r & 7)(l + 128 (r >> 3)) / 2048), at M_bin 1024 [l][r] =
    // exp(+2 pi i (r & 3)(l + 64 (r >> 2)) / 1024), at M_bin 1024 [l][r] =
    // exp(+2 pi i (r & 3)(l + 64 (r >> 2)) / 1024)
    std::vector<float2> t1(16 * 16), t2(256 * 16), t2h(128 * 16), t2q(64 * 16);
    for (int g = 0; g < 16; ++g)
        for (int k = 0; k < 16; ++k) {
            const double ang = 2.0 * M_PI * ((double)((g * k) % 256) / 256.0);
            t1[16 * g + k] = make_float2((float)std::cos(ang), (float)std::sin(ang));
        }
    for (int l = 0; l < 256; ++l)
        for (int r = 0; r < 16; ++r) {
            const double ang = 2.0 * M_PI * ((double)((l * r) % 4096) / 4096.0);
            t2[16 * l + r] = make_float2((float)std::cos(ang), (float)std::sin(ang));
        }
    for (int l = 0; l < 128; ++l)
        for (int r = 0; r < 16; ++r) {
            const int e = ((r & 7) * (l + 128 * (r >> 3))) % 2048;
            const double ang = 2.0 * M_PI * ((double)e / 2048.0);
            t2h[16 * l + r] = make_float2((float)std::cos(ang), (float)std::sin(ang));
        }
    for (int l = 0; l < 64; ++l)
        for (int r = 0; r < 16; ++r) {
            const int e = ((r & 3) * (l + 64 * (r >> 2))) % 1024;
            const double ang = 2.0 * M_PI * ((double)e / 1024.0);
            t2q[16 * l + r] = make_float2((float)std::cos(ang), (float)std::sin(ang));
        }
    if (hipMemcpyToSymbol(HIP_SYMBOL(g_tw1), t1.data(), sizeof(float2) * t1.size()) !=
            hipSuccess ||
        hipMemcpyToSymbol(HIP_SYMBOL(g_tw2), t2.data(), sizeof(float2) * t2.size()) !=
            hipSuccess ||
        hipMemcpyToSymbol(HIP_SYMBOL(g_tw2h), t2h.data(), sizeof(float2) * t2h.size()) !=
            hipSuccess ||
        hipMemcpyToSymbol(HIP_SYMBOL(g_tw2q), t2q.data(), sizeof(float2) * t2q.size()) !=
            hipSuccess)
        return CDMT_E_DEVICE;
    g_init_done[dev] = 1;
    return CDMT_OK;
}


}  // namespace


namespace {

template <int P>
void launch_col(const FwdArgs &a, int ci8, int grid, hipStream_t st) {
    if (ci8)
        fwd_col<P, true><<<grid, 256, 0, st>>>(a);
    else
        fwd_col<P, false><<<grid, 256, 0, st>>>(a);
}


int launch_forward(const cdmt_plan_s *p, void *ws, const void *x, int nblock, hipStream_t st) {
    const long long nspec = (long long)nblock * p->nsub * p->nfft;
    FwdArgs a;
    a.x = x;
    a.spec = reinterpret_cast<cpair *>(ws);
    a.ybuf = a.spec + nspec;
    a.ntime_in = (long long)nblock * (p->nfft - p->noverlap) + p->noverlap;
    a.nsub = p->nsub;
    a.nblock = nblock;
    a.n1 = p->n1;
    a.n2 = p->n2;
    a.n = p->nfft;
    a.step = p->nfft - p->noverlap;
    a.inv_n = 1.0f / (float)p->nfft;

    const long long bsn = (long long)nblock * p->nsub;
    if (p->nfft <= 2048) {
        const int C = 4096 / p->nfft;
        const long long grid = (bsn + C - 1) / C;
        if (grid * 256 > 0xffffffffLL)
            return CDMT_E_SHAPE;
        const bool ci8 = p->input_kind != 0;
        if (p->nfft == 1024)
            ci8 ? fwd_one<1024, true><<<(int)grid, 256, 0, st>>>(a)
                : fwd_one<1024, false><<<(int)grid, 256, 0, st>>>(a);
        else if (p->nfft == 2048)
            ci8 ? fwd_one<2048, true><<<(int)grid, 256, 0, st>>>(a)
                : fwd_one<2048, false><<<(int)grid, 256, 0, st>>>(a);
        else
            return CDMT_E_UNSUPPORTED;
        return hipGetLastError() == hipSuccess ? CDMT_OK : CDMT_E_DEVICE;
    }
    const long long gcol = bsn * (p->n1 / (4096 / p->n2));
    const long long grow = bsn * (p->n2 / (4096 / p->n1));
    // a dispatch covers at most 2^32 - 1 work-items
    if (gcol * 256 > 0xffffffffLL || grow * 256 > 0xffffffffLL)
        return CDMT_E_SHAPE;
    switch (p->n2) {
    case 64: launch_col<64>(a, p->input_kind, (int)gcol, st); break;
    case 128: launch_col<128>(a, p->input_kind, (int)gcol, st); break;
    case 256: launch_col<256>(a, p->input_kind, (int)gcol, st); break;
    default: return CDMT_E_UNSUPPORTED;
    }
    switch (p->n1) {
    case 64: fwd_row<64><<<(int)grow, 256, 0, st>>>(a); break;
    case 128: fwd_row<128><<<(int)grow, 256, 0, st>>>(a); break;
    case 256: fwd_row<256><<<(int)grow, 256, 0, st>>>(a); break;
    case 512: fwd_row<512><<<(int)grow, 256, 0, st>>>(a); break;
    default: return CDMT_E_UNSUPPORTED;
    }
    return hipGetLastError() == hipSuccess ? CDMT_OK : CDMT_E_DEVICE;
}



// The three-pass schedules (M_bin 4096, 2048, 1024) sum ndec = 2^K samples across lanes
// aligned to multiples of ndec: K for this launch, or -1 when the plan needs
// the general kernel (other ndec, n_d / 2 not a multiple of ndec, a block's
// column spanning 2^31 bytes or more, or the schedule switched off).
int x3_k(const FusedArgs &a) {
    if (a.schedule != 0 || 4LL * a.tblk * a.t_stride >= 0x80000000LL)
        return -1;
    for (int k = 0; k <= 3; ++k)
        if (a.ndec == (1 << k))
            return a.nd_half % a.ndec == 0 ? k : -1;
    return -1;
}

template <int M>
void launch_x3(bool recur, int k, int grid, const FusedArgs &a, const DmList &dl,
              hipStream_t st) {
    switch (k + (recur ? 4 : 0)) {
    case 0: fused_dedisperse_x3<false, 0, M><<<grid, 256, 0, st>>>(a, dl); break;
    case 1: fused_dedisperse_x3<false, 1, M><<<grid, 256, 0, st>>>(a, dl); break;
    case 2: fused_dedisperse_x3<false, 2, M><<<grid, 256, 0, st>>>(a, dl); break;
    case 3: fused_dedisperse_x3<false, 3, M><<<grid, 256, 0, st>>>(a, dl); break;
    case 4: fused_dedisperse_x3<true, 0, M><<<grid, 256, 0, st>>>(a, dl); break;
    case 5: fused_dedisperse_x3<true, 1, M><<<grid, 256, 0, st>>>(a, dl); break;
    case 6: fused_dedisperse_x3<true, 2, M><<<grid, 256, 0, st>>>(a, dl); break;
    default: fused_dedisperse_x3<true, 3, M><<<grid, 256, 0, st>>>(a, dl); break;
    }
}

// A dispatch covers at most 2^32 - 1 work-items, so large jobs are split into
// several launches: by DM (at most kMaxDmPerLaunch per launch, passed by
// value) and, when the grid would still be too large, by chunk groups.
// MX = 0: FP32 vector path; 1: BF16x3 and 2: FP16x3 matrix-core path (M = 4096)
template <int M, int R, int MX = 0>
int launch_fused_m(const FusedArgs &a0, const double *dms, int ndm, hipStream_t st) {
    constexpr int WG = MX ? 256 : FusedShape<M, R>::WG;
    constexpr int C = MX ? 1 : FusedShape<M, R>::C;
    constexpr long long kMaxGroups = 0xffffffffLL / WG;
    const long long ncg = (a0.nchunks + C - 1) / C;
    const int inner = a0.nchan >= C ? a0.nchan / C : 1;
    for (int first = 0; first < ndm; first += kMaxDmPerLaunch) {
        FusedArgs a = a0;
        const int cnt = ndm - first < kMaxDmPerLaunch ? ndm - first : kMaxDmPerLaunch;
        DmList dl;
        std::memset(&dl, 0, sizeof(dl));
        for (int i = 0; i < cnt; ++i)
            dl.dm[i] = dms[first + i];
        a.ndm = cnt;
        a.out = a0.out + (long long)first * a0.ntime_out * a0.nch_out;
        a.inner = inner;
        a.ndt = (cnt + a.dm_tile - 1) / a.dm_tile;
        const bool recur = a0.dm_step != 0.0 && a.dm_tile > 1 && cnt > 1 &&
                           arithmetic(dl.dm, cnt, a0.dm_step);
        a.dm_step = recur ? dl.dm[1] - dl.dm[0] : 0.0;
        long long per = kMaxGroups / a.ndt / inner * inner;   // chunk groups per launch
        if (per < inner)
            return CDMT_E_SHAPE;
        for (long long cg0 = 0; cg0 < ncg; cg0 += per) {
            const long long n = ncg - cg0 < per ? ncg - cg0 : per;
            a.cg0 = (int)cg0;
            const int grid = (int)(n * a.ndt);
            if constexpr (MX != 0) {
                static_assert(M == 4096, "matrix-core path is built for M = 4096");
                constexpr bool BF = MX == 1;
                if (recur)
                    fused_dedisperse_mx<true, BF><<<grid, WG, 0, st>>>(a, dl);
                else
                    fused_dedisperse_mx<false, BF><<<grid, WG, 0, st>>>(a, dl);
            } else if ((M == 4096 || M == 2048 || M == 1024) && R == 16 && x3_k(a) >= 0) {
                launch_x3<(M == 4096 || M == 2048 ? M : 1024)>(recur, x3_k(a), grid, a, dl, st);
            } else {
                if (recur)
                    fused_dedisperse<M, R, true><<<grid, WG, 0, st>>>(a, dl);
                else
                    fused_dedisperse<M, R, false><<<grid, WG, 0, st>>>(a, dl);
            }
            if (hipGetLastError() != hipSuccess)
                return CDMT_E_DEVICE;
        }
    }
    return CDMT_OK;
}

FusedArgs fused_args(const cdmt_plan_s *p, void *ws, int nblock, float *out) {
    FusedArgs a;
    std::memset(&a, 0, sizeof(a));
    a.spec = reinterpret_cast<const cpair *>(ws);
    a.out = out;
    a.ntime_out = (long long)nblock * p->tblk;
    a.nsub = p->nsub;
    a.nchan = p->nchan;
    a.n = p->nfft;
    a.nchunks = nblock * p->nsub * p->nchan;
    a.dm_tile = p->dm_tile;
    a.nd_half = p->nd / 2;
    a.ndec = p->ndec;
    a.tblk = p->tblk;
    a.nch_out = p->nsub * p->nchan;
    a.t_stride = p->out_layout ? 1 : a.nch_out;
    a.col_stride = p->out_layout ? a.ntime_out : 1;
    a.chirp_ref = p->chirp_ref;
    a.sign = (float)p->sign;
    a.f_centre = p->f_centre;
    a.bw = p->bw;
    a.delta = p->bw / p->nfft;
    a.kk = 1e6 * kKdm;
    a.schedule = p->fft_schedule;
    // recurrence allowed when every DM sits on the progression to within a
    // phase error of 1e-7 half-cycles (dm_step carries the tolerance here)
    a.dm_step = p->chirp_exact ? 0.0 : 1e-7 / max_half_cycles_per_dm(p);
    return a;
}

int launch_dedisperse(const cdmt_plan_s *p, void *ws, int nblock, const double *dms, int ndm,
                      float *out, hipStream_t st) {
    const FusedArgs a = fused_args(p, ws, nblock, out);
    const bool r8 = p->lane_bins == 8;
    switch (p->m) {
    case 64: return launch_fused_m<64, 16>(a, dms, ndm, st);
    case 128: return launch_fused_m<128, 16>(a, dms, ndm, st);
    case 256: return launch_fused_m<256, 16>(a, dms, ndm, st);
    case 512: return launch_fused_m<512, 16>(a, dms, ndm, st);
    case 1024: return launch_fused_m<1024, 16>(a, dms, ndm, st);
    case 2048: return r8 ? launch_fused_m<2048, 8>(a, dms, ndm, st)
                         : launch_fused_m<2048, 16>(a, dms, ndm, st);
    case 4096:
        if (p->precision == 1)
            return launch_fused_m<4096, 16, 1>(a, dms, ndm, st);
        if (p->precision == 2)
            return launch_fused_m<4096, 16, 2>(a, dms, ndm, st);
        return r8 ? launch_fused_m<4096, 8>(a, dms, ndm, st)
                  : launch_fused_m<4096, 16>(a, dms, ndm, st);
    case 8192: return launch_fused_m<8192, 16>(a, dms, ndm, st);
    default: return CDMT_E_UNSUPPORTED;
    }
}

template <int M>
int launch_grad_m(const FusedArgs &a0, const double *dms, int ndm, const float *gout, double *part,
                  long long ncg, double *dldm, hipStream_t st) {
    constexpr long long kMaxGroups = 0xffffffffLL / 256;
    for (int first = 0; first < ndm; first += kMaxDmPerLaunch) {
        FusedArgs a = a0;
        const int cnt = ndm - first < kMaxDmPerLaunch ? ndm - first : kMaxDmPerLaunch;
        DmList dl;
        std::memset(&dl, 0, sizeof(dl));
        for (int i = 0; i < cnt; ++i)
            dl.dm[i] = dms[first + i];
        a.ndm = cnt;
        const float *g = gout + (long long)first * a0.ntime_out * a0.nch_out;
        // chunk groups per subband block (the launch order keeps a block's
        // groups together), and launches cut at multiples of it
        const int C = 4096 / M;
        a.inner = a0.nchan >= C ? a0.nchan / C : 1;
        if (M == 4096 && a0.schedule == 0 && (long long)a0.tblk * a0.t_stride < 0x7fffffffLL) {
            // three-pass kernel, DM tiles of kGradTile
            a.dm_tile = kGradTile;
            a.ndt = (cnt + kGradTile - 1) / kGradTile;
            const long long per = kMaxGroups / a.ndt / a.inner * a.inner;
            for (long long cg0 = 0; cg0 < ncg; cg0 += per) {
                const long long n = ncg - cg0 < per ? ncg - cg0 : per;
                a.cg0 = (int)cg0;
                dm_grad_x3<kGradTile><<<(unsigned)(n * a.ndt), 256, 0, st>>>(a, dl, g, part, ncg,
                                                                            first);
                if (hipGetLastError() != hipSuccess)
                    return CDMT_E_DEVICE;
            }
            continue;
        }
        const long long per = kMaxGroups / cnt / a.inner * a.inner;
        for (long long cg0 = 0; cg0 < ncg; cg0 += per) {
            const long long n = ncg - cg0 < per ? ncg - cg0 : per;
            a.cg0 = (int)cg0;
            dm_grad<M><<<(unsigned)(n * cnt), 256, 0, st>>>(a, dl, g, part, ncg, first);
            if (hipGetLastError() != hipSuccess)
                return CDMT_E_DEVICE;
        }
    }
    dm_grad_sum<<<ndm, 256, 0, st>>>(part, ncg, dldm);
    return hipGetLastError() == hipSuccess ? CDMT_OK : CDMT_E_DEVICE;
}

template <int M>
int launch_dv_m(const FusedArgs &a0, double dm, const float *gout, cpair *gin, long long ncg,
                hipStream_t st) {
    constexpr long long kMaxGroups = 0xffffffffLL / 256;
    FusedArgs a = a0;
    for (long long cg0 = 0; cg0 < ncg; cg0 += kMaxGroups) {
        const long long n = ncg - cg0 < kMaxGroups ? ncg - cg0 : kMaxGroups;
        a.cg0 = (int)cg0;
        dv_spec<M><<<(unsigned)n, 256, 0, st>>>(a, dm, gout, gin);
        if (hipGetLastError() != hipSuccess)
            return CDMT_E_DEVICE;
    }
    return CDMT_OK;
}


// cdmt_dm_gradient with the partial sums in the caller's workspace gws, or
// (use_scratch) in this device's library-owned scratch array.
int dm_gradient(cdmt_plan_t p, void *ws, size_t ws_bytes, int nblock, const double *dm_list,
                int ndm, const float *grad_out, void *gws, size_t gws_bytes, bool use_scratch,
                double *dldm, void *hip_stream) {
    int st = check_call(p, ws, ws_bytes, nblock);
    if (st)
        return st;
    if (ndm < 0)
        return CDMT_E_ARG;
    if (p->m > 4096)
        return CDMT_E_UNSUPPORTED;
    if (ndm == 0 || nblock == 0)
        return CDMT_OK;
    if (!dm_list || !grad_out || (!use_scratch && !gws) || !dldm)
        return CDMT_E_ARG;
    if ((st = check_dms(p, dm_list, ndm)))
        return st;
    size_t need = 0;
    cdmt_gradient_workspace_size(p, nblock, ndm, &need);
    if (gws_bytes < need)
        return CDMT_E_WORKSPACE;
    if ((st = ensure_twiddles()))
        return st;
    if (use_scratch) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess)
            return CDMT_E_DEVICE;
        std::lock_guard<std::mutex> lk(g_init_mu);
        gws = g_scratch_ptr[dev];
    }
    const FusedArgs a = fused_args(p, ws, nblock, nullptr);
    const long long ncg = grad_groups(p, nblock);
    double *part = static_cast<double *>(gws);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    switch (p->m) {
    case 64: return launch_grad_m<64>(a, dm_list, ndm, grad_out, part, ncg, dldm, s);
    case 128: return launch_grad_m<128>(a, dm_list, ndm, grad_out, part, ncg, dldm, s);
    case 256: return launch_grad_m<256>(a, dm_list, ndm, grad_out, part, ncg, dldm, s);
    case 512: return launch_grad_m<512>(a, dm_list, ndm, grad_out, part, ncg, dldm, s);
    case 1024: return launch_grad_m<1024>(a, dm_list, ndm, grad_out, part, ncg, dldm, s);
    case 2048: return launch_grad_m<2048>(a, dm_list, ndm, grad_out, part, ncg, dldm, s);
    case 4096: return launch_grad_m<4096>(a, dm_list, ndm, grad_out, part, ncg, dldm, s);
    default: return CDMT_E_UNSUPPORTED;
    }
}


}  // namespace

extern "C" {


int cdmt_forward(cdmt_plan_t p, void *ws, size_t ws_bytes, const void *voltages, int nblock,
                 void *hip_stream) {
    int st = check_call(p, ws, ws_bytes, nblock);
    if (st)
        return st;
    if (nblock == 0)
        return CDMT_OK;
    if (!voltages)
        return CDMT_E_ARG;
    if ((st = ensure_twiddles()))
        return st;
    return launch_forward(p, ws, voltages, nblock, (hipStream_t)hip_stream);
}

int cdmt_dedisperse_spectra(cdmt_plan_t p, void *ws, size_t ws_bytes, int nblock,
                            const double *dm_list, int ndm, float *out, void *hip_stream) {
    int st = check_call(p, ws, ws_bytes, nblock);
    if (st)
        return st;
    if (ndm < 0)
        return CDMT_E_ARG;
    if (ndm == 0 || nblock == 0)
        return CDMT_OK;
    if (!dm_list || !out)
        return CDMT_E_ARG;
    if ((st = check_dms(p, dm_list, ndm)))
        return st;
    if ((st = ensure_twiddles()))
        return st;
    return launch_dedisperse(p, ws, nblock, dm_list, ndm, out, (hipStream_t)hip_stream);
}

int cdmt_dedisperse(cdmt_plan_t p, void *ws, size_t ws_bytes, const void *voltages, int nblock,
                    const double *dm_list, int ndm, float *out, void *hip_stream) {
    int st = check_call(p, ws, ws_bytes, nblock);
    if (st)
        return st;
    if (ndm < 0)
        return CDMT_E_ARG;
    if (ndm == 0 || nblock == 0)
        return CDMT_OK;
    if (!voltages || !dm_list || !out)
        return CDMT_E_ARG;
    if ((st = check_dms(p, dm_list, ndm)))
        return st;
    if ((st = cdmt_forward(p, ws, ws_bytes, voltages, nblock, hip_stream)))
        return st;
    return cdmt_dedisperse_spectra(p, ws, ws_bytes, nblock, dm_list, ndm, out, hip_stream);
}


int cdmt_dm_gradient(cdmt_plan_t p, void *ws, size_t ws_bytes, int nblock, const double *dm_list,
                     int ndm, const float *grad_out, void *gws, size_t gws_bytes, double *dldm,
                     void *hip_stream) {
    return dm_gradient(p, ws, ws_bytes, nblock, dm_list, ndm, grad_out, gws, gws_bytes, false, dldm,
                       hip_stream);
}


int cdmt_dm_gradient_noalloc(cdmt_plan_t p, void *ws, size_t ws_bytes, int nblock,
                             const double *dm_list, int ndm, const float *grad_out, double *dldm,
                             void *hip_stream) {
    return dm_gradient(p, ws, ws_bytes, nblock, dm_list, ndm, grad_out, nullptr, kScratchBytes, true,
                       dldm, hip_stream);
}


size_t cdmt_noalloc_scratch_bytes(void) { return kScratchBytes; }


int cdmt_voltage_gradient(cdmt_plan_t p, void *ws, size_t ws_bytes, int nblock, double dm,
                          const float *grad_out, void *gws, size_t gws_bytes, float *grad_v,
                          int accumulate, void *hip_stream) {
    int st = check_call(p, ws, ws_bytes, nblock);
    if (st)
        return st;
    if (p->m > 4096)
        return CDMT_E_UNSUPPORTED;
    if (accumulate != 0 && accumulate != 1)
        return CDMT_E_ARG;
    if (nblock == 0)
        return CDMT_OK;
    if (!grad_out || !gws || !grad_v)
        return CDMT_E_ARG;
    if ((st = check_dms(p, &dm, 1)))
        return st;
    size_t need = 0;
    cdmt_voltage_gradient_workspace_size(p, nblock, &need);
    if (gws_bytes < need)
        return CDMT_E_WORKSPACE;
    if ((st = ensure_twiddles()))
        return st;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const FusedArgs a = fused_args(p, ws, nblock, nullptr);
    const long long ncg = grad_groups(p, nblock);
    cpair *gin = static_cast<cpair *>(gws);
    const long long nspec = (long long)nblock * p->nsub * p->nfft;
    switch (p->m) {
    case 64: st = launch_dv_m<64>(a, dm, grad_out, gin, ncg, s); break;
    case 128: st = launch_dv_m<128>(a, dm, grad_out, gin, ncg, s); break;
    case 256: st = launch_dv_m<256>(a, dm, grad_out, gin, ncg, s); break;
    case 512: st = launch_dv_m<512>(a, dm, grad_out, gin, ncg, s); break;
    case 1024: st = launch_dv_m<1024>(a, dm, grad_out, gin, ncg, s); break;
    case 2048: st = launch_dv_m<2048>(a, dm, grad_out, gin, ncg, s); break;
    case 4096: st = launch_dv_m<4096>(a, dm, grad_out, gin, ncg, s); break;
    default: return CDMT_E_UNSUPPORTED;
    }
    if (st)
        return st;
    // the forward kernels on the spectrum gradient: every subband-block as
    // one block of its own subband, float32 input, no overlap
    cdmt_plan_s q = *p;
    q.nsub = nblock * p->nsub;
    q.noverlap = 0;
    q.input_kind = 0;
    cpair *fws = gin + nspec;
    if ((st = launch_forward(&q, fws, gin, 1, s)))
        return st;
    const long long ntime = (long long)nblock * (p->nfft - p->noverlap) + p->noverlap;
    const long long items = (long long)p->nsub * ntime;
    dv_gather<<<(unsigned)((items + 255) / 256), 256, 0, s>>>(
        fws, p->nsub, p->nfft, p->nfft - p->noverlap, nblock, ntime,
        reinterpret_cast<float4 *>(grad_v), accumulate);
    return hipGetLastError() == hipSuccess ? CDMT_OK : CDMT_E_DEVICE;
}


}  // extern "C"

// ---------------------------------------------------------------------------
// Batches of beams (host side).

struct cdmt_batch_s {
    std::vector<cdmt_beam_t> beams;           // the caller's descriptors
    std::vector<std::vector<double>> dms;     // host copies of the DM lists
    std::vector<size_t> spec_off;             // per beam: spectra in the workspace
    std::vector<int> fwd_n2;                  // per beam: forward split (0: the plan's)
    std::vector<int> fft_sched;               // per beam: DM-stage schedule (-1: the plan's)
    std::vector<int> lane_bins;               // per beam: bins per lane (0: the plan's)
    size_t dm_off = 0, tab_off = 0, ctr_off = 0;
    char *ws = nullptr;
    int device = 0;
    int dm_tile = 0;                          // 0: each plan's own
    int wg_per_cu = 2;
    long long total = 0;                      // work items over all launches
    struct Launch {
        int m, recur, k, r, first, count;     // M_bin, form, three-pass K (-1: none), bins per lane,
        long long items;                      // table rows [first, first + count)
    };
    std::vector<Launch> launches;             // one persistent launch per (M_bin, form)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t graph_stream = nullptr;
    bool dirty = true;                        // the graph must be captured again
};

namespace {

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// channel chunks per workgroup of the batched DM-stage item
int batch_chunks_per_wg(int m, int r) {
    return r == 8 ? (m == 4096 ? FusedShape<4096, 8>::C : FusedShape<2048, 8>::C) : 4096 / m;
}

int batch_layout(const cdmt_beam_t *beams, int nbeam, std::vector<size_t> *spec_off,
                 size_t *dm_off, size_t *tab_off, size_t *ctr_off, size_t *total) {
    if (!beams || nbeam < 1 || nbeam > 4096)
        return CDMT_E_ARG;
    size_t off = 0;
    size_t ndm_all = 0;
    for (int b = 0; b < nbeam; ++b) {
        const cdmt_beam_t &B = beams[b];
        const cdmt_plan_s *p = B.plan;
        if (!p || B.nblock < 1 || B.ndm < 1 || !B.voltages || !B.dm_list || !B.out)
            return CDMT_E_ARG;
        if (p->precision != 0)
            return CDMT_E_UNSUPPORTED;          // FP32
        if (p->m > 4096)
            return CDMT_E_UNSUPPORTED;          // 512-lane workgroups: use cdmt_dedisperse
        if ((long long)B.nblock * p->nsub * p->nchan > 0x7fffffffLL)
            return CDMT_E_SHAPE;
        const int dst = check_dms(p, B.dm_list, B.ndm);
        if (dst)
            return dst;
        size_t w = 0;
        workspace_bytes(p, B.nblock, &w);
        if (spec_off)
            spec_off->push_back(off);
        off = align256(off + w);
        ndm_all += (size_t)B.ndm;
    }
    *dm_off = off;
    off = align256(off + ndm_all * sizeof(double));
    *tab_off = off;
    off = align256(off + (size_t)nbeam * sizeof(BatchBeam));
    *ctr_off = off;
    *total = off + kBatchGroups * kBatchQueues * sizeof(unsigned long long);
    return CDMT_OK;
}

// device table of the batch for its current settings (synchronous copy):
// rows grouped by M_bin, one persistent launch per group
int batch_upload(cdmt_batch_s *bt) {
    const int nbeam = (int)bt->beams.size();
    std::vector<BatchBeam> tab;
    std::vector<double> dmall;
    std::vector<size_t> dm_at(nbeam);
    for (int b = 0; b < nbeam; ++b) {
        dm_at[b] = dmall.size();
        dmall.insert(dmall.end(), bt->dms[b].begin(), bt->dms[b].end());
    }
    bt->launches.clear();
    bt->total = 0;
    std::vector<BatchBeam> rows(nbeam);
    std::vector<int> rec(nbeam), kk(nbeam), rr(nbeam);
    for (int b = 0; b < nbeam; ++b) {
        const cdmt_beam_t &B = bt->beams[b];
        const cdmt_plan_s *p = B.plan;
        BatchBeam &T = rows[b];
        std::memset(&T, 0, sizeof(T));
        T.a = fused_args(p, bt->ws + bt->spec_off[b], B.nblock, B.out);
        T.a.dm_tile = bt->dm_tile > 0 ? bt->dm_tile : p->dm_tile;
        const int lb = bt->lane_bins[b] ? bt->lane_bins[b] : p->lane_bins;
        rr[b] = lb == 8 && (p->m == 2048 || p->m == 4096) ? 8 : 16;
        const int C = batch_chunks_per_wg(p->m, rr[b]);
        T.a.inner = p->nchan >= C ? p->nchan / C : 1;
        T.a.ndm = B.ndm;
        T.a.ndt = (B.ndm + T.a.dm_tile - 1) / T.a.dm_tile;
        const std::vector<double> &d = bt->dms[b];
        const bool recur = T.a.dm_step != 0.0 && T.a.dm_tile > 1 && B.ndm > 1 &&
                           arithmetic(d.data(), B.ndm, T.a.dm_step);
        T.a.dm_step = recur ? d[1] - d[0] : 0.0;
        rec[b] = recur ? 1 : 0;
        if (bt->fft_sched[b] >= 0)
            T.a.schedule = bt->fft_sched[b];
        kk[b] = p->m >= 1024 && rr[b] == 16 ? x3_k(T.a) : -1;
        T.dms = reinterpret_cast<const double *>(bt->ws + bt->dm_off) + dm_at[b];
    }
    for (int m = 64; m <= 4096; m *= 2) {
      for (int r = 1; r >= 0; --r) {
        for (int R = 16; R >= 8; R -= 8) {
          for (int k = -1; k <= (m >= 1024 && R == 16 ? 3 : -1); ++k) {
            cdmt_batch_s::Launch L{m, r, k, R, (int)tab.size(), 0, 0};
            for (int b = 0; b < nbeam; ++b) {
                if (bt->beams[b].plan->m != m || rec[b] != r || kk[b] != k || rr[b] != R)
                    continue;
                BatchBeam T = rows[b];
                const int C = batch_chunks_per_wg(m, R);
                T.item0 = L.items;
                L.items += ((long long)T.a.nchunks + C - 1) / C * T.a.ndt;
                tab.push_back(T);
                ++L.count;
            }
            if (L.count) {
                if ((int)bt->launches.size() == kBatchGroups)
                    return CDMT_E_UNSUPPORTED;   // no counters left (not reached: see kBatchGroups)
                bt->launches.push_back(L);
                bt->total += L.items;
            }
          }
        }
      }
    }
    if (hipMemcpy(bt->ws + bt->dm_off, dmall.data(), dmall.size() * sizeof(double),
                  hipMemcpyHostToDevice) != hipSuccess)
        return CDMT_E_DEVICE;
    if (hipMemcpy(bt->ws + bt->tab_off, tab.data(), tab.size() * sizeof(BatchBeam),
                  hipMemcpyHostToDevice) != hipSuccess)
        return CDMT_E_DEVICE;
    bt->dirty = true;
    return CDMT_OK;
}

template <int M>
void batch_launch(int recur, const BatchBeam *tab, int count, long long items,
                  unsigned long long *ctr, int grid, hipStream_t st) {
    if (recur)
        dm_batch<M, true><<<grid, 256, 0, st>>>(tab, count, items, ctr);
    else
        dm_batch<M, false><<<grid, 256, 0, st>>>(tab, count, items, ctr);
}

template <int M>
void batch_launch8(int recur, const BatchBeam *tab, int count, long long items,
                   unsigned long long *ctr, int grid, hipStream_t st) {
    constexpr int WG = FusedShape<M, 8>::WG;
    if (recur)
        dm_batch<M, true, -1, 8><<<grid, WG, 0, st>>>(tab, count, items, ctr);
    else
        dm_batch<M, false, -1, 8><<<grid, WG, 0, st>>>(tab, count, items, ctr);
}

template <int M>
void batch_launch_x3(int recur, int k, const BatchBeam *tab, int count, long long items,
                    unsigned long long *ctr, int grid, hipStream_t st) {
    switch (k + (recur ? 4 : 0)) {
    case 0: dm_batch<M, false, 0><<<grid, 256, 0, st>>>(tab, count, items, ctr); break;
    case 1: dm_batch<M, false, 1><<<grid, 256, 0, st>>>(tab, count, items, ctr); break;
    case 2: dm_batch<M, false, 2><<<grid, 256, 0, st>>>(tab, count, items, ctr); break;
    case 3: dm_batch<M, false, 3><<<grid, 256, 0, st>>>(tab, count, items, ctr); break;
    case 4: dm_batch<M, true, 0><<<grid, 256, 0, st>>>(tab, count, items, ctr); break;
    case 5: dm_batch<M, true, 1><<<grid, 256, 0, st>>>(tab, count, items, ctr); break;
    case 6: dm_batch<M, true, 2><<<grid, 256, 0, st>>>(tab, count, items, ctr); break;
    default: dm_batch<M, true, 3><<<grid, 256, 0, st>>>(tab, count, items, ctr); break;
    }
}

// forward stage of beam b with the batch's split for it
int batch_forward(cdmt_batch_s *bt, int b, hipStream_t st) {
    const cdmt_beam_t &B = bt->beams[b];
    cdmt_plan_s q = *B.plan;
    if (bt->fwd_n2[b]) {
        q.n2 = bt->fwd_n2[b];
        q.n1 = q.nfft / q.n2;
    }
    return launch_forward(&q, bt->ws + bt->spec_off[b], B.voltages, B.nblock, st);
}

int batch_enqueue(cdmt_batch_s *bt, hipStream_t st) {
    for (size_t b = 0; b < bt->beams.size(); ++b) {
        const int r = batch_forward(bt, (int)b, st);
        if (r)
            return r;
    }
    unsigned long long *ctr = reinterpret_cast<unsigned long long *>(bt->ws + bt->ctr_off);
    batch_reset<<<1, 128, 0, st>>>(ctr, kBatchGroups * kBatchQueues);
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, bt->device) !=
        hipSuccess || ncu < 1)
        return CDMT_E_DEVICE;
    const int grid = ncu * bt->wg_per_cu;
    const BatchBeam *tab = reinterpret_cast<const BatchBeam *>(bt->ws + bt->tab_off);
    for (size_t k = 0; k < bt->launches.size(); ++k) {
        const cdmt_batch_s::Launch &L = bt->launches[k];
        unsigned long long *c = ctr + k * kBatchQueues;
        const BatchBeam *t = tab + L.first;
        if (L.k >= 0) {
            if (L.m == 4096)
                batch_launch_x3<4096>(L.recur, L.k, t, L.count, L.items, c, grid, st);
            else if (L.m == 2048)
                batch_launch_x3<2048>(L.recur, L.k, t, L.count, L.items, c, grid, st);
            else
                batch_launch_x3<1024>(L.recur, L.k, t, L.count, L.items, c, grid, st);
            if (hipGetLastError() != hipSuccess)
                return CDMT_E_DEVICE;
            continue;
        }
        if (L.r == 8) {
            if (L.m == 4096)
                batch_launch8<4096>(L.recur, t, L.count, L.items, c, grid, st);
            else
                batch_launch8<2048>(L.recur, t, L.count, L.items, c, grid, st);
            if (hipGetLastError() != hipSuccess)
                return CDMT_E_DEVICE;
            continue;
        }
        switch (L.m) {
        case 64: batch_launch<64>(L.recur, t, L.count, L.items, c, grid, st); break;
        case 128: batch_launch<128>(L.recur, t, L.count, L.items, c, grid, st); break;
        case 256: batch_launch<256>(L.recur, t, L.count, L.items, c, grid, st); break;
        case 512: batch_launch<512>(L.recur, t, L.count, L.items, c, grid, st); break;
        case 1024: batch_launch<1024>(L.recur, t, L.count, L.items, c, grid, st); break;
        case 2048: batch_launch<2048>(L.recur, t, L.count, L.items, c, grid, st); break;
        case 4096: batch_launch<4096>(L.recur, t, L.count, L.items, c, grid, st); break;
        default: return CDMT_E_UNSUPPORTED;
        }
        if (hipGetLastError() != hipSuccess)
            return CDMT_E_DEVICE;
    }
    return CDMT_OK;
}

void batch_drop_graph(cdmt_batch_s *bt) {
    if (bt->exec)
        (void)hipGraphExecDestroy(bt->exec);
    if (bt->graph)
        (void)hipGraphDestroy(bt->graph);
    bt->exec = nullptr;
    bt->graph = nullptr;
    bt->graph_stream = nullptr;
}

}  // namespace

extern "C" {

int cdmt_batch_workspace_size(const cdmt_beam_t *beams, int nbeam, size_t *bytes) {
    if (!bytes)
        return CDMT_E_ARG;
    size_t a, b, c;
    return batch_layout(beams, nbeam, nullptr, &a, &b, &c, bytes);
}

int cdmt_batch_create(cdmt_batch_t *out, const cdmt_beam_t *beams, int nbeam, void *workspace,
                      size_t ws_bytes) {
    if (!out)
        return CDMT_E_ARG;
    *out = nullptr;
    std::vector<size_t> off;
    size_t dm_off, tab_off, ctr_off, need;
    int st = batch_layout(beams, nbeam, &off, &dm_off, &tab_off, &ctr_off, &need);
    if (st)
        return st;
    if (!workspace)
        return CDMT_E_ARG;
    if (ws_bytes < need)
        return CDMT_E_WORKSPACE;
    if ((st = ensure_twiddles()))
        return st;
    cdmt_batch_s *bt = new cdmt_batch_s;
    bt->beams.assign(beams, beams + nbeam);
    for (int b = 0; b < nbeam; ++b) {
        bt->dms.emplace_back(beams[b].dm_list, beams[b].dm_list + beams[b].ndm);
        bt->beams[b].dm_list = nullptr;       // read during this call only
    }
    bt->spec_off = off;
    bt->fwd_n2.assign(nbeam, 0);
    bt->fft_sched.assign(nbeam, -1);
    bt->lane_bins.assign(nbeam, 0);
    bt->dm_off = dm_off;
    bt->tab_off = tab_off;
    bt->ctr_off = ctr_off;
    bt->ws = static_cast<char *>(workspace);
    if (hipGetDevice(&bt->device) != hipSuccess || (st = batch_upload(bt))) {
        delete bt;
        return st ? st : CDMT_E_DEVICE;
    }
    *out = bt;
    return CDMT_OK;
}

int cdmt_batch_set(cdmt_batch_t bt, int opt, int value) {
    if (!bt)
        return CDMT_E_ARG;
    switch (opt) {
    case CDMT_BATCH_DM_TILE:
        if (value < 0 || value > 64)
            return CDMT_E_ARG;
        // the table is rewritten in place: no run of the batch may be in flight
        if (hipDeviceSynchronize() != hipSuccess)
            return CDMT_E_DEVICE;
        bt->dm_tile = value;
        return batch_upload(bt);
    case CDMT_BATCH_WG_PER_CU:
        if (value < 1 || value > 8)
            return CDMT_E_ARG;
        bt->wg_per_cu = value;
        bt->dirty = true;
        return CDMT_OK;
    default: return CDMT_E_ARG;
    }
}

int cdmt_batch_get(cdmt_batch_t bt, int opt, long long *value) {
    if (!bt || !value)
        return CDMT_E_ARG;
    switch (opt) {
    case CDMT_BATCH_DM_TILE: *value = bt->dm_tile; return CDMT_OK;
    case CDMT_BATCH_WG_PER_CU: *value = bt->wg_per_cu; return CDMT_OK;
    case CDMT_BATCH_ITEMS: *value = bt->total; return CDMT_OK;
    case CDMT_BATCH_LAUNCHES: *value = (long long)bt->launches.size(); return CDMT_OK;
    default: return CDMT_E_ARG;
    }
}

int cdmt_batch_beam_set(cdmt_batch_t bt, int beam, int opt, int value) {
    if (!bt || beam < 0 || beam >= (int)bt->beams.size())
        return CDMT_E_ARG;
    if (opt == CDMT_BATCH_BEAM_FWD_N2) {
        if (value != 0 && !fwd_split_ok(bt->beams[beam].plan->nfft, value))
            return CDMT_E_ARG;
        bt->fwd_n2[beam] = value;
        bt->dirty = true;
        return CDMT_OK;
    }
    if (opt == CDMT_BATCH_BEAM_FFT_SCHEDULE || opt == CDMT_BATCH_BEAM_LANE_BINS) {
        const bool sched = opt == CDMT_BATCH_BEAM_FFT_SCHEDULE;
        if (sched ? (value < -1 || value > 1) : (value != 0 && value != 8 && value != 16))
            return CDMT_E_ARG;
        int &slot = sched ? bt->fft_sched[beam] : bt->lane_bins[beam];
        if (slot == value)
            return CDMT_OK;
        // these decide the beam's launch group: rewrite the table
        if (hipDeviceSynchronize() != hipSuccess)
            return CDMT_E_DEVICE;
        const int old = slot;
        slot = value;
        const int r = batch_upload(bt);
        if (r)
            slot = old;
        return r;
    }
    return CDMT_E_ARG;
}
int cdmt_batch_beam_get(cdmt_batch_t bt, int beam, int opt, int *value) {
    if (!bt || !value || beam < 0 || beam >= (int)bt->beams.size())
        return CDMT_E_ARG;
    if (opt == CDMT_BATCH_BEAM_FWD_N2) {
        *value = bt->fwd_n2[beam] ? bt->fwd_n2[beam] : bt->beams[beam].plan->n2;
        return CDMT_OK;
    }
    if (opt == CDMT_BATCH_BEAM_FFT_SCHEDULE) {
        *value = bt->fft_sched[beam] >= 0 ? bt->fft_sched[beam]
                                          : bt->beams[beam].plan->fft_schedule;
        return CDMT_OK;
    }
    if (opt == CDMT_BATCH_BEAM_LANE_BINS) {
        *value = bt->lane_bins[beam] ? bt->lane_bins[beam] : bt->beams[beam].plan->lane_bins;
        return CDMT_OK;
    }
    return CDMT_E_ARG;
}

int cdmt_batch_run(cdmt_batch_t bt, void *hip_stream) {
    if (!bt)
        return CDMT_E_ARG;
    return batch_enqueue(bt, static_cast<hipStream_t>(hip_stream));
}

int cdmt_batch_run_graph(cdmt_batch_t bt, void *hip_stream) {
    if (!bt || !hip_stream)
        return CDMT_E_ARG;                     // capture needs a created stream
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (bt->dirty || !bt->exec || bt->graph_stream != st) {
        batch_drop_graph(bt);
        if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return CDMT_E_DEVICE;
        const int r = batch_enqueue(bt, st);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(st, &g);
        if (r || e != hipSuccess || !g) {
            if (g)
                (void)hipGraphDestroy(g);
            return r ? r : CDMT_E_DEVICE;
        }
        bt->graph = g;
        if (hipGraphInstantiate(&bt->exec, g, nullptr, nullptr, 0) != hipSuccess) {
            batch_drop_graph(bt);
            return CDMT_E_DEVICE;
        }
        bt->graph_stream = st;
        bt->dirty = false;
    }
    return hipGraphLaunch(bt->exec, st) == hipSuccess ? CDMT_OK : CDMT_E_DEVICE;
}

int cdmt_batch_autotune(cdmt_batch_t bt, void *hip_stream, int reps, float *best_ms) {
    if (!bt || reps < 1)
        return CDMT_E_ARG;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess)
        return CDMT_E_DEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return CDMT_E_DEVICE;
    }
    // time reps runs of enqueue() after one warm-up
    const auto timed = [&](auto enqueue, float *ms) {
        int rc = enqueue();
        if (rc)
            return rc;
        if (hipEventRecord(e0, st) != hipSuccess)
            return (int)CDMT_E_DEVICE;
        for (int i = 0; i < reps && !rc; ++i)
            rc = enqueue();
        if (rc)
            return rc;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(ms, e0, e1) != hipSuccess)
            return (int)CDMT_E_DEVICE;
        *ms /= reps;
        return (int)CDMT_OK;
    };
    int r = CDMT_OK;
    // the forward FFT's radix schedule, beam by beam (each beam's forward
    // stage is its own launches, so the choices are independent)
    for (int b = 0; b < (int)bt->beams.size() && !r; ++b) {
        float fbest = 0.f;
        int fn2 = 0;
        for (int n2 = 64; n2 <= 256 && !r; n2 *= 2) {
            if (!fwd_split_ok(bt->beams[b].plan->nfft, n2))
                continue;
            bt->fwd_n2[b] = n2;
            float ms = 0.f;
            r = timed([&] { return batch_forward(bt, b, st); }, &ms);
            if (!r && (fbest == 0.f || ms < fbest)) {
                fbest = ms;
                fn2 = n2;
            }
        }
        bt->fwd_n2[b] = fn2;
    }
    bt->dirty = true;
    // the DM stage's radix schedule, per M_bin (the beams of one M_bin share
    // its launches), each candidate timed on the whole batch with the other
    // M_bin unchanged: at M_bin 4096 and 2048 the three-pass transform
    // (schedule 0, where the beam allows it), radix-16 and radix-8 Stockham
    // stages (schedule 1 with 16 or 8 bins per lane); at 1024 the three-pass
    // transform and radix-16 stages; other M_bin have the radix-16 stages only
    for (int m = 1024; m <= 4096 && !r; m *= 2) {
        std::vector<int> beams_m;
        for (int b = 0; b < (int)bt->beams.size(); ++b)
            if (bt->beams[b].plan->m == m)
                beams_m.push_back(b);
        if (beams_m.empty())
            continue;
        struct Cand { int sched, bins; };
        const Cand cands[] = {{0, 16}, {1, 16}, {1, 8}};
        float best_c = 0.f;
        int pick = 0;
        for (int ci = 0; ci < (m == 1024 ? 2 : 3) && !r; ++ci) {
            for (int b : beams_m) {
                bt->fft_sched[b] = cands[ci].sched;
                bt->lane_bins[b] = cands[ci].bins;
            }
            if ((r = batch_upload(bt)))
                break;
            float ms = 0.f;
            r = timed([&] { return batch_enqueue(bt, st); }, &ms);
            if (!r && (best_c == 0.f || ms < best_c)) {
                best_c = ms;
                pick = ci;
            }
        }
        if (!r) {
            for (int b : beams_m) {
                bt->fft_sched[b] = cands[pick].sched;
                bt->lane_bins[b] = cands[pick].bins;
            }
            r = batch_upload(bt);
        }
    }
    static const int kTiles[] = {8, 16, 32, 64};
    static const int kWg[] = {2, 4};
    float best = 0.f;
    int bt_tile = 16, bt_wg = 2;
    for (int tile : kTiles) {
        for (int wg : kWg) {
            if ((r = cdmt_batch_set(bt, CDMT_BATCH_DM_TILE, tile)) ||
                (r = cdmt_batch_set(bt, CDMT_BATCH_WG_PER_CU, wg)))
                break;
            float ms = 0.f;
            if ((r = timed([&] { return batch_enqueue(bt, st); }, &ms)))
                break;
            if (best == 0.f || ms < best) {
                best = ms;
                bt_tile = tile;
                bt_wg = wg;
            }
        }
        if (r)
            break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (r)
        return r;
    if ((r = cdmt_batch_set(bt, CDMT_BATCH_DM_TILE, bt_tile)) ||
        (r = cdmt_batch_set(bt, CDMT_BATCH_WG_PER_CU, bt_wg)))
        return r;
    if (best_ms)
        *best_ms = best;
    return CDMT_OK;
}

void cdmt_batch_destroy(cdmt_batch_t bt) {
    if (!bt)
        return;
    batch_drop_graph(bt);
    delete bt;
}

}  // extern "C"
