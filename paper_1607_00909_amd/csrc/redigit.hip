// Redigitisation of a filterbank to 8-bit codes (Bassa, Pleunis & Hessels
// 2016, Sec. 3, the paragraph after the transpose; Alg. 1 "redigitize"):
// per DM trial and channel, the mean and standard deviation of the channel's
// time series give an offset and a scale, which map each sample to a byte.
// As in the paper, three kernels: partial sums over time segments, their
// combination per channel, and the conversion.
//
//   redig_partial   one workgroup per (64 channels, segment of 1024 samples,
//                   DM); lane = channel, so every load of a wave is 256
//                   contiguous bytes of one time row.  Four waves take four
//                   sub-ranges of the segment; each lane accumulates FP64
//                   sums of (x - K) and (x - K)^2 about its first sample K,
//                   converts them to (mean, M2) and the four are merged in
//                   LDS (pairwise update of Chan, Golub & LeVeque).
//   redig_params    one lane per (DM, channel): merges the segments in order,
//                   sigma = sqrt(M2 / T), and writes the FP32 parameters
//                   mean and scale = counts_per_sigma / sigma (0 if sigma = 0).
//   redig_quantise  code = clamp(rint((x - mean) * scale + zero), 0, 255) in
//                   FP32 with each operation rounded separately; a workgroup
//                   per time row, four channels per lane (16-byte loads,
//                   4-byte store).
// Two passes over the FP32 filterbank are inherent (the parameters depend on
// the whole series); both are HBM-bound streams.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/cdmt.h"

namespace {

constexpr int kRdChan = 64;                    // channels per workgroup
constexpr int kRdWaves = 4;                    // sub-ranges per segment
constexpr int kRdSub = 256;                    // samples per sub-range
constexpr int kRdSeg = kRdWaves * kRdSub;      // samples per segment

// merge (nb, mb, qb) into (na, ma, qa): counts, means, sums of squared deviations
__device__ __forceinline__ void merge_moments(double &na, double &ma, double &qa, double nb,
                                              double mb, double qb) {
    if (nb == 0.0)
        return;
    if (na == 0.0) {
        na = nb;
        ma = mb;
        qa = qb;
        return;
    }
    const double n = na + nb;
    const double d = mb - ma;
    ma += d * (nb / n);
    qa += qb + d * d * (na * nb / n);
    na = n;
}

__global__ __launch_bounds__(256) void redig_partial(const float *__restrict__ in, long long ntime,
                                                     int nchan, int nseg,
                                                     double2 *__restrict__ part) {
    __shared__ double sn[kRdWaves][kRdChan], sm[kRdWaves][kRdChan], sq[kRdWaves][kRdChan];
    const int c = threadIdx.x % kRdChan;
    const int r = threadIdx.x / kRdChan;
    const int ch = blockIdx.x * kRdChan + c;
    const int seg = blockIdx.y;
    const long long d = blockIdx.z;
    const long long t0 = (long long)seg * kRdSeg + (long long)r * kRdSub;
    const long long t1 = t0 + kRdSub < ntime ? t0 + kRdSub : ntime;
    double n = 0.0, mean = 0.0, m2 = 0.0;
    if (ch < nchan && t0 < t1) {
        const float *p = in + (d * ntime + t0) * nchan + ch;
        const double k = p[0];
        double s1 = 0.0, s2 = 0.0;
        const int cnt = (int)(t1 - t0);
        int t = 0;
        for (; t + 8 <= cnt; t += 8) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                v[u] = p[(long long)(t + u) * nchan];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const double e = (double)v[u] - k;
                s1 += e;
                s2 = fma(e, e, s2);
            }
        }
        for (; t < cnt; ++t) {
            const double e = (double)p[(long long)t * nchan] - k;
            s1 += e;
            s2 = fma(e, e, s2);
        }
        n = cnt;
        mean = k + s1 / n;
        m2 = fmax(0.0, s2 - s1 * (s1 / n));
    }
    sn[r][c] = n;
    sm[r][c] = mean;
    sq[r][c] = m2;
    __syncthreads();
    if (r == 0 && ch < nchan) {
        for (int w = 1; w < kRdWaves; ++w)
            merge_moments(n, mean, m2, sn[w][c], sm[w][c], sq[w][c]);
        part[(d * nseg + seg) * nchan + ch] = make_double2(mean, m2);
    }
}

__global__ __launch_bounds__(256) void redig_params(const double2 *__restrict__ part, long long ntime,
                                                    int nchan, int nseg, int ndm, float cps,
                                                    float *__restrict__ mean_out,
                                                    float *__restrict__ scale_out) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)ndm * nchan)
        return;
    const long long d = i / nchan;
    const int ch = (int)(i % nchan);
    double n = 0.0, mean = 0.0, m2 = 0.0;
    for (int s = 0; s < nseg; ++s) {
        const double2 v = part[(d * nseg + s) * nchan + ch];
        const long long len = ntime - (long long)s * kRdSeg;
        merge_moments(n, mean, m2, (double)(len < kRdSeg ? len : kRdSeg), v.x, v.y);
    }
    const double sigma = sqrt(m2 / (double)ntime);
    mean_out[i] = (float)mean;
    scale_out[i] = sigma > 0.0 ? (float)((double)cps / sigma) : 0.0f;
}

__device__ __forceinline__ uint32_t code_of(float x, float m, float k, float zero) {
#pragma clang fp contract(off)
    // three separately rounded operations (no fused multiply-add)
    float t = x - m;
    t = t * k;
    t = t + zero;
    t = rintf(t);
    t = fminf(fmaxf(t, 0.0f), 255.0f);
    return (uint32_t)t;
}

// one workgroup per time row (d, t) at a time, lanes across the row: the
// parameters of DM d are contiguous and shared by every row of that DM.
// Vector form: four channels per lane (16-byte loads, one 4-byte store).
__global__ __launch_bounds__(256) void redig_quantise4(const float4 *__restrict__ in,
                                                       long long ntime, int q4, long long nrows,
                                                       const float4 *__restrict__ mean,
                                                       const float4 *__restrict__ scale,
                                                       float zero, uint32_t *__restrict__ out) {
    for (long long row = blockIdx.x; row < nrows; row += gridDim.x) {
        const long long d = row / ntime;
        const float4 *src = in + row * q4;
        uint32_t *dst = out + row * q4;
        const float4 *mr = mean + d * q4;
        const float4 *kr = scale + d * q4;
        for (int j = threadIdx.x; j < q4; j += blockDim.x) {
            const float4 x = src[j], m = mr[j], k = kr[j];
            dst[j] = code_of(x.x, m.x, k.x, zero) | (code_of(x.y, m.y, k.y, zero) << 8) |
                     (code_of(x.z, m.z, k.z, zero) << 16) | (code_of(x.w, m.w, k.w, zero) << 24);
        }
    }
}

__global__ __launch_bounds__(256) void redig_quantise1(const float *__restrict__ in, long long ntime,
                                                       int nchan, long long nrows,
                                                       const float *__restrict__ mean,
                                                       const float *__restrict__ scale, float zero,
                                                       uint8_t *__restrict__ out) {
    for (long long row = blockIdx.x; row < nrows; row += gridDim.x) {
        const long long d = row / ntime;
        for (int c = threadIdx.x; c < nchan; c += blockDim.x)
            out[row * nchan + c] =
                (uint8_t)code_of(in[row * nchan + c], mean[d * nchan + c], scale[d * nchan + c], zero);
    }
}

int rd_nseg(long long ntime) { return (int)((ntime + kRdSeg - 1) / kRdSeg); }

}  // namespace

extern "C" int cdmt_redigitise_workspace_size(int ndm, long long ntime, int nchan, size_t *bytes) {
    if (!bytes || ndm < 0 || ntime < 1 || nchan < 1)
        return CDMT_E_ARG;
    *bytes = (size_t)ndm * (size_t)rd_nseg(ntime) * (size_t)nchan * sizeof(double2);
    return CDMT_OK;
}

extern "C" int cdmt_redigitise(const float *filterbank, int ndm, long long ntime, int nchan,
                               float zero, float counts_per_sigma, void *workspace,
                               size_t ws_bytes, unsigned char *codes, float *mean, float *scale,
                               void *hip_stream) {
    if (ndm < 0 || ntime < 1 || nchan < 1 || !std::isfinite(zero) ||
        !std::isfinite(counts_per_sigma) || !(counts_per_sigma > 0.0f))
        return CDMT_E_ARG;
    if (ndm == 0)
        return CDMT_OK;
    if (!filterbank || !workspace || !codes || !mean || !scale)
        return CDMT_E_ARG;
    const int nseg = rd_nseg(ntime);
    if (ndm > 65535 || nseg > 65535)
        return CDMT_E_SHAPE;
    size_t need = 0;
    cdmt_redigitise_workspace_size(ndm, ntime, nchan, &need);
    if (ws_bytes < need)
        return CDMT_E_WORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    double2 *part = static_cast<double2 *>(workspace);

    const dim3 g1((nchan + kRdChan - 1) / kRdChan, nseg, ndm);
    redig_partial<<<g1, 256, 0, st>>>(filterbank, ntime, nchan, nseg, part);
    if (hipGetLastError() != hipSuccess)
        return CDMT_E_DEVICE;
    const long long npar = (long long)ndm * nchan;
    redig_params<<<(unsigned)((npar + 255) / 256), 256, 0, st>>>(part, ntime, nchan, nseg, ndm,
                                                                counts_per_sigma, mean, scale);
    if (hipGetLastError() != hipSuccess)
        return CDMT_E_DEVICE;
    const long long nrows = (long long)ndm * ntime;
    const auto a16 = [](const void *q) { return (reinterpret_cast<uintptr_t>(q) & 15) == 0; };
    const bool vec = (nchan % 4 == 0) && a16(filterbank) && a16(mean) && a16(scale) &&
                     ((reinterpret_cast<uintptr_t>(codes) & 3) == 0);
    const unsigned blocks = (unsigned)(nrows < (1LL << 20) ? nrows : (1LL << 20));
    if (vec)
        redig_quantise4<<<blocks, 256, 0, st>>>(
            reinterpret_cast<const float4 *>(filterbank), ntime, nchan / 4, nrows,
            reinterpret_cast<const float4 *>(mean), reinterpret_cast<const float4 *>(scale), zero,
            reinterpret_cast<uint32_t *>(codes));
    else
        redig_quantise1<<<blocks, 256, 0, st>>>(filterbank, ntime, nchan, nrows, mean, scale, zero,
                                                codes);
    if (hipGetLastError() != hipSuccess)
        return CDMT_E_DEVICE;
    return CDMT_OK;
}
