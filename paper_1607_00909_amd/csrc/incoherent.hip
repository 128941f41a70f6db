// Incoherent stage of a semi-coherent search (Sec. 1; Sec. 4): the channel
// sums of coherently dedispersed filterbanks at fine DM steps around each
// coherent trial.  Built into libcdmt.so with cdmt.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>

#include "../../include/cdmt.h"
#include "plan.hpp"
#include "xcd.hpp"

using cdmt::kKdm;
using cdmt::xcd_remap;

// ---------------------------------------------------------------------------
// Incoherent stage of a semi-coherent search: each coherently dedispersed
// filterbank (one per coherent DM trial) is dedispersed incoherently at fine
// DM steps around its trial, i.e. every channel's series is shifted by its
// dispersion delay behind the highest channel (Eq. 2, in whole output
// samples) and the channels are summed.
//   inc_delays     delay table in FP64, rounded half to even, in groups of
//                  kIncK trials (padding repeats the last trial): per group
//                  and channel the first delay, then the others relative to
//                  it, as int32 laid out [d][ch][k] or, when every spread is
//                  below kIncSpan, as bytes packed in 8 int32 laid out
//                  [d][group][ch] (a channel pair is one 64-byte load)
//   inc_transpose  [d][t][ch] -> [d][ch][t] through LDS, so that the sums
//                  read each channel's series contiguously (32-channel x
//                  256-sample tiles moved as float4 where the sizes allow,
//                  else 32 x 32)
//   inc_sum        one wave per (coherent DM, kIncK fine trials, kIncT output
//                  samples), each lane owning kIncS samples 64 apart (so LDS
//                  reads of consecutive lanes hit consecutive banks).  Per
//                  channel the wave stages the window its trials read (the
//                  tile plus the spread of their delays) in LDS once; the
//                  delays grow with the trial index, so a lane re-reads its
//                  kIncS values only when the delay changes and otherwise
//                  adds the ones it holds.  Windows wider than the LDS buffer
//                  (very coarse steps) read global memory per trial instead.

namespace {

// DM list passed by value in the kernel arguments
constexpr int kIncDms = 256;

struct IncDms {
    double dm[kIncDms];
};

struct IncArgs {
    int nsub, nchan, nch, ntrial, kpad, chirp_ref;
    long long ntime, nout;
    double f_centre, bw, tsamp, ddm0, ddm;
};

constexpr int kIncS = 4;                      // samples per lane, 64 apart
constexpr int kIncT = 64 * kIncS;             // output samples per workgroup
constexpr int kIncK = 12;                     // fine trials per workgroup (<= 16)
constexpr int kIncSpan = 256;                 // widest delay spread staged in LDS
constexpr int kIncW = 4;                      // trial groups (waves) sharing a staged window
constexpr int kIncG = kIncW * kIncK;          // fine trials per shared-window workgroup

// (both functions evaluate exactly as written, with no fused multiply-adds,
// so that every rounding of a delay to whole samples is reproducible)
__host__ __device__ inline double inc_frequency(const IncArgs &a, int ch) {
#pragma clang fp contract(off)
    const int s = a.nsub - 1 - ch / a.nchan;
    const int c = a.nchan - 1 - ch % a.nchan;
    const double fs = a.f_centre + ((double)s - (a.nsub - 1) / 2.0) * a.bw;
    return a.chirp_ref == 1 ? fs : fs - a.bw / 2.0 + (c + 0.5) * a.bw / a.nchan;
}

__host__ __device__ inline long long inc_delay(const IncArgs &a, double dm, int ch) {
#pragma clang fp contract(off)
    const double nu = inc_frequency(a, ch);
    const double top = inc_frequency(a, 0);
    const double u = 1.0 / (nu * nu) - 1.0 / (top * top);
    return (long long)rint(kKdm * dm * u / a.tsamp);
}

__global__ __launch_bounds__(256) void inc_delays(IncArgs a, IncDms dl, int first, int cnt,
                                                  int packed, int *__restrict__ D) {
#pragma clang fp contract(off)
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int ngroup = a.kpad / kIncK;
    const long long per = (long long)a.nch * ngroup;
    if (i >= per * cnt)
        return;
    const int dl_i = (int)(i / per);
    const int ch = (int)((i % per) / ngroup);
    const int k0 = (int)(i % ngroup) * kIncK;       // first trial of the group (< ntrial)
    const auto delay = [&](int k) {
        return (int)inc_delay(a, dl.dm[dl_i] + (a.ddm0 + a.ddm * (double)min(k, a.ntrial - 1)), ch);
    };
    const int lo = delay(k0);
    if (packed) {
        const long long npair = (a.nch + 1) / 2;
        int *slot = D + (((long long)(first + dl_i) * ngroup + k0 / kIncK) * npair) * 16 + ch * 8;
        unsigned b[4] = {0u, 0u, 0u, 0u};
        for (int k = 1; k < kIncK; ++k)
            b[k / 4] |= (unsigned)min(delay(k0 + k) - lo, kIncSpan - 1) << (8 * (k % 4));
        slot[0] = lo;
        for (int q = 0; q < 4; ++q)
            slot[1 + q] = (int)b[q];
        if (ch == a.nch - 1 && a.nch % 2)            // the all-zero channel completing the pair
            for (int q = 8; q < 16; ++q)
                slot[q] = 0;
    } else {
        int *slot = D + ((long long)(first + dl_i) * a.nch + ch) * a.kpad + k0;
        slot[0] = lo;
        for (int k = 1; k < kIncK; ++k)
            slot[k] = delay(k0 + k) - lo;
    }
}

// Delays for inc_sum_shared: per (DM, supergroup of kIncG trials, channel)
// 16 words, the supergroup's first delay in word 0, then the offset of each
// of its trials relative to it in bytes (trial k in byte k % 4 of word
// 1 + k / 4), then in word 13 the largest offset (the window's extent),
// laid out [d][supergroup][channel pair][32]; a missing second channel of an
// odd count is all zero.
__global__ __launch_bounds__(256) void inc_delays_shared(IncArgs a, IncDms dl, int first, int cnt,
                                                         int *__restrict__ D) {
#pragma clang fp contract(off)
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int nsg = a.kpad / kIncG;
    const long long per = (long long)a.nch * nsg;
    if (i >= per * cnt)
        return;
    const int dl_i = (int)(i / per);
    const int ch = (int)((i % per) / nsg);
    const int k0 = (int)(i % nsg) * kIncG;
    const auto delay = [&](int k) {
        return (int)inc_delay(a, dl.dm[dl_i] + (a.ddm0 + a.ddm * (double)min(k, a.ntrial - 1)), ch);
    };
    const int lo = delay(k0);
    const long long npair = (a.nch + 1) / 2;
    int *slot = D + (((long long)(first + dl_i) * nsg + k0 / kIncG) * npair) * 32 + ch * 16;
    unsigned b[kIncG / 4];
    for (int q = 0; q < kIncG / 4; ++q)
        b[q] = 0u;
    for (int k = 1; k < kIncG; ++k)
        b[k / 4] |= (unsigned)min(delay(k0 + k) - lo, kIncSpan - 1) << (8 * (k % 4));
    slot[0] = lo;
    for (int q = 0; q < kIncG / 4; ++q)
        slot[1 + q] = (int)b[q];
    for (int q = 1 + kIncG / 4; q < 16; ++q)
        slot[q] = 0;
    slot[1 + kIncG / 4] = min(delay(k0 + kIncG - 1) - lo, kIncSpan - 1);
    if (ch == a.nch - 1 && a.nch % 2)
        for (int q = 16; q < 32; ++q)
            slot[q] = 0;
}

// TC channels x TT samples per tile, moved as float4 (nch and ntime
// multiples of 4): reads of TC channels per time row, writes of TT samples
// per channel row
template <int TC, int TT>
__global__ __launch_bounds__(256) void inc_transpose4(const float *__restrict__ fb,
                                                      float *__restrict__ ft, long long ntime,
                                                      int nch) {
    __shared__ float tile[TT][TC + 1];
    const long long t0 = (long long)blockIdx.x * TT;
    const int c0 = blockIdx.y * TC;
    const long long d = blockIdx.z;
    constexpr int RQ = TC / 4, RP = 256 / RQ;       // read: float4 per row, rows per pass
    constexpr int WQ = TT / 4, WP = 256 / WQ;       // write: float4 per row, rows per pass
    {
        const int q = (threadIdx.x % RQ) * 4, r0 = threadIdx.x / RQ;
#pragma unroll
        for (int r = r0; r < TT; r += RP) {
            const long long t = t0 + r;
            if (t < ntime && c0 + q < nch) {
                const float4 v =
                    *reinterpret_cast<const float4 *>(fb + (d * ntime + t) * nch + c0 + q);
                tile[r][q] = v.x;
                tile[r][q + 1] = v.y;
                tile[r][q + 2] = v.z;
                tile[r][q + 3] = v.w;
            }
        }
    }
    __syncthreads();
    {
        const int q = (threadIdx.x % WQ) * 4, r0 = threadIdx.x / WQ;
#pragma unroll
        for (int r = r0; r < TC; r += WP) {
            const long long t = t0 + q;
            if (c0 + r < nch && t < ntime) {
                const float4 v = {tile[q][r], tile[q + 1][r], tile[q + 2][r], tile[q + 3][r]};
                *reinterpret_cast<float4 *>(ft + (d * nch + c0 + r) * ntime + t) = v;
            }
        }
    }
}

__global__ __launch_bounds__(256) void inc_transpose(const float *__restrict__ fb,
                                                     float *__restrict__ ft, long long ntime,
                                                     int nch) {
    __shared__ float tile[32][33];
    const long long t0 = (long long)blockIdx.x * 32;
    const int c0 = blockIdx.y * 32;
    const long long d = blockIdx.z;
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;     // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const long long t = t0 + r;
        const int ch = c0 + tx;
        tile[r][tx] = (t < ntime && ch < nch) ? fb[(d * ntime + t) * nch + ch] : 0.f;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int ch = c0 + r;
        const long long t = t0 + tx;
        if (ch < nch && t < ntime)
            ft[(d * nch + ch) * ntime + t] = tile[tx][r];
    }
}

// Adds v to a without letting the compiler move the addition: each trial's
// sums then follow the window load they use, and the window registers are not
// duplicated to serve additions deferred past the next reload.
__device__ __forceinline__ void inc_add(float &a, float v) {
    asm volatile("v_add_f32 %0, %1, %0" : "+v"(a) : "v"(v));
}

// Raw buffer view of the n floats at p: loads at byte offsets >= 4n read 0
// (the hardware range check), which replaces clamping of window indexes.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t inc_view(const float *p, int n) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(p), (short)0, 4 * n, 0x00020000);
}

__device__ __forceinline__ float inc_load(__amdgpu_buffer_rsrc_t v, int byte_off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(v, byte_off, 0, 0));
}

// WIDE = false: every trial group's delay spread in every channel is below
// kIncSpan (the host proves it from the lowest channel's delay per DM), so
// the window fits the LDS buffer; WIDE = true reads global memory per trial.
template <bool WIDE>
__global__ __launch_bounds__(64) void inc_sum(const float *__restrict__ ft,
                                              const int *__restrict__ D, IncArgs a, int ntile,
                                              int ngroup, float *__restrict__ out) {
    constexpr int kPf = kIncT / 64 + 1;             // window loads per lane for spreads < 64
    __shared__ float win[WIDE ? 1 : 2][WIDE ? 1 : kIncT + kIncSpan];
    // XCD-aware order: the trial groups of one time tile run on one XCD
    // together and share its L2 copy of the tile's windows
    const int lw = xcd_remap(blockIdx.x, gridDim.x);
    const int kgi = lw % ngroup;
    const int tile = (lw / ngroup) % ntile;
    const long long d = lw / (ngroup * ntile);
    const int kg = kgi * kIncK;
    const long long t0 = (long long)tile * kIncT;
    const int lane = threadIdx.x;
    float acc[kIncK][kIncS];
#pragma unroll
    for (int k = 0; k < kIncK; ++k)
#pragma unroll
        for (int j = 0; j < kIncS; ++j)
            acc[k][j] = 0.f;
    // this group's delays: [d][ch][k] (wide) or [d][group][channel pair][16]
    const int *dk = WIDE ? D + d * a.nch * a.kpad + kg
                         : D + ((d * ngroup + kgi) * ((a.nch + 1) / 2)) * 16;
    const float *row = ft + d * a.nch * a.ntime + t0;      // channel ch's series at t0
    const int room = (int)(a.ntime - 1 - t0);           // last readable offset from row
    if constexpr (WIDE) {
        for (int ch = 0; ch < a.nch; ++ch, dk += a.kpad, row += a.ntime) {
            const int lo = dk[0];
            const int last = room - lo;
#pragma unroll
            for (int k = 0; k < kIncK; ++k) {
                const int o = k == 0 ? 0 : dk[k];
#pragma unroll
                for (int j = 0; j < kIncS; ++j)
                    acc[k][j] += row[lo + min(lane + 64 * j + o, last)];
            }
        }
    } else {
        // Channels go in pairs whose trial sums interleave, so that the two
        // windows' LDS reads overlap.  A pair's delays (per channel: the first
        // delay and kIncK - 1 byte offsets packed in words, padded to 8 words) are
        // one 64-byte scalar load, issued two pairs ahead; its windows are
        // loaded one pair ahead, while the current pair's trials are summed.
        // The delays rotate through three arrays, so that none are copied.
        // view(r, lo) covers the kIncT + kIncSpan samples of series r from
        // delay lo on (fewer at the end of the series).
        const auto view = [&](const float *r, int lo) {
            return inc_view(r + lo, min(room - lo + 1, kIncT + kIncSpan));
        };
        const auto offset = [](const int (&dl)[16], int c, int k) {
            return k == 0 ? 0 : (int)(((unsigned)dl[8 * c + 1 + k / 4] >> (8 * (k % 4))) & 0xffu);
        };
        // stage channel c of a pair in LDS buffer c: the kPf loads in pf plus,
        // for spreads of 64 or more, the rest loaded now
        const auto stage = [&](int c, const int (&dl)[16], const float (&pf)[kPf]) {
#pragma unroll
            for (int m = 0; m < kPf; ++m)
                win[c][lane + 64 * m] = pf[m];
            const int span = offset(dl, c, kIncK - 1);
            if (span >= 64 * kPf - kIncT) {
                const auto v = view(row + c * a.ntime, dl[8 * c]);
#pragma unroll 1
                for (int m = kPf; 64 * m < kIncT + span; ++m)
                    win[c][lane + 64 * m] = inc_load(v, 4 * (lane + 64 * m));
            }
        };
        // window loads of channel c of the pair at r (a missing second
        // channel of an odd count is all zero: adding +0 changes no sum)
        const auto fetch = [&](bool real, const float *r, int lo, float (&pf)[kPf]) {
            if (real) {
                const auto v = view(r, lo);
                // the lane's byte offset, opaque to the compiler here so that
                // each load adds its constant in the instruction's offset
                // field instead of holding kPf offsets in registers
                int off = 4 * lane;
                asm volatile("" : "+v"(off));
#pragma unroll
                for (int m = 0; m < kPf; ++m)
                    pf[m] = inc_load(v, off + 256 * m);
            } else {
#pragma unroll
                for (int m = 0; m < kPf; ++m)
                    pf[m] = 0.f;
            }
        };
        const auto delays = [&](int p, int (&dl)[16]) {
#pragma unroll
            for (int q = 0; q < 16; ++q)
                dl[q] = dk[16 * p + q];
        };
        // trial sums of the two staged channels, channel by channel per trial
        const auto sums = [&](const int (&dl)[16]) {
            int held[2];
            float w[2][kIncS];
#pragma unroll
            for (int k = 0; k < kIncK; ++k) {
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const int o = offset(dl, c, k);
                    if (k == 0 || o != held[c]) {
                        held[c] = o;
#pragma unroll
                        for (int j = 0; j < kIncS; ++j)
                            w[c][j] = win[c][lane + 64 * j + o];
                    }
                }
#pragma unroll
                for (int c = 0; c < 2; ++c)
#pragma unroll
                    for (int j = 0; j < kIncS; ++j)
                        inc_add(acc[k][j], w[c][j]);
            }
        };
        const int npair = (a.nch + 1) / 2;
        int dla[16], dlb[16], dlc[16];
        float pf[2][kPf];
        delays(0, dla);
        if (npair > 1)
            delays(1, dlb);
        fetch(true, row, dla[0], pf[0]);
        fetch(a.nch > 1, row + a.ntime, dla[8], pf[1]);
        // pair p: delays in cur, the next pair's in nxt, pair p + 2's loaded
        // into far
        const auto pair = [&](int p, const int (&cur)[16], const int (&nxt)[16], int (&far)[16]) {
            __syncthreads();
            stage(0, cur, pf[0]);
            stage(1, cur, pf[1]);
            row += 2 * a.ntime;
            if (p + 1 < npair) {
                fetch(true, row, nxt[0], pf[0]);
                fetch(2 * p + 3 < a.nch, row + a.ntime, nxt[8], pf[1]);
            }
            if (p + 2 < npair)
                delays(p + 2, far);
            __syncthreads();
            sums(cur);
        };
        int p = 0;
        for (; p + 2 < npair; p += 3) {
            pair(p, dla, dlb, dlc);
            pair(p + 1, dlb, dlc, dla);
            pair(p + 2, dlc, dla, dlb);
        }
        if (p < npair)
            pair(p, dla, dlb, dlc);
        if (p + 1 < npair)
            pair(p + 1, dlb, dlc, dla);
    }
    const int nk = min(kIncK, a.ntrial - kg);
#pragma unroll
    for (int k = 0; k < kIncK; ++k) {
        if (k < nk) {
            float *o = out + (d * a.ntrial + kg + k) * a.nout + t0 + lane;
#pragma unroll
            for (int j = 0; j < kIncS; ++j)
                if (t0 + lane + 64 * j < a.nout)
                    o[64 * j] = acc[k][j];
        }
    }
}

// inc_sum with one staged window shared by kIncW trial groups: a workgroup
// of kIncW waves per (coherent DM, kIncG fine trials, kIncT output samples),
// wave w summing trials 12 w .. 12 w + 11 of the supergroup exactly as
// inc_sum<false> does (same additions in the same channel order, so the same
// sums bit for bit).  Per channel pair the 256 lanes stage both channels'
// windows (kIncT samples plus the supergroup's delay spread, below kIncSpan)
// in LDS, two loads per lane and channel, loaded one pair ahead into
// registers and stored into one of two buffers (one barrier per pair); the
// pair's delays are wave-uniform scalar loads two pairs ahead.  Each window
// is read from memory once per kIncG trials instead of once per kIncK.
__global__ __launch_bounds__(64 * kIncW) void inc_sum_shared(const float *__restrict__ ft,
                                                             const int *__restrict__ D, IncArgs a,
                                                             int ntile, int nsg,
                                                             float *__restrict__ out) {
    constexpr int kWin = kIncT + kIncSpan;
    static_assert(kWin == 2 * 64 * kIncW, "two window samples per lane and channel");
    // two buffers, alternating by pair: a pair's windows are stored while the
    // previous pair's are still being summed, one barrier per pair
    __shared__ float win[2][2][kWin];
    const int lw = xcd_remap(blockIdx.x, gridDim.x);
    const int sgi = lw % nsg;
    const int tile = (lw / nsg) % ntile;
    const long long d = lw / ((long long)nsg * ntile);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int kg = sgi * kIncG + wv * kIncK;
    const long long t0 = (long long)tile * kIncT;
    float acc[kIncK][kIncS];
#pragma unroll
    for (int k = 0; k < kIncK; ++k)
#pragma unroll
        for (int j = 0; j < kIncS; ++j)
            acc[k][j] = 0.f;
    const int *dk = D + ((d * nsg + sgi) * ((a.nch + 1) / 2)) * 32;
    const float *row = ft + d * a.nch * a.ntime + t0;
    const int room = (int)(a.ntime - 1 - t0);
    // a pair's delays as this wave needs them: both channels' first delay and
    // the three words holding its own twelve offsets
    struct Dl {
        int lo[2], span[2];
        int w[2][3];
    };
    const auto delays = [&](int p, Dl &r) {
        const int *rec = dk + 32 * p;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            r.lo[c] = rec[16 * c];
            r.span[c] = rec[16 * c + 1 + kIncG / 4];
#pragma unroll
            for (int q = 0; q < 3; ++q)
                r.w[c][q] = rec[16 * c + 1 + 3 * wv + q];
        }
    };
    const auto offset = [](const Dl &r, int c, int k) {
        return (int)(((unsigned)r.w[c][k / 4] >> (8 * (k % 4))) & 0xffu);
    };
    // the window covers kIncT samples plus the supergroup's spread; loads
    // past it fall outside the view and read 0 without touching memory
    const auto fetch = [&](bool real, const float *r, int lo, int span, float (&pf)[2]) {
        if (real) {
            const auto v = inc_view(r + lo, min(room - lo + 1, kIncT + span));
            pf[0] = inc_load(v, 4 * tid);
            pf[1] = inc_load(v, 4 * (tid + 64 * kIncW));
        } else {
            pf[0] = pf[1] = 0.f;
        }
    };
    const auto sums = [&](const Dl &dl, int buf) {
        int held[2];
        float w[2][kIncS];
#pragma unroll
        for (int k = 0; k < kIncK; ++k) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int o = offset(dl, c, k);
                if (k == 0 || o != held[c]) {
                    held[c] = o;
#pragma unroll
                    for (int j = 0; j < kIncS; ++j)
                        w[c][j] = win[buf][c][lane + 64 * j + o];
                }
            }
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int j = 0; j < kIncS; ++j)
                    inc_add(acc[k][j], w[c][j]);
        }
    };
    const int npair = (a.nch + 1) / 2;
    Dl dla, dlb, dlc;
    float pf[2][2];
    delays(0, dla);
    if (npair > 1)
        delays(1, dlb);
    fetch(true, row, dla.lo[0], dla.span[0], pf[0]);
    fetch(a.nch > 1, row + a.ntime, dla.lo[1], dla.span[1], pf[1]);
    const auto pair = [&](int p, const Dl &cur, const Dl &nxt, Dl &far) {
        // buffer p & 1 was last read for pair p - 2, which every wave summed
        // before the previous pair's barrier
        const int buf = p & 1;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            win[buf][c][tid] = pf[c][0];
            win[buf][c][tid + 64 * kIncW] = pf[c][1];
        }
        row += 2 * a.ntime;
        if (p + 1 < npair) {
            fetch(true, row, nxt.lo[0], nxt.span[0], pf[0]);
            fetch(2 * p + 3 < a.nch, row + a.ntime, nxt.lo[1], nxt.span[1], pf[1]);
        }
        if (p + 2 < npair)
            delays(p + 2, far);
        __syncthreads();
        sums(cur, buf);
    };
    int p = 0;
    for (; p + 2 < npair; p += 3) {
        pair(p, dla, dlb, dlc);
        pair(p + 1, dlb, dlc, dla);
        pair(p + 2, dlc, dla, dlb);
    }
    if (p < npair)
        pair(p, dla, dlb, dlc);
    if (p + 1 < npair)
        pair(p + 1, dlb, dlc, dla);
    const int nk = min(kIncK, a.ntrial - kg);
#pragma unroll
    for (int k = 0; k < kIncK; ++k) {
        if (k < nk) {
            float *o = out + (d * a.ntrial + kg + k) * a.nout + t0 + lane;
#pragma unroll
            for (int j = 0; j < kIncS; ++j)
                if (t0 + lane + 64 * j < a.nout)
                    o[64 * j] = acc[k][j];
        }
    }
}

// Bound on the delay spread of kIncK consecutive trials in any channel: the
// delay rint(c DM) of channel ch has c = k_DM u / tsamp, largest in the lowest
// channel, so the spread is at most c_max (kIncK - 1) ddm + 1.
bool inc_narrow(const IncArgs &a, int ntrials = kIncK) {
    const double nu = inc_frequency(a, a.nch - 1), top = inc_frequency(a, 0);
    const double cmax = kKdm * (1.0 / (nu * nu) - 1.0 / (top * top)) / a.tsamp;
    return cmax * (ntrials - 1) * a.ddm * (1.0 + 1e-9) + 2.0 < (double)kIncSpan;
}

int inc_setup(const cdmt_plan_s *p, int nblock, const double *dm_coh, int ndm, double ddm0,
              double ddm, int ntrial, IncArgs *a) {
    if (!p || nblock < 1 || ndm < 1 || !dm_coh || ntrial < 1 || !std::isfinite(ddm0) ||
        !std::isfinite(ddm) || (ntrial > 1 && !(ddm > 0.0)))
        return CDMT_E_ARG;
    std::memset(a, 0, sizeof(*a));
    a->nsub = p->nsub;
    a->nchan = p->nchan;
    a->nch = p->nsub * p->nchan;
    a->ntrial = ntrial;
    a->kpad = (ntrial + kIncK - 1) / kIncK * kIncK;
    a->chirp_ref = p->chirp_ref;
    a->ntime = (long long)nblock * p->tblk;
    a->f_centre = p->f_centre;
    a->bw = p->bw;
    a->tsamp = (double)(p->nchan * p->ndec) / (p->bw * 1e6);
    a->ddm0 = ddm0;
    a->ddm = ddm;
    // every trial DM non-negative (delays behind the top channel); the delay
    // grows with DM and is largest in the lowest channel
    double dmax = -1.0;
    for (int d = 0; d < ndm; ++d) {
        if (!std::isfinite(dm_coh[d]) || dm_coh[d] + (ddm0 + ddm * 0.0) < 0.0)
            return CDMT_E_ARG;
        dmax = std::fmax(dmax, dm_coh[d] + (ddm0 + ddm * (double)(ntrial - 1)));
    }
    if (a->ntime > 0x7fffffffLL)
        return CDMT_E_SHAPE;
    const long long dl = inc_delay(*a, dmax, a->nch - 1);
    a->nout = a->ntime - dl;
    if (a->nout < 1)
        return CDMT_E_SHAPE;
    // one workgroup per (DM, time tile, trial group) in a 1-D grid
    const long long groups = (long long)ndm * ((a->nout + kIncT - 1) / kIncT) * (a->kpad / kIncK);
    return groups <= 0x7fffffffLL ? CDMT_OK : CDMT_E_SHAPE;
}

}  // namespace

extern "C" {

int cdmt_incoherent_shape(cdmt_plan_t p, int nblock, const double *dm_coh, int ndm, double ddm0,
                          double ddm, int ntrial, long long *nout) {
    if (!nout)
        return CDMT_E_ARG;
    IncArgs a;
    const int st = inc_setup(p, nblock, dm_coh, ndm, ddm0, ddm, ntrial, &a);
    if (st)
        return st;
    *nout = a.nout;
    return CDMT_OK;
}

int cdmt_incoherent_workspace_size(cdmt_plan_t p, int nblock, int ndm, int ntrial, size_t *bytes) {
    if (!p || !bytes || nblock < 0 || ndm < 0 || ntrial < 0)
        return CDMT_E_ARG;
    const size_t nch = (size_t)p->nsub * p->nchan;
    const size_t ntime = (size_t)nblock * p->tblk;
    // a transposed copy of the filterbanks unless the plan writes them
    // channel-major already
    const size_t ft = p->out_layout ? 0 : (size_t)ndm * nch * ntime * sizeof(float);
    const size_t kpad = ((size_t)ntrial + kIncK - 1) / kIncK * kIncK;
    const size_t nsg = ((size_t)ntrial + kIncG - 1) / kIncG;
    const size_t table = std::max((size_t)ndm * kpad * nch,                 // [d][ch][k]
                                  (size_t)ndm * nsg * ((nch + 1) / 2) * 32); // shared layout
    *bytes = ((ft + 255) & ~(size_t)255) + table * sizeof(int);
    return CDMT_OK;
}

int cdmt_incoherent(cdmt_plan_t p, int nblock, const float *fb, const double *dm_coh, int ndm,
                    double ddm0, double ddm, int ntrial, void *ws, size_t ws_bytes, float *out,
                    void *hip_stream) {
    IncArgs a;
    int st = inc_setup(p, nblock, dm_coh, ndm, ddm0, ddm, ntrial, &a);
    if (st)
        return st;
    if (!fb || !ws || !out)
        return CDMT_E_ARG;
    size_t need = 0;
    cdmt_incoherent_workspace_size(p, nblock, ndm, ntrial, &need);
    if (ws_bytes < need)
        return CDMT_E_WORKSPACE;
    const long long tiles_t = (a.ntime + 31) / 32;
    const long long ndelay = ((long long)std::min(ndm, kIncDms) * a.kpad * a.nch + 255) / 256;
    if ((a.nch + 31) / 32 > 65535 || ndm > 65535 || ndelay > 0x7fffffffLL)
        return CDMT_E_SHAPE;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const bool chan_major = p->out_layout == 1;
    float *ft = chan_major ? nullptr : static_cast<float *>(ws);
    const size_t ftb = chan_major ? 0 : (size_t)ndm * a.nch * a.ntime * sizeof(float);
    int *D = reinterpret_cast<int *>(static_cast<char *>(ws) + ((ftb + 255) & ~(size_t)255));
    const bool narrow = a.ntrial == 1 || inc_narrow(a);
    // several trial groups share each staged window when there are more
    // than one and the spread of kIncG trials fits the window
    const bool shared = a.ntrial > kIncK && inc_narrow(a, kIncG);
    IncArgs as = a;
    as.kpad = (a.ntrial + kIncG - 1) / kIncG * kIncG;
    const int nsg = as.kpad / kIncG;
    for (int first = 0; first < ndm; first += kIncDms) {
        const int cnt = ndm - first < kIncDms ? ndm - first : kIncDms;
        IncDms dl;
        std::memset(&dl, 0, sizeof(dl));
        for (int i = 0; i < cnt; ++i)
            dl.dm[i] = dm_coh[first + i];
        if (shared) {
            const long long n = (long long)cnt * nsg * a.nch;
            inc_delays_shared<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(as, dl, first, cnt, D);
        } else {
            const long long n = (long long)cnt * (a.kpad / kIncK) * a.nch;
            inc_delays<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(a, dl, first, cnt,
                                                                  narrow ? 1 : 0, D);
        }
        if (hipGetLastError() != hipSuccess)
            return CDMT_E_DEVICE;
    }
    if (chan_major) {
        ft = const_cast<float *>(fb);                 // read as is (the kernels only read it)
    } else {
        if (a.nch % 4 == 0 && a.ntime % 4 == 0 && reinterpret_cast<uintptr_t>(fb) % 16 == 0 &&
            reinterpret_cast<uintptr_t>(ft) % 16 == 0)
            inc_transpose4<32, 256><<<dim3((unsigned)((a.ntime + 255) / 256),
                                           (unsigned)((a.nch + 31) / 32), (unsigned)ndm), 256, 0,
                                      s>>>(fb, ft, a.ntime, a.nch);
        else
            inc_transpose<<<dim3((unsigned)tiles_t, (unsigned)((a.nch + 31) / 32),
                                 (unsigned)ndm), 256, 0, s>>>(fb, ft, a.ntime, a.nch);
        if (hipGetLastError() != hipSuccess)
            return CDMT_E_DEVICE;
    }
    const int ntile = (int)((a.nout + kIncT - 1) / kIncT);
    if (shared) {
        const unsigned gs = (unsigned)((long long)ndm * ntile * nsg);
        inc_sum_shared<<<gs, 64 * kIncW, 0, s>>>(ft, D, as, ntile, nsg, out);
        return hipGetLastError() == hipSuccess ? CDMT_OK : CDMT_E_DEVICE;
    }
    const int ngroup = a.kpad / kIncK;
    const unsigned grid = (unsigned)((long long)ndm * ntile * ngroup);
    if (narrow)
        inc_sum<false><<<grid, 64, 0, s>>>(ft, D, a, ntile, ngroup, out);
    else
        inc_sum<true><<<grid, 64, 0, s>>>(ft, D, a, ntile, ngroup, out);
    return hipGetLastError() == hipSuccess ? CDMT_OK : CDMT_E_DEVICE;
}

}  // extern "C"
