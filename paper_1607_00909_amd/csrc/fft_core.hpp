// Workgroup-level complex FFT building blocks for gfx950.
//
// Data type: a "pair" (float4) holds the same sample or bin of both
// polarisations, (X.re, X.im, Y.re, Y.im); every butterfly works on both at
// once, so one twiddle or transfer-function factor serves two complex values.
//
// Transform layout: a P-point transform (P a power of two, 32 <= P <= 8192)
// is spread over T = P/R lanes (R = 8 or 16 elements per lane); lane tt holds
// elements tt + T*slot in registers v[slot], slot = 0..R-1, at the input and
// at the output (natural order both ways).  Stages are Stockham autosort,
// decimation in time: radix R while at least R elements remain, then one
// smaller radix.
// Between stages the values go through LDS once (write in the stage's output
// order, read back in the next stage's input order); the first stage reads
// registers and the last leaves its outputs in registers.
//
// Twiddles come from per-stage row tables (below), computed on the host in
// double precision; the forward sign conjugates them on the fly.
#pragma once

#include <hip/hip_runtime.h>

namespace cdmt {

typedef float4 cpair;

__device__ __forceinline__ cpair padd(cpair a, cpair b) {
    return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w);
}
__device__ __forceinline__ cpair psub(cpair a, cpair b) {
    return make_float4(a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w);
}
// both complex values times the complex number w
__device__ __forceinline__ cpair pmul(cpair a, float2 w) {
    return make_float4(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x,
                       a.z * w.x - a.w * w.y, a.z * w.y + a.w * w.x);
}
__device__ __forceinline__ cpair pscale(cpair a, float s) {
    return make_float4(a.x * s, a.y * s, a.z * s, a.w * s);
}
// the same operations on a single complex value (one polarisation)
__device__ __forceinline__ float2 padd(float2 a, float2 b) {
    return make_float2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ float2 psub(float2 a, float2 b) {
    return make_float2(a.x - b.x, a.y - b.y);
}
__device__ __forceinline__ float2 pmul(float2 a, float2 w) {
    return make_float2(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x);
}
template <int S>
__device__ __forceinline__ float2 pmuli(float2 a) {
    if constexpr (S > 0)
        return make_float2(-a.y, a.x);
    else
        return make_float2(a.y, -a.x);
}

// both complex values times S*i (S = +1 or -1)
template <int S>
__device__ __forceinline__ cpair pmuli(cpair a) {
    if constexpr (S > 0)
        return make_float4(-a.y, a.x, -a.w, a.z);
    else
        return make_float4(a.y, -a.x, a.w, -a.z);
}

// cos and sin of 2 pi e / 16
__device__ __forceinline__ constexpr float c16(int e) {
    constexpr float t[16] = {1.0f, 0.92387953251128674f, 0.70710678118654752f,
                             0.38268343236508977f, 0.0f, -0.38268343236508977f,
                             -0.70710678118654752f, -0.92387953251128674f, -1.0f,
                             -0.92387953251128674f, -0.70710678118654752f,
                             -0.38268343236508977f, 0.0f, 0.38268343236508977f,
                             0.70710678118654752f, 0.92387953251128674f};
    return t[e & 15];
}
__device__ __forceinline__ constexpr float s16(int e) { return c16(e + 12); }

// times exp(S 2 pi i E / 16), with the trivial and 1/sqrt(2) cases special-cased
template <int S, int E>
__device__ __forceinline__ cpair pmul16(cpair a) {
    constexpr int e = E & 15;
    if constexpr (e == 0) {
        return a;
    } else if constexpr (e == 4) {
        return pmuli<S>(a);
    } else if constexpr (e == 8) {
        return make_float4(-a.x, -a.y, -a.z, -a.w);
    } else if constexpr (e == 12) {
        return pmuli<-S>(a);
    } else if constexpr ((e & 3) == 2) {
        // (c + i S s) with |c| = |s| = 1/sqrt(2)
        constexpr float h = 0.70710678118654752f;
        constexpr float cr = (e == 2 || e == 14) ? h : -h;
        constexpr float ci = (e == 2 || e == 6) ? (S > 0 ? h : -h) : (S > 0 ? -h : h);
        // (a + ib)(cr + i ci) with |cr| = |ci|
        if constexpr (cr == ci) {
            return make_float4(cr * (a.x - a.y), cr * (a.x + a.y), cr * (a.z - a.w),
                               cr * (a.z + a.w));
        } else {
            return make_float4(cr * (a.x + a.y), cr * (a.y - a.x), cr * (a.z + a.w),
                               cr * (a.w - a.z));
        }
    } else {
        constexpr float cr = c16(e);
        constexpr float ci = S > 0 ? s16(e) : -s16(e);
        return make_float4(a.x * cr - a.y * ci, a.x * ci + a.y * cr, a.z * cr - a.w * ci,
                           a.z * ci + a.w * cr);
    }
}

template <int S, int E>
__device__ __forceinline__ float2 pmul16(float2 a) {
    constexpr int e = E & 15;
    if constexpr (e == 0) {
        return a;
    } else if constexpr (e == 4) {
        return pmuli<S>(a);
    } else if constexpr (e == 8) {
        return make_float2(-a.x, -a.y);
    } else if constexpr (e == 12) {
        return pmuli<-S>(a);
    } else if constexpr ((e & 3) == 2) {
        constexpr float h = 0.70710678118654752f;
        constexpr float cr = (e == 2 || e == 14) ? h : -h;
        constexpr float ci = (e == 2 || e == 6) ? (S > 0 ? h : -h) : (S > 0 ? -h : h);
        if constexpr (cr == ci)
            return make_float2(cr * (a.x - a.y), cr * (a.x + a.y));
        else
            return make_float2(cr * (a.x + a.y), cr * (a.y - a.x));
    } else {
        constexpr float cr = c16(e);
        constexpr float ci = S > 0 ? s16(e) : -s16(e);
        return make_float2(a.x * cr - a.y * ci, a.x * ci + a.y * cr);
    }
}

// ---------------------------------------------------------------------------
// Small DFTs in registers: y[k] = sum_n a[n] exp(S 2 pi i n k / r), natural
// order in and out.

template <int S, class T>
__device__ __forceinline__ void dft2(T *a) {
    T t = a[0];
    a[0] = padd(t, a[1]);
    a[1] = psub(t, a[1]);
}

template <int S, class T>
__device__ __forceinline__ void dft4(T &a0, T &a1, T &a2, T &a3) {
    T s02 = padd(a0, a2), d02 = psub(a0, a2);
    T s13 = padd(a1, a3), d13 = pmuli<S>(psub(a1, a3));
    a0 = padd(s02, s13);
    a2 = psub(s02, s13);
    a1 = padd(d02, d13);
    a3 = psub(d02, d13);
}

template <int S, class T>
__device__ __forceinline__ void dft4(T *a) { dft4<S>(a[0], a[1], a[2], a[3]); }

template <int S, class T>
__device__ __forceinline__ void dft8(T *a) {
    // even / odd split: y[k] = E[k] + w8^k O[k], y[k+4] = E[k] - w8^k O[k]
    T e[4] = {a[0], a[2], a[4], a[6]};
    T o[4] = {a[1], a[3], a[5], a[7]};
    dft4<S>(e);
    dft4<S>(o);
    o[1] = pmul16<S, 2>(o[1]);
    o[2] = pmul16<S, 4>(o[2]);
    o[3] = pmul16<S, 6>(o[3]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        a[k] = padd(e[k], o[k]);
        a[k + 4] = psub(e[k], o[k]);
    }
}

template <int S, class T>
__device__ __forceinline__ void dft16(T *a) {
    // n = 4m + e: four DFT-4 over m, twiddle w16^(e k'), four DFT-4 over e.
#pragma unroll
    for (int e = 0; e < 4; ++e)
        dft4<S>(a[e], a[e + 4], a[e + 8], a[e + 12]);
    a[5] = pmul16<S, 1>(a[5]);
    a[6] = pmul16<S, 2>(a[6]);
    a[7] = pmul16<S, 3>(a[7]);
    a[9] = pmul16<S, 2>(a[9]);
    a[10] = pmul16<S, 4>(a[10]);
    a[11] = pmul16<S, 6>(a[11]);
    a[13] = pmul16<S, 3>(a[13]);
    a[14] = pmul16<S, 6>(a[14]);
    a[15] = pmul16<S, 9>(a[15]);
#pragma unroll
    for (int k = 0; k < 4; ++k)
        dft4<S>(a[4 * k], a[4 * k + 1], a[4 * k + 2], a[4 * k + 3]);
    // y[k] sits at a[4 (k mod 4) + k / 4]: transpose the 4x4 block
    T y[16];
#pragma unroll
    for (int k = 0; k < 16; ++k)
        y[k] = a[4 * (k & 3) + (k >> 2)];
#pragma unroll
    for (int k = 0; k < 16; ++k)
        a[k] = y[k];
}

// The same 16-point DFT of pairs with the inner twiddles in tangent form:
// w16^1 = c1 (1 + i S t1), w16^3 = i S c1 (1 - i S t1), w16^9 = -w16^1,
// w16^2 = c2 (1 + i S), w16^6 = i S w16^2 (c1 = cos(pi/8), t1 = tan(pi/8),
// c2 = 1/sqrt(2)): the rotations by (1 +- i S t1) are two fused multiply-adds
// per complex value and (1 + i S) two additions, and the common factors c1
// and c2 of a row ride in the fused multiply-adds of its second-stage
// butterflies, so no multiplication is spent on them (144 instead of 160
// operations per complex transform).
template <int S>
__device__ __forceinline__ cpair rot_t(cpair z, float t) {   // z (1 + i S t)
    const float st = S > 0 ? t : -t;
    return make_float4(fmaf(-st, z.y, z.x), fmaf(st, z.x, z.y), fmaf(-st, z.w, z.z),
                       fmaf(st, z.z, z.w));
}
template <int S>
__device__ __forceinline__ cpair rot_1(cpair z) {            // z (1 + i S)
    if constexpr (S > 0)
        return make_float4(z.x - z.y, z.y + z.x, z.z - z.w, z.w + z.z);
    else
        return make_float4(z.x + z.y, z.y - z.x, z.z + z.w, z.w - z.z);
}
__device__ __forceinline__ cpair pfma(cpair p, float c, cpair q) {   // p + c q
    return make_float4(fmaf(c, q.x, p.x), fmaf(c, q.y, p.y), fmaf(c, q.z, p.z), fmaf(c, q.w, p.w));
}
template <int S>
__device__ __forceinline__ void dft16t(cpair *a) {
    constexpr float c1 = 0.92387953251128674f, t1 = 0.41421356237309505f;
    constexpr float c2 = 0.70710678118654752f;
#pragma unroll
    for (int e = 0; e < 4; ++e)
        dft4<S>(a[e], a[e + 4], a[e + 8], a[e + 12]);
    dft4<S>(a[0], a[1], a[2], a[3]);
    {   // row 1: twiddles w^1, w^2, w^3
        const cpair r5 = rot_t<S>(a[5], t1), q6 = rot_1<S>(a[6]), r7 = rot_t<S>(a[7], -t1);
        const cpair s02 = pfma(a[4], c2, q6), d02 = pfma(a[4], -c2, q6);
        const cpair u = padd(r5, pmuli<S>(r7)), v = padd(pmuli<S>(r5), r7);
        a[4] = pfma(s02, c1, u);
        a[6] = pfma(s02, -c1, u);
        a[5] = pfma(d02, c1, v);
        a[7] = pfma(d02, -c1, v);
    }
    {   // row 2: w^2, w^4 = i S, w^6
        const cpair q9 = rot_1<S>(a[9]), q11 = rot_1<S>(a[11]), i10 = pmuli<S>(a[10]);
        const cpair s02 = padd(a[8], i10), d02 = psub(a[8], i10);
        const cpair u = padd(q9, pmuli<S>(q11)), v = padd(pmuli<S>(q9), q11);
        a[8] = pfma(s02, c2, u);
        a[10] = pfma(s02, -c2, u);
        a[9] = pfma(d02, c2, v);
        a[11] = pfma(d02, -c2, v);
    }
    {   // row 3: w^3, w^6, w^9
        const cpair r13 = rot_t<S>(a[13], -t1), q14 = rot_1<S>(a[14]), r15 = rot_t<S>(a[15], t1);
        const cpair iq14 = pmuli<S>(q14);
        const cpair s02 = pfma(a[12], c2, iq14), d02 = pfma(a[12], -c2, iq14);
        const cpair u = psub(pmuli<S>(r13), r15), v = psub(pmuli<S>(r15), r13);
        a[12] = pfma(s02, c1, u);
        a[14] = pfma(s02, -c1, u);
        a[13] = pfma(d02, c1, v);
        a[15] = pfma(d02, -c1, v);
    }
    // y[k] sits at a[4 (k mod 4) + k / 4]: transpose the 4x4 block
    cpair y[16];
#pragma unroll
    for (int k = 0; k < 16; ++k)
        y[k] = a[4 * (k & 3) + (k >> 2)];
#pragma unroll
    for (int k = 0; k < 16; ++k)
        a[k] = y[k];
}

template <int R, int S, class T>
__device__ __forceinline__ void dft(T *a) {
    if constexpr (R == 16)
        dft16<S>(a);
    else if constexpr (R == 8)
        dft8<S>(a);
    else if constexpr (R == 4)
        dft4<S>(a);
    else if constexpr (R == 2)
        dft2<S>(a);
}

// ---------------------------------------------------------------------------
// LDS views of one transform's elements.

// element e at base[e + e/PAD]: one padding slot per PAD elements keeps the
// stride-R writes of the first stage spread over the banks (PAD = R)
template <int PAD>
struct LdsPad {
    cpair *base;
    __device__ __forceinline__ void store(int e, cpair v) const { base[e + e / PAD] = v; }
    __device__ __forceinline__ cpair load(int e) const { return base[e + e / PAD]; }
};
typedef LdsPad<16> LdsPadded;

// element e of transform f at base[e*C + f]: several transforms interleaved,
// consecutive lanes (consecutive f) touch consecutive addresses
template <int C>
struct LdsInterleaved {
    cpair *base;  // already offset by f
    __device__ __forceinline__ void store(int e, cpair v) const { base[e * C] = v; }
    __device__ __forceinline__ cpair load(int e) const { return base[e * C]; }
};

// ---------------------------------------------------------------------------
// Twiddle row tables.  For a stage of radix r that completes sub-transforms
// of length L = NS * r, lane butterfly j needs exp(+2 pi i k q / L) for
// k = j mod NS and q = 0..r-1.  Row k of the table for (L, r) holds exactly
// these r values, so a lane fetches its twiddles with r/2 16-byte loads.
// Family r (r = 2, 4, 8, 16) occupies 16384 entries; the table for L starts
// at entry L of its family (L <= 8192).  Filled once per device from double
// precision on the host.
constexpr int kStageFamily = 16384;
__device__ __align__(16) float2 g_stage_tw[4 * kStageFamily];

template <int r>
__device__ __forceinline__ const float2 *stage_table(int len) {
    constexpr int fam = r == 2 ? 0 : r == 4 ? 1 : r == 8 ? 2 : 3;
    return g_stage_tw + fam * kStageFamily + len;
}

// ---------------------------------------------------------------------------
// One Stockham stage (and, recursively, the rest) of a P-point transform with
// sign S, R elements per lane (R = 8 or 16).  NS = product of the radices
// already applied.  w holds this stage's twiddles (w[u*r + q] for butterfly
// u, input q); the next stage's rows are fetched before the LDS exchange so
// that their latency overlaps the barrier.
template <int P, int R, int NS, int S>
struct Stage {
    static constexpr int T = P / R;
    static constexpr int r = (P / NS >= R) ? R : P / NS;
    static constexpr int U = R / r;          // butterflies per lane
    static constexpr bool LAST = (NS * r == P);

    __device__ __forceinline__ static void load_twiddles(float2 (&w)[R], int tt) {
        if constexpr (NS > 1) {
            const float2 *tab = stage_table<r>(NS * r);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = (tt + T * u) & (NS - 1);
                const float4 *row = reinterpret_cast<const float4 *>(tab + k * r);
#pragma unroll
                for (int h = 0; h < r / 2; ++h) {
                    const float4 x = row[h];
                    w[u * r + 2 * h] = make_float2(x.x, x.y);
                    w[u * r + 2 * h + 1] = make_float2(x.z, x.w);
                }
            }
        }
    }

    template <class Lds>
    __device__ __forceinline__ static void run(cpair (&v)[R], int tt, const Lds &lds,
                                               const float2 (&w)[R]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = tt + T * u;
            const int k = j & (NS - 1);
            cpair a[r];
#pragma unroll
            for (int q = 0; q < r; ++q)
                a[q] = v[u + q * U];
            if constexpr (NS > 1) {
#pragma unroll
                for (int q = 1; q < r; ++q) {
                    float2 tw = w[u * r + q];
                    if constexpr (S < 0)
                        tw.y = -tw.y;
                    a[q] = pmul(a[q], tw);
                }
            }
            dft<r, S>(a);
            if constexpr (LAST) {
#pragma unroll
                for (int q = 0; q < r; ++q)
                    v[u + q * U] = a[q];
            } else {
                const int base = (j / NS) * NS * r + k;
#pragma unroll
                for (int q = 0; q < r; ++q)
                    lds.store(base + q * NS, a[q]);
            }
        }
        if constexpr (!LAST) {
            using Next = Stage<P, R, NS * r, S>;
            float2 wn[R];
            Next::load_twiddles(wn, tt);
            __syncthreads();
#pragma unroll
            for (int s = 0; s < R; ++s)
                v[s] = lds.load(tt + T * s);
            __syncthreads();
            Next::run(v, tt, lds, wn);
        }
    }
};

// Whole P-point transform of the lane's registers (first stage has no
// twiddles).
template <int P, int S, int R, class Lds>
__device__ __forceinline__ void wg_fft(cpair (&v)[R], int tt, const Lds &lds) {
    float2 w0[R];
    Stage<P, R, 1, S>::run(v, tt, lds, w0);
}

}  // namespace cdmt
