// Issue-rate probe for wave64 FP32 vector instructions on gfx950.
//
// Each lane runs CH independent (or, with CH = 1, dependent) chains of one
// instruction form, 8 x CH instructions per loop trip; the launch holds one,
// two or four 256-lane workgroups per CU, i.e. one, two or four waves per
// SIMD.  The figure printed is SIMD clocks per retired wave instruction at the
// nominal 2.4 GHz engine clock.  The forms are written as inline assembly so
// that the compiler neither merges nor re-encodes them.  The kernel reads no
// memory and writes one float per lane into a buffer sized for the largest
// grid, so every access is in bounds.
//
// Build:  hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature
//         -Xclang -packed-fp32-ops valu_rate.hip -o valu_rate
#include <hip/hip_runtime.h>

#include <cstdio>

#define CHECK(x)                                                                 \
    do {                                                                         \
        hipError_t e_ = (x);                                                     \
        if (e_ != hipSuccess) {                                                  \
            std::printf("HIP error %s (line %d)\n", hipGetErrorString(e_), __LINE__); \
            return 1;                                                            \
        }                                                                        \
    } while (0)

enum Form { ADD, MUL, FMAC, FMA3, MOV };

template <int F, int CH>
__global__ __launch_bounds__(256) void chains(float *out, int trips, float b, float c) {
    float a[CH];
#pragma unroll
    for (int i = 0; i < CH; ++i)
        a[i] = threadIdx.x * 1e-3f + i;
    const float bb = b + threadIdx.x * 1e-7f;
    for (int t = 0; t < trips; ++t) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                if constexpr (F == ADD)
                    asm volatile("v_add_f32 %0, %1, %0" : "+v"(a[i]) : "v"(bb));
                else if constexpr (F == MUL)
                    asm volatile("v_mul_f32 %0, %1, %0" : "+v"(a[i]) : "v"(bb));
                else if constexpr (F == FMAC)
                    asm volatile("v_fmac_f32 %0, %1, %2" : "+v"(a[i]) : "v"(bb), "v"(c));
                else if constexpr (F == FMA3)
                    asm volatile("v_fma_f32 %0, -%1, %2, %0" : "+v"(a[i]) : "v"(bb), "v"(c));
                else
                    asm volatile("v_mov_b32 %0, %1" : "=v"(a[i]) : "v"(a[(i + 1) % CH]));
            }
        }
    }
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < CH; ++i)
        s += a[i];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

constexpr int kCUs = 256, kSimds = 1024, kMaxBlocksPerCU = 4;

template <int F, int CH>
int measure(const char *name, float *out, int blocks_per_cu, int trips) {
    const int blocks = kCUs * blocks_per_cu;
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    chains<F, CH><<<blocks, 256>>>(out, trips, 1.0000001f, 0.5f);   // warm-up
    CHECK(hipGetLastError());
    CHECK(hipEventRecord(e0));
    chains<F, CH><<<blocks, 256>>>(out, trips, 1.0000001f, 0.5f);
    CHECK(hipEventRecord(e1));
    CHECK(hipEventSynchronize(e1));
    float ms = 0.f;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    const double waves = 4.0 * blocks;
    const double per_simd = waves * trips * 8.0 * CH / kSimds;
    std::printf("| %-9s | %s | %d | %.3f | %.2f |\n", name, CH == 1 ? "dependent" : "8 chains",
                blocks_per_cu, ms, ms * 1e-3 * 2.4e9 / per_simd);
    CHECK(hipEventDestroy(e0));
    CHECK(hipEventDestroy(e1));
    return 0;
}

int main() {
    float *out = nullptr;
    CHECK(hipMalloc(&out, sizeof(float) * kCUs * kMaxBlocksPerCU * 256));
    const int trips = 4096;
    std::printf("| form | chains per lane | waves per SIMD | ms | SIMD clocks per wave instruction |\n");
    std::printf("|---|---|---|---|---|\n");
    for (int bpc = 1; bpc <= kMaxBlocksPerCU; bpc *= 2) {
        if (measure<ADD, 8>("v_add", out, bpc, trips) || measure<MUL, 8>("v_mul", out, bpc, trips) ||
            measure<FMAC, 8>("v_fmac", out, bpc, trips) ||
            measure<FMA3, 8>("v_fma", out, bpc, trips) ||
            measure<MOV, 8>("v_mov", out, bpc, trips) ||
            measure<FMAC, 1>("v_fmac", out, bpc, trips))
            return 1;
    }
    CHECK(hipFree(out));
    std::printf("done\n");
    return 0;
}
