// LDS throughput probe on gfx950: CU clocks per wave64 LDS instruction for
// 128-, 64- and 32-bit reads and writes at several lane strides.
//
// Lane l of every wave addresses slot l * stride of a 16-byte-slot buffer
// (the stride in 16-byte slots; for 32-bit writes in 4-byte words).  Each
// loop trip issues 8 instructions of one form and waits for them; two
// 256-lane workgroups per CU.  The buffer holds 64 * 33 + 64 slots, past the
// largest address used (63 * 33 slots + 16 bytes), so every access is in
// bounds; the kernel writes one float per lane into a buffer sized for the
// grid.  Clocks are at the nominal 2.4 GHz.
//
// Build:  hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature
//         -Xclang -packed-fp32-ops lds_rate.hip -o lds_rate
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

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));

enum Form { READ128, WRITE128, WRITE64X2, WRITE2_64, WRITE32 };
constexpr int kSlots = 64 * 33 + 64;
constexpr int kCUs = 256, kBlocksPerCU = 2;

#define X8(s) s s s s s s s s

template <int F>
__global__ __launch_bounds__(256) void lds_probe(float *out, int stride, int trips) {
    __shared__ float4 buf[kSlots];
    const int lane = threadIdx.x & 63;
    const unsigned a16 = (unsigned)(lane * stride) * 16u;
    const unsigned a4 = (unsigned)(lane * stride) * 4u;
    f4 v = {(float)lane, 1.f, 2.f, 3.f};
    for (int i = threadIdx.x; i < kSlots; i += 256)
        buf[i] = make_float4(v.x, v.y, v.z, v.w);
    __syncthreads();
    const f2 lo = v.xy, hi = v.zw;
    for (int t = 0; t < trips; ++t) {
        if constexpr (F == READ128) {
            f4 r0, r1;
            asm volatile("ds_read_b128 %0, %2\n ds_read_b128 %1, %2\n ds_read_b128 %0, %2\n ds_read_b128 %1, %2\n"
                         "ds_read_b128 %0, %2\n ds_read_b128 %1, %2\n ds_read_b128 %0, %2\n ds_read_b128 %1, %2\n"
                         "s_waitcnt lgkmcnt(0)"
                         : "=&v"(r0), "=&v"(r1) : "v"(a16) : "memory");
            v.x += r0.x + r1.y;
        } else if constexpr (F == WRITE128) {
            asm volatile(X8("ds_write_b128 %0, %1\n") "s_waitcnt lgkmcnt(0)"
                         :: "v"(a16), "v"(v) : "memory");
        } else if constexpr (F == WRITE64X2) {
            asm volatile(X8("ds_write_b64 %0, %1\n") "s_waitcnt lgkmcnt(0)"
                         :: "v"(a16), "v"(lo) : "memory");
        } else if constexpr (F == WRITE2_64) {
            asm volatile(X8("ds_write2_b64 %0, %1, %2 offset1:1\n") "s_waitcnt lgkmcnt(0)"
                         :: "v"(a16), "v"(lo), "v"(hi) : "memory");
        } else {
            asm volatile(X8("ds_write_b32 %0, %1\n") "s_waitcnt lgkmcnt(0)"
                         :: "v"(a4), "v"(v.x) : "memory");
        }
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = v.x;
}

template <int F>
int measure(const char *name, float *out, int stride) {
    const int blocks = kCUs * kBlocksPerCU, trips = 2048;
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    lds_probe<F><<<blocks, 256>>>(out, stride, trips);   // warm-up
    CHECK(hipGetLastError());
    CHECK(hipEventRecord(e0));
    lds_probe<F><<<blocks, 256>>>(out, stride, trips);
    CHECK(hipEventRecord(e1));
    CHECK(hipEventSynchronize(e1));
    float ms = 0.f;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    const double per_cu = 4.0 * kBlocksPerCU * trips * 8.0;   // wave instructions per CU
    const int bytes = F == WRITE32 ? 4 : F == WRITE64X2 ? 8 : 16;
    const double clk = ms * 1e-3 * 2.4e9 / per_cu;
    std::printf("| %s | %d | %.3f | %.2f | %.0f |\n", name, stride, ms, clk, 64.0 * bytes / clk);
    CHECK(hipEventDestroy(e0));
    CHECK(hipEventDestroy(e1));
    return 0;
}

int main() {
    float *out = nullptr;
    CHECK(hipMalloc(&out, sizeof(float) * kCUs * kBlocksPerCU * 256));
    std::printf("| instruction | lane stride | ms | CU clocks per wave instruction | bytes per CU clock |\n");
    std::printf("|---|---|---|---|---|\n");
    for (int s : {1, 17, 33}) {
        if (measure<READ128>("ds_read_b128", out, s) || measure<WRITE128>("ds_write_b128", out, s) ||
            measure<WRITE64X2>("ds_write_b64", out, s) ||
            measure<WRITE2_64>("ds_write2_b64 (16 B)", out, s))
            return 1;
    }
    for (int s : {1, 17})
        if (measure<WRITE32>("ds_write_b32", out, s))
            return 1;
    CHECK(hipFree(out));
    std::printf("done\n");
    return 0;
}
