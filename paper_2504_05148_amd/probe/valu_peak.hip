// Vector-ALU throughput probe: the instruction rate of the integer ops the
// SGM kernels are made of, measured on the device the library runs on.  Each
// lane runs 16 independent chains of one operation in a loop (no dependency
// between consecutive instructions of a wave), enough waves to fill every
// SIMD, and the rate is instructions x 64 lanes / elapsed time.  The ops:
//   0 v_pk_add_u16       1 v_pk_min_u16      2 v_pk_minimum3_f16
//   3 v_add3_u32         4 v_alignbit_b32    5 v_bcnt_u32_b32
//   6 v_xor_b32          7 v_min_u32 with a DPP row rotation
#include <hip/hip_runtime.h>
#include <cstdint>

#include "../../include/valu_peak.h"

namespace {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

template <int OP>
__device__ __forceinline__ uint32_t op(uint32_t a, uint32_t b, uint32_t c)
{
    if constexpr (OP == 0) {
        return __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, a) + __builtin_bit_cast(u16x2, b));
    } else if constexpr (OP == 1) {
        return __builtin_bit_cast(uint32_t, __builtin_elementwise_min(__builtin_bit_cast(u16x2, a),
                                                                      __builtin_bit_cast(u16x2, b)));
    } else if constexpr (OP == 2) {
        const f16x2 x = __builtin_bit_cast(f16x2, a), y = __builtin_bit_cast(f16x2, b),
                    z = __builtin_bit_cast(f16x2, c);
        return __builtin_bit_cast(uint32_t, __builtin_elementwise_minimum(
                                                __builtin_elementwise_minimum(x, y), z));
    } else if constexpr (OP == 3) {
        return a + b + c;
    } else if constexpr (OP == 4) {
        // written out: the compiler folds chains of the builtin
        uint32_t r;
        asm volatile("v_alignbit_b32 %0, %1, %2, 16" : "=v"(r) : "v"(a), "v"(b));
        return r;
    } else if constexpr (OP == 5) {
        return __builtin_popcount(b) + a;
    } else if constexpr (OP == 6) {
        uint32_t r;
        asm volatile("v_xor_b32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
        return r;
    } else {
        // row_ror:1 (DPP control 0x121)
        return min(a, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)b, 0x121, 0xf, 0xf, false));
    }
}

constexpr int kChains = 16;
constexpr int kUnroll = 8;

template <int OP>
__global__ __launch_bounds__(256) void valu_peak_kernel(uint32_t* out, int iters, uint32_t seed)
{
    uint32_t r[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) r[k] = (seed * (threadIdx.x + 7 * k + 1)) & 0x3bff3bffu;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
            for (int k = 0; k < kChains; ++k)
                r[k] = op<OP>(r[k], r[(k + 5) % kChains], r[(k + 11) % kChains]);
        }
    }
    uint32_t x = 0;
#pragma unroll
    for (int k = 0; k < kChains; ++k) x ^= r[k];
    if (x == seed) out[blockIdx.x * blockDim.x + threadIdx.x] = x;   // never taken in practice
}

template <int OP>
hipError_t launch(uint32_t* out, int blocks, int iters, uint32_t seed, hipStream_t s)
{
    hipLaunchKernelGGL(valu_peak_kernel<OP>, dim3(blocks), dim3(256), 0, s, out, iters, seed);
    return hipGetLastError();
}

}  // namespace

extern "C" int valu_peak_ops(void)
{
    return kValuPeakOps;
}

extern "C" int valu_peak_measure(int op, int iters, double* lane_ops_per_s, double* ms)
{
    if (op < 0 || op >= kValuPeakOps || iters < 1 || iters > (1 << 20) || !lane_ops_per_s || !ms)
        return 1;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 2;
    // 4 waves of 256 lanes per SIMD: 16 x 64 lanes per compute unit, 8 blocks
    const int blocks = cus * 8;
    uint32_t* out = nullptr;
    hipEvent_t e0, e1;
    if (hipMalloc(&out, (size_t)blocks * 256 * 4) != hipSuccess) return 2;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipFree(out);
        return 2;
    }
    hipStream_t s = nullptr;
    auto run = [&](int n) {
        switch (op) {
        case 0: return launch<0>(out, blocks, n, 0x9e3779b9u, s);
        case 1: return launch<1>(out, blocks, n, 0x9e3779b9u, s);
        case 2: return launch<2>(out, blocks, n, 0x9e3779b9u, s);
        case 3: return launch<3>(out, blocks, n, 0x9e3779b9u, s);
        case 4: return launch<4>(out, blocks, n, 0x9e3779b9u, s);
        case 5: return launch<5>(out, blocks, n, 0x9e3779b9u, s);
        case 6: return launch<6>(out, blocks, n, 0x9e3779b9u, s);
        default: return launch<7>(out, blocks, n, 0x9e3779b9u, s);
        }
    };
    int rc = 0;
    float t = 0.f;
    if (run(iters / 8 + 1) != hipSuccess || hipEventRecord(e0, s) != hipSuccess ||
        run(iters) != hipSuccess || hipEventRecord(e1, s) != hipSuccess ||
        hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess)
        rc = 2;
    if (rc == 0) {
        const double insts = (double)blocks * 4 * iters * kUnroll * kChains;   // wave instructions
        *ms = t;
        *lane_ops_per_s = insts * 64 / (t * 1e-3);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(out);
    return rc;
}
