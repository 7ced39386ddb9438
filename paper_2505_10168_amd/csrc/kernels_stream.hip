// Plain streaming kernels that calibrate what this device sustains on HBM: a copy
// (one read stream, one write stream) and a triad y = a + s b (two reads, one write,
// the read/write mix of the fused smoothing passes).  They use the access pattern of
// those passes: 16-byte loads and stores, consecutive lanes on consecutive 16-byte
// chunks, several chunks in flight per thread, non-temporal stores optional.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "stmg_launch.hpp"

namespace stmg {

namespace {

constexpr int kStreamBlock = 256;
constexpr int kStreamUnroll = 4;   // 16-byte chunks per thread in flight

template <bool NT>
__device__ __forceinline__ void store2(double* p, double2 v) {
    if constexpr (NT) {
        __builtin_nontemporal_store(v.x, p);
        __builtin_nontemporal_store(v.y, p + 1);
    } else {
        *reinterpret_cast<double2*>(p) = v;
    }
}

// n2 = number of double2 chunks; every thread handles kStreamUnroll chunks spaced by
// the block size, blocks take consecutive tiles of kStreamBlock * kStreamUnroll chunks
template <bool NT, bool TRIAD>
__global__ __launch_bounds__(kStreamBlock) void k_stream(const double* __restrict__ a,
                                                         const double* __restrict__ b,
                                                         double s, double* __restrict__ y,
                                                         int64_t n2) {
    const int64_t tile = (int64_t)kStreamBlock * kStreamUnroll;
    const int64_t base = (int64_t)blockIdx.x * tile + threadIdx.x;
    double2 va[kStreamUnroll], vb[kStreamUnroll];
#pragma unroll
    for (int k = 0; k < kStreamUnroll; ++k) {
        const int64_t i = base + (int64_t)k * kStreamBlock;
        if (i < n2) {
            va[k] = reinterpret_cast<const double2*>(a)[i];
            if constexpr (TRIAD) vb[k] = reinterpret_cast<const double2*>(b)[i];
        }
    }
#pragma unroll
    for (int k = 0; k < kStreamUnroll; ++k) {
        const int64_t i = base + (int64_t)k * kStreamBlock;
        if (i < n2) {
            double2 v = va[k];
            if constexpr (TRIAD) {
                v.x = __builtin_fma(s, vb[k].x, v.x);
                v.y = __builtin_fma(s, vb[k].y, v.y);
            }
            store2<NT>(y + 2 * i, v);
        }
    }
}

}  // namespace

int launch_stream(const double* a, const double* b, double s, double* y, int64_t n, bool nt,
                  hipStream_t st) {
    if (n < 0 || (n & 1)) return -1;
    const int64_t n2 = n / 2;
    const int64_t tile = (int64_t)kStreamBlock * kStreamUnroll;
    const int64_t blocks = (n2 + tile - 1) / tile;
    if (blocks == 0) return 0;
    if (blocks > 0x7fffffff) return -1;
    const dim3 g((unsigned)blocks), t(kStreamBlock);
    if (b) {
        if (nt) hipLaunchKernelGGL((k_stream<true, true>), g, t, 0, st, a, b, s, y, n2);
        else hipLaunchKernelGGL((k_stream<false, true>), g, t, 0, st, a, b, s, y, n2);
    } else {
        if (nt) hipLaunchKernelGGL((k_stream<true, false>), g, t, 0, st, a, b, s, y, n2);
        else hipLaunchKernelGGL((k_stream<false, false>), g, t, 0, st, a, b, s, y, n2);
    }
    return 0;
}

}  // namespace stmg
