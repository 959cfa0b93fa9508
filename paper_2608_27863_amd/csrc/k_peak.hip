// Attainable peaks of this chip, measured by the library itself, so that each
// roofline fraction can be given against the datasheet and against what a
// plain kernel reaches:
//   k_peak_mfma  back-to-back 16x16x4 matrix-core products (FP64 or FP32) from
//                register operands, kPeakChains independent accumulators per
//                wave, no memory traffic but one store per lane at the end
//   k_peak_read  a streaming read in 64 KB chunks per workgroup, four
//                nontemporal 16-byte loads in flight per lane, the words
//                XOR-reduced into one value
//   k_peak_copy  the same walk copying, nontemporal loads and stores
// The matrix-core accumulators must sit in VGPRs (the library is built with
// -amdgpu-mfma-vgpr-form): with AGPR accumulators the FP64 16x16x4 product
// issues at about two thirds of the rate.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "hdg_internal.h"

namespace hdg {
namespace {

constexpr int kPeakChains = 8;  // independent accumulators per wave

template <typename T> struct PeakOp;
template <> struct PeakOp<double> {
    typedef double acc_t __attribute__((ext_vector_type(4)));
    __device__ static acc_t mfma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <> struct PeakOp<float> {
    typedef float acc_t __attribute__((ext_vector_type(4)));
    __device__ static acc_t mfma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

// Every operand equals `one`, so each product adds 4 one^2 to every output and
// lane l's sink value is kPeakChains * 4 * (4 iters one^2).
template <typename T>
__global__ void __launch_bounds__(256) k_peak_mfma(int iters, T one, T *__restrict__ sink) {
    typedef typename PeakOp<T>::acc_t acc_t;
    acc_t acc[kPeakChains];
#pragma unroll
    for (int j = 0; j < kPeakChains; ++j) acc[j] = (acc_t){T(0), T(0), T(0), T(0)};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < kPeakChains; ++j) acc[j] = PeakOp<T>::mfma(one, one, acc[j]);
    }
    T s = T(0);
#pragma unroll
    for (int j = 0; j < kPeakChains; ++j) s += (acc[j][0] + acc[j][1]) + (acc[j][2] + acc[j][3]);
    sink[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

typedef unsigned int u4 __attribute__((ext_vector_type(4)));
// Each workgroup streams whole chunks of kChunk16 16-byte units (64 KB), four
// nontemporal 4 KB rows of its chunk in flight; chunk c goes to workgroup
// c mod the grid.  Contiguous chunks per workgroup read faster than a
// grid-stride walk (7.2 against 6.4 TB/s on 4 GiB).
constexpr int kPeakBlocks = 1024;
constexpr int64_t kChunk16 = 4096;

__global__ void __launch_bounds__(256) k_peak_read(const u4 *__restrict__ src, unsigned *__restrict__ sink,
                                                   int64_t n16) {
    unsigned x = 0;
    for (int64_t c0 = (int64_t)blockIdx.x * kChunk16; c0 < n16; c0 += (int64_t)gridDim.x * kChunk16) {
        const int64_t c1 = std::min(c0 + kChunk16, n16);
        int64_t i = c0 + threadIdx.x;
        for (; i + 3 * 256 < c1; i += 4 * 256) {
            u4 v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = __builtin_nontemporal_load(src + i + q * 256);
#pragma unroll
            for (int q = 0; q < 4; ++q) x ^= v[q].x ^ v[q].y ^ v[q].z ^ v[q].w;
        }
        for (; i < c1; i += 256) {
            const u4 v = src[i];
            x ^= v.x ^ v.y ^ v.z ^ v.w;
        }
    }
    __shared__ unsigned s_x;
    if (threadIdx.x == 0) s_x = 0;
    __syncthreads();
    atomicXor(&s_x, x);
    __syncthreads();
    if (threadIdx.x == 0) atomicXor(sink, s_x);
}

__global__ void __launch_bounds__(256) k_peak_copy(const u4 *__restrict__ src, u4 *__restrict__ dst, int64_t n16) {
    for (int64_t c0 = (int64_t)blockIdx.x * kChunk16; c0 < n16; c0 += (int64_t)gridDim.x * kChunk16) {
        const int64_t c1 = std::min(c0 + kChunk16, n16);
        int64_t i = c0 + threadIdx.x;
        for (; i + 3 * 256 < c1; i += 4 * 256) {
            u4 v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = __builtin_nontemporal_load(src + i + q * 256);
#pragma unroll
            for (int q = 0; q < 4; ++q) __builtin_nontemporal_store(v[q], dst + i + q * 256);
        }
        for (; i < c1; i += 256) dst[i] = src[i];
    }
}

}  // namespace

int launch_peak_mfma(int fp_bits, int n_wg, int iters, double one, void *sink, hipStream_t s) {
    if (fp_bits == 64)
        hipLaunchKernelGGL(k_peak_mfma<double>, dim3(n_wg), dim3(256), 0, s, iters, one, (double *)sink);
    else
        hipLaunchKernelGGL(k_peak_mfma<float>, dim3(n_wg), dim3(256), 0, s, iters, (float)one, (float *)sink);
    return (int)hipGetLastError();
}

int launch_peak_read(const void *src, size_t bytes, unsigned *sink, hipStream_t s) {
    const int64_t n16 = (int64_t)(bytes / 16);
    const int64_t blocks = std::min<int64_t>((n16 + kChunk16 - 1) / kChunk16, kPeakBlocks);
    hipLaunchKernelGGL(k_peak_read, dim3((unsigned)blocks), dim3(256), 0, s, (const u4 *)src, sink, n16);
    return (int)hipGetLastError();
}

int launch_peak_copy(const void *src, void *dst, size_t bytes, hipStream_t s) {
    const int64_t n16 = (int64_t)(bytes / 16);
    const int64_t blocks = std::min<int64_t>((n16 + kChunk16 - 1) / kChunk16, kPeakBlocks);
    hipLaunchKernelGGL(k_peak_copy, dim3((unsigned)blocks), dim3(256), 0, s, (const u4 *)src, (u4 *)dst, n16);
    return (int)hipGetLastError();
}

}  // namespace hdg
