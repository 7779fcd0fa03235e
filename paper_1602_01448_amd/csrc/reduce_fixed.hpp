// Fixed-order reductions shared by the kernel files: the sum of the per-block
// residual partials behind eps_a (Eq. (amplitudemetric)) and the loss, and
// eps_a formed by one workgroup of another launch.
#pragma once

#include <hip/hip_runtime.h>

#include "sharp_internal.hpp"

namespace sharp {

// Fixed-order sum of n partials by one workgroup of kRedThreads threads:
// thread t keeps eight running sums over partials t + k kRedThreads (k mod 8
// picks the sum), the eight are added pairwise, then the workgroup's values
// are added in wave order.  The order depends on n only.  (With 1024 threads
// the 32,400 column-block partials of a 2025-frame 256^2 plan take four
// rounds of eight loads; with 256 threads it took sixteen, 16 us against 13.5.)
constexpr int kRedThreads = 1024;
__device__ inline float reduce_fixed(const float* __restrict__ partials, int n, float* red) {
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int i = threadIdx.x;
    for (; i + 7 * kRedThreads < n; i += 8 * kRedThreads) {
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[k] += partials[i + k * kRedThreads];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (i + k * kRedThreads < n) acc[k] += partials[i + k * kRedThreads];
    float s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;   // red: kRedThreads / 64 floats
    __syncthreads();
    float t = 0.f;
    if (threadIdx.x == 0) {
        float q[4];
#pragma unroll
        for (int g = 0; g < 4; ++g) q[g] = (red[4 * g] + red[4 * g + 1]) + (red[4 * g + 2] + red[4 * g + 3]);
        t = (q[0] + q[1]) + (q[2] + q[3]);
    }
    __syncthreads();
    return t;
}

// reduce_fixed's sum by a 256-thread workgroup: thread t plays threads
// t + 256 v (v < 4) of the kRedThreads-thread reduction -- each with its eight
// running sums and its wavefront's shuffle sums (lane t mod 64 of wave
// t / 64 + 4 v) -- then thread 0 adds the sixteen wave sums in that order:
// the same additions, so the same bits.
__device__ inline float reduce_fixed256(const float* __restrict__ partials, int n, float* red) {
    static_assert(kRedThreads == 1024, "four played threads per thread");
    float sv[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        int i = threadIdx.x + 256 * v;
        for (; i + 7 * kRedThreads < n; i += 8 * kRedThreads) {
#pragma unroll
            for (int k = 0; k < 8; ++k) acc[k] += partials[i + k * kRedThreads];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (i + k * kRedThreads < n) acc[k] += partials[i + k * kRedThreads];
        float s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        sv[v] = s;
    }
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int v = 0; v < 4; ++v) red[(threadIdx.x >> 6) + 4 * v] = sv[v];
    }
    __syncthreads();
    float t = 0.f;
    if (threadIdx.x == 0) {
        float q[4];
#pragma unroll
        for (int g = 0; g < 4; ++g) q[g] = (red[4 * g] + red[4 * g + 1]) + (red[4 * g + 2] + red[4 * g + 3]);
        t = (q[0] + q[1]) + (q[2] + q[3]);
    }
    return t;
}

__device__ inline void eps_epilogue(const EpsArgs& E) {
    __shared__ float red[kRedThreads / 64];
    const float s = reduce_fixed256(E.partials, E.n, red);
    if (threadIdx.x == 0) {
        float e = s;   // no norm: the sum itself (the gradient's loss)
        if (E.norm_a2) {
            const float na2 = E.norm_a2[0];
            e = na2 > 0.f ? sqrtf(s / na2) : 0.f;
        }
        E.hist[E.idx] = e;
        if (!isfinite(e)) E.flag[0] = 1;
    }
}

}  // namespace sharp
