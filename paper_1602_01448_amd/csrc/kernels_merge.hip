// Overlap merge Q*z and (Q*Q)^{-1} (Eqs. (Pq), (standardobject)), the
// illumination density D = diag(Q*Q), data preparation a = sqrt(I) (Sec.
// "Forward model") and the fixed-order reductions behind eps_a (Eq.
// (amplitudemetric)) and the loss.
//
// The merge is a tile-owner gather, not a scatter: the object is cut into
// T x T tiles, the plan lists for every tile the frames touching it (in
// ascending frame order), and one workgroup per (tile, frame chunk) sums the
// frame pixels landing in its tile in that order.  With more than one chunk a
// second pass adds the chunk partials in chunk order.  No atomics are used and
// the result does not depend on scheduling.
#include <algorithm>

#include "fft_lds.hpp"
#include "reduce_fixed.hpp"
#include "sharp_internal.hpp"

namespace sharp {

template <int KIND> struct KindTraits {
    static constexpr bool V = (KIND == MK_V || KIND == MK_VU || KIND == MK_RAW);
    static constexpr bool U = (KIND == MK_VU || KIND == MK_U || KIND == MK_RAWW || KIND == MK_OBJ);
    static constexpr bool Dn = (KIND == MK_DENS);
    static constexpr int NV = (KIND == MK_VU) ? 2 : 1;  // complex partials per pixel
};

template <int KIND>
__device__ __forceinline__ void merge_finalize(const MergeArgs& A, size_t idx, float2 acc, float2 accu, float accd) {
    if constexpr (KIND == MK_DENS) {
        A.D_out[idx] = accd;
        A.Dinv_out[idx] = accd > A.eps_D ? 1.0f / accd : 0.f;
    } else {
        const float di = (KIND == MK_RAW || KIND == MK_RAWW) ? 1.f : A.Dinv[idx];
        if constexpr (KIND == MK_V) {
            A.out[idx] = cscale(acc, di);
        } else if constexpr (KIND == MK_VU) {
            const float2 pv = cscale(acc, di);
            A.out[idx] = pv;
            A.out2[idx] = di > 0.f ? cadd(cscale(accu, di), cscale(pv, A.g)) : make_float2(0.f, 0.f);
        } else if constexpr (KIND == MK_U) {
            A.out[idx] = di > 0.f ? cadd(cscale(accu, di), cscale(A.psi_v_in[idx], A.g)) : make_float2(0.f, 0.f);
        } else if constexpr (KIND == MK_RAW) {
            A.out[idx] = acc;
        } else if constexpr (KIND == MK_RAWW) {
            A.out[idx] = accu;
        } else if constexpr (KIND == MK_OBJ) {
            A.out[idx] = cscale(accu, di);
        }
    }
}

// One (tile, frame chunk) of the merge: sums the chunk's frames in ascending
// order into the tile's pixels, then finalises (one chunk) or stores the
// chunk partial.
template <int T, int KIND>
__device__ __forceinline__ void merge_tile(const MergeArgs& A, int tile, int chunk) {
    using KT = KindTraits<KIND>;
    constexpr int PPT = T * T / 256;
    constexpr int RS = 256 / T;
    constexpr int FB = (PPT >= 16) ? 2 : 4;  // frames loaded ahead per step
    const int tx0 = (tile % A.tiles_x) * T, ty0 = (tile / A.tiles_x) * T;
    const int lx = threadIdx.x % T, ly0 = threadIdx.x / T;
    const int X = tx0 + lx;
    const int b = A.tile_ptr[tile], e = A.tile_ptr[tile + 1];
    const int n = e - b;
    const int cb = b + (int)((long long)n * chunk / A.split);
    const int ce = b + (int)((long long)n * (chunk + 1) / A.split);
    const int M = A.M, MM = M * M;

    float2 acc[PPT], accu[PPT];
    float accd[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        acc[k] = accu[k] = make_float2(0.f, 0.f);
        accd[k] = 0.f;
    }
    for (int i = cb; i < ce; i += FB) {
        float2 va[FB][PPT], ua[FB][PPT], wa[FB][PPT];
#pragma unroll
        for (int q = 0; q < FB; ++q) {
            const bool fin = i + q < ce;
            const int f = fin ? A.tile_frames[i + q] : 0;
            const int py = A.pos[2 * f], px = A.pos[2 * f + 1];
            int fx = X - px;
            if (A.periodic && fx < 0) fx += A.nx;
            const bool xin = fin && (unsigned)fx < (unsigned)M && X < A.nx;
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const int Y = ty0 + ly0 + RS * k;
                int fy = Y - py;
                if (A.periodic && fy < 0) fy += A.ny;
                const bool in = xin && (unsigned)fy < (unsigned)M && Y < A.ny;
                const size_t o = (size_t)f * MM + (size_t)fy * M + fx;
                const int wo = fy * M + fx;
                va[q][k] = ua[q][k] = wa[q][k] = make_float2(0.f, 0.f);
                if (in) {
                    if constexpr (KT::V) va[q][k] = A.v[o];
                    if constexpr (KT::U) {
                        ua[q][k] = A.u[o];
                        wa[q][k] = A.w[wo];
                    }
                    if constexpr (KT::Dn) wa[q][k] = A.w[wo];
                }
            }
        }
#pragma unroll
        for (int q = 0; q < FB; ++q)
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                if constexpr (KT::V) acc[k] = cadd(acc[k], va[q][k]);
                if constexpr (KT::U) accu[k] = cadd(accu[k], cconjmul(wa[q][k], ua[q][k]));
                if constexpr (KT::Dn) accd[k] += cabs2(wa[q][k]);
            }
    }
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int Y = ty0 + ly0 + RS * k;
        const int local = (ly0 + RS * k) * T + lx;
        if (A.split == 1) {
            if (X < A.nx && Y < A.ny) merge_finalize<KIND>(A, (size_t)Y * A.nx + X, acc[k], accu[k], accd[k]);
        } else {
            float4* p = A.part + ((size_t)(tile * A.split + chunk) * T * T + local) * KT::NV;
            if constexpr (KT::Dn) p[0] = make_float4(accd[k], 0.f, 0.f, 0.f);
            else if constexpr (KT::NV == 2) {
                p[0] = make_float4(acc[k].x, acc[k].y, 0.f, 0.f);
                p[1] = make_float4(accu[k].x, accu[k].y, 0.f, 0.f);
            } else if constexpr (KT::V) p[0] = make_float4(acc[k].x, acc[k].y, 0.f, 0.f);
            else p[0] = make_float4(accu[k].x, accu[k].y, 0.f, 0.f);
        }
    }
}

// Workgroups are dealt to the XCDs round-robin (b mod 8); xcd_order gives
// each XCD a contiguous run of tiles instead, so that horizontally adjacent
// tiles run on one XCD at about the same time: the 128-byte lines that a
// frame row shares between two tiles are then fetched from HBM once and hit
// that XCD's L2 for the second tile.
__device__ __forceinline__ int xcd_order(int b, int G) { return (G & 7) ? b : (b & 7) * (G >> 3) + (b >> 3); }

// Workgroup (0, 0) also forms eps_a when E.partials is set; it reads only
// the frame launch's partials, which are complete before the merge starts.
template <int T, int KIND>
__global__ void __launch_bounds__(256) merge_kernel(MergeArgs A, EpsArgs E) {
    merge_tile<T, KIND>(A, xcd_order(blockIdx.x, gridDim.x), blockIdx.y);
    if (E.partials && blockIdx.x == 0 && blockIdx.y == 0) eps_epilogue(E);
}

// Second merge pass: chunk partials of one tile added in chunk order.
template <int T, int KIND>
__device__ __forceinline__ void merge_finish_tile(const MergeArgs& A, int tile) {
    using KT = KindTraits<KIND>;
    constexpr int PPT = T * T / 256;
    constexpr int RS = 256 / T;
    const int tx0 = (tile % A.tiles_x) * T, ty0 = (tile / A.tiles_x) * T;
    const int lx = threadIdx.x % T, ly0 = threadIdx.x / T;
    const int X = tx0 + lx;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int Y = ty0 + ly0 + RS * k;
        const int local = (ly0 + RS * k) * T + lx;
        float2 acc = make_float2(0.f, 0.f), accu = acc;
        float accd = 0.f;
        for (int c = 0; c < A.split; ++c) {
            const float4* p = A.part + ((size_t)(tile * A.split + c) * T * T + local) * KT::NV;
            if constexpr (KT::Dn) accd += p[0].x;
            else if constexpr (KT::NV == 2) {
                acc = cadd(acc, make_float2(p[0].x, p[0].y));
                accu = cadd(accu, make_float2(p[1].x, p[1].y));
            } else if constexpr (KT::V) acc = cadd(acc, make_float2(p[0].x, p[0].y));
            else accu = cadd(accu, make_float2(p[0].x, p[0].y));
        }
        if (X < A.nx && Y < A.ny) merge_finalize<KIND>(A, (size_t)Y * A.nx + X, acc, accu, accd);
    }
}

template <int T, int KIND>
__global__ void __launch_bounds__(256) merge_finish_kernel(MergeArgs A) {
    merge_finish_tile<T, KIND>(A, blockIdx.x);
}

template <int T, int KIND>
static hipError_t launch_merge_tk(const MergeArgs& A, int tiles, hipStream_t s, const EpsArgs& E) {
    hipLaunchKernelGGL((merge_kernel<T, KIND>), dim3(tiles, A.split), dim3(256), 0, s, A, E);
    if (A.split > 1) hipLaunchKernelGGL((merge_finish_kernel<T, KIND>), dim3(tiles), dim3(256), 0, s, A);
    return hipGetLastError();
}

template <int T>
static hipError_t launch_merge_t(int kind, const MergeArgs& A, int tiles, hipStream_t s, const EpsArgs& E) {
    switch (kind) {
        case MK_V: return launch_merge_tk<T, MK_V>(A, tiles, s, E);
        case MK_VU: return launch_merge_tk<T, MK_VU>(A, tiles, s, E);
        case MK_U: return launch_merge_tk<T, MK_U>(A, tiles, s, E);
        case MK_RAW: return launch_merge_tk<T, MK_RAW>(A, tiles, s, E);
        case MK_RAWW: return launch_merge_tk<T, MK_RAWW>(A, tiles, s, E);
        case MK_OBJ: return launch_merge_tk<T, MK_OBJ>(A, tiles, s, E);
        case MK_DENS: return launch_merge_tk<T, MK_DENS>(A, tiles, s, E);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_merge(int kind, const MergeArgs& A, int tiles, hipStream_t s, const EpsArgs* eps) {
    const EpsArgs E = eps ? *eps : EpsArgs{};
    switch (A.T) {
        case 16: return launch_merge_t<16>(kind, A, tiles, s, E);
        case 32: return launch_merge_t<32>(kind, A, tiles, s, E);
        case 64: return launch_merge_t<64>(kind, A, tiles, s, E);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// data preparation and fixed-order reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ float block_sum256(float x, float* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    float s = 0.f;
    if (threadIdx.x == 0) s = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return s;
}

__global__ void __launch_bounds__(256) set_data_kernel(const float* __restrict__ I, float* __restrict__ a, size_t n,
                                                       float* __restrict__ partials, int* __restrict__ flag,
                                                       int blocked256, float* __restrict__ a2, int a2_q256) {
    __shared__ float red[4];
    float s = 0.f;
    bool bad = false;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const float v = I[i];
        bad |= !isfinite(v);
        const float r = sqrtf(fmaxf(v, 0.f));
        size_t o = i;
        if (blocked256) {
            const unsigned p = (unsigned)(i & 65535u);
            o = (i - p) + cb256(p >> 8, p & 255u);
        }
        a[o] = r;
        if (a2) {
            if (a2_q256) {  // second copy of a 256 x 256 frame in the q256 layout
                const unsigned p = (unsigned)(i & 65535u);
                a2[(i - p) + q256(p >> 8, p & 255u)] = r;
            } else {        // second copy, each 128 x 128 frame transposed
                const unsigned p = (unsigned)(i & 16383u);
                a2[(i - p) + (p & 127u) * 128u + (p >> 7)] = r;
            }
        }
        s += r * r;
    }
    if (bad) flag[0] = 1;
    s = block_sum256(s, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kRedThreads) reduce_kernel(const float* __restrict__ partials, int n, float* out) {
    __shared__ float red[kRedThreads / 64];
    const float s = reduce_fixed(partials, n, red);
    if (threadIdx.x == 0) out[0] = s;
}

__global__ void __launch_bounds__(kRedThreads) loss_kernel(const float* __restrict__ partials, int n, float* out,
                                                           int* flag) {
    __shared__ float red[kRedThreads / 64];
    const float s = reduce_fixed(partials, n, red);
    if (threadIdx.x == 0) {
        out[0] = s;
        if (!isfinite(s)) flag[0] = 1;
    }
}

__global__ void __launch_bounds__(256) mean_amp_kernel(const float* __restrict__ a, int K, int MM,
                                                       float2* __restrict__ out) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= MM) return;
    const unsigned ap = (MM == 65536) ? cb256(p >> 8, p & 255) : (unsigned)p;  // m = 256: column-block layout
    float s = 0.f;
    for (int f = 0; f < K; ++f) {
        const float v = a[(size_t)f * MM + ap];
        s += v * v;
    }
    out[p] = make_float2(sqrtf(s / K), 0.f);
}

__global__ void __launch_bounds__(256) roll_probe_kernel(const float2* __restrict__ src, int M,
                                                         float2* __restrict__ w_cur, float2* __restrict__ w_gat) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= M * M) return;
    const int y = p / M, x = p % M, h = M / 2;
    const int d = ((y + h) % M) * M + (x + h) % M;
    w_cur[d] = src[p];
    w_gat[d] = src[p];
}

__global__ void __launch_bounds__(256) fill_kernel(uint4* __restrict__ p, size_t n16, unsigned char* tail,
                                                   size_t ntail) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += (size_t)gridDim.x * 256)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
    if (blockIdx.x == 0 && threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

hipError_t launch_set_data(const float* I, float* a, size_t n, float* partials, int* flag, hipStream_t s,
                           int* blocks_used, int blocked256, float* a2, int a2_q256) {
    const int grid = (int)std::min<size_t>(std::max<size_t>((n + 255) / 256, 1), 2048);
    hipLaunchKernelGGL(set_data_kernel, dim3(grid), dim3(256), 0, s, I, a, n, partials, flag, blocked256, a2,
                       a2_q256);
    *blocks_used = grid;
    return hipGetLastError();
}

hipError_t launch_reduce(const float* partials, int n, float* out, hipStream_t s) {
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kRedThreads), 0, s, partials, n, out);
    return hipGetLastError();
}

hipError_t launch_loss(const float* partials, int n, float* out, int* flag, hipStream_t s) {
    hipLaunchKernelGGL(loss_kernel, dim3(1), dim3(kRedThreads), 0, s, partials, n, out, flag);
    return hipGetLastError();
}

hipError_t launch_mean_amp(const float* a, int K, int M, float2* out, hipStream_t s) {
    hipLaunchKernelGGL(mean_amp_kernel, dim3((M * M + 255) / 256), dim3(256), 0, s, a, K, M * M, out);
    return hipGetLastError();
}

hipError_t launch_roll_probe(const float2* src, int M, float2* w_cur, float2* w_gat, hipStream_t s) {
    hipLaunchKernelGGL(roll_probe_kernel, dim3((M * M + 255) / 256), dim3(256), 0, s, src, M, w_cur, w_gat);
    return hipGetLastError();
}

hipError_t launch_fill(void* p, size_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    const size_t n16 = bytes / 16, ntail = bytes % 16;
    const int grid = (int)std::min<size_t>(std::max<size_t>((n16 + 255) / 256, 1), 4096);
    hipLaunchKernelGGL(fill_kernel, dim3(grid), dim3(256), 0, s, (uint4*)p, n16,
                       (unsigned char*)p + n16 * 16, ntail);
    return hipGetLastError();
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s);
}

// ---------------------------------------------------------------------------
// Batched merge and residual reduction over a table of scans
// ---------------------------------------------------------------------------
template <int T>
__global__ void __launch_bounds__(256) batch_merge_kernel(const BatchMergeArgs CH, const int4* __restrict__ items,
                                                          int n) {
    // one item per workgroup, dealt round-robin: item costs differ between
    // scans (frames per tile grow with (m / step)^2), and contiguous runs per
    // XCD (as in merge_kernel) measured slower here
    const int it = blockIdx.x;
    if (it >= n) return;
    const int4 w = items[it];
    merge_tile<T, MK_V>(CH.a[w.x - CH.base], w.y, w.z);
}

template <int T>
__global__ void __launch_bounds__(256) batch_merge_finish_kernel(const BatchMergeArgs CH,
                                                                 const int2* __restrict__ items, int n) {
    const int it = blockIdx.x;
    if (it >= n) return;
    const int2 w = items[it];
    merge_finish_tile<T, MK_V>(CH.a[w.x - CH.base], w.y);
}

hipError_t launch_batch_merge(int T, const BatchMergeArgs& C, const int4* items, int n, const int2* fin, int nfin,
                              hipStream_t s) {
    if (n > 0) {
        switch (T) {
            case 16: hipLaunchKernelGGL(batch_merge_kernel<16>, dim3(n), dim3(256), 0, s, C, items, n); break;
            case 32: hipLaunchKernelGGL(batch_merge_kernel<32>, dim3(n), dim3(256), 0, s, C, items, n); break;
            case 64: hipLaunchKernelGGL(batch_merge_kernel<64>, dim3(n), dim3(256), 0, s, C, items, n); break;
            default: return hipErrorInvalidValue;
        }
    }
    if (nfin > 0) {
        switch (T) {
            case 16: hipLaunchKernelGGL(batch_merge_finish_kernel<16>, dim3(nfin), dim3(256), 0, s, C, fin, nfin); break;
            case 32: hipLaunchKernelGGL(batch_merge_finish_kernel<32>, dim3(nfin), dim3(256), 0, s, C, fin, nfin); break;
            case 64: hipLaunchKernelGGL(batch_merge_finish_kernel<64>, dim3(nfin), dim3(256), 0, s, C, fin, nfin); break;
            default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

// One block per scan: eps_a of the iteration into the scan's history ring,
// then the gather coefficient of the scan's next iteration becomes beta.
__global__ void __launch_bounds__(kRedThreads) batch_eps_kernel(EpsDesc* __restrict__ E, FrameArgs* __restrict__ D,
                                                                float beta) {
    __shared__ float red[kRedThreads / 64];
    EpsDesc& e = E[blockIdx.x];
    const float s = reduce_fixed(e.partials, e.n, red);
    if (threadIdx.x == 0) {
        const float na2 = e.norm_a2[0];
        const float v = na2 > 0.f ? sqrtf(s / na2) : 0.f;
        const int idx = e.hist_idx;
        e.hist[idx % kHistCap] = v;
        e.hist_idx = (idx + 1) % kHistCap;
        if (!isfinite(v)) e.flag[0] = 1;
        D[blockIdx.x].g = beta;
    }
}

__global__ void __launch_bounds__(256) batch_begin_kernel(FrameArgs* __restrict__ D, EpsDesc* __restrict__ E,
                                                          BatchBegin b, float beta) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= b.n) return;
    D[s].g = b.g[s];
    D[s].beta = beta;
    D[s].gather = b.gather[s];
    E[s].hist_idx = b.hist[s];
}

hipError_t launch_batch_eps(EpsDesc* E, FrameArgs* D, int nscans, float beta, hipStream_t s) {
    hipLaunchKernelGGL(batch_eps_kernel, dim3(nscans), dim3(kRedThreads), 0, s, E, D, beta);
    return hipGetLastError();
}

hipError_t launch_batch_begin(FrameArgs* D, EpsDesc* E, const BatchBegin& b, float beta, hipStream_t s) {
    hipLaunchKernelGGL(batch_begin_kernel, dim3((b.n + 255) / 256), dim3(256), 0, s, D, E, b, beta);
    return hipGetLastError();
}

// Device read-rate reference: 16-byte nontemporal loads, eight requests in
// flight per thread, kReadRefBlocks workgroups striding over the buffer.  The
// sums only keep the loads alive; thread 0 of each workgroup stores its own.
__global__ void __launch_bounds__(256) read_reference_kernel(const float4* __restrict__ p, size_t n,
                                                             float* __restrict__ sink) {
    typedef float sf4 __attribute__((ext_vector_type(4)));
    constexpr int U = 8;
    float acc = 0.f;
    const size_t stride = (size_t)gridDim.x * 256 * U;
    for (size_t i = (size_t)blockIdx.x * 256 * U + threadIdx.x; i < n; i += stride) {
        sf4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const size_t j = i + (size_t)u * 256;
            v[u] = j < n ? __builtin_nontemporal_load(reinterpret_cast<const sf4*>(p + j)) : sf4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int u = 0; u < U; ++u) acc += (v[u].x + v[u].y) + (v[u].z + v[u].w);
    }
    if (threadIdx.x == 0) sink[blockIdx.x] = acc;
}

hipError_t launch_read_reference(const void* src, size_t bytes, float* sink, hipStream_t s) {
    hipLaunchKernelGGL(read_reference_kernel, dim3(kReadRefBlocks), dim3(256), 0, s,
                       reinterpret_cast<const float4*>(src), bytes / 16, sink);
    return hipGetLastError();
}

}  // namespace sharp
