// Batched 2-D FFT building blocks for gfx950: radix-2/4/8/16 butterflies in
// registers and Stockham autosort stages whose operands live in LDS.
//
// The transform is the paper's F (Sec. "Forward model"): unitary, with the
// e^{+2 pi i q.r} sign for DIR = +1 and e^{-2 pi i q.r} for DIR = -1 (F*).
// Scaling by 1/m is applied by the caller once per 2-D transform.
//
// Stockham stage (radix R, span L, line length N): butterfly j of a line reads
// x[j + r N/R] (r < R), multiplies by e^{DIR 2 pi i (j mod L) r / (L R)},
// takes an R-point DFT, and writes element q to ((j / L) L R + j mod L + q L).
// Running the stages with L = 1, R1, R1 R2, ... yields natural-order output.
#pragma once
#include <hip/hip_runtime.h>

namespace sharp {

// ---------------------------------------------------------------------------
// complex helpers (float2 = re, im)
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// conj(a) * b
__device__ __forceinline__ float2 cconjmul(float2 a, float2 b) {
    return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float cabs2(float2 a) { return a.x * a.x + a.y * a.y; }

// clang vector types for the nontemporal load/store builtins
typedef float sf4 __attribute__((ext_vector_type(4)));
typedef float sf2 __attribute__((ext_vector_type(2)));

// multiply by DIR * i
template <int DIR>
__device__ __forceinline__ float2 mul_i(float2 a) {
    return DIR > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// e^{DIR 2 pi i k / 16} for compile-time k after unrolling.
// cos(pi/8), sin(pi/8) and cos(pi/4) are the exact-rounded float values.
template <int DIR>
__device__ __forceinline__ float2 w16(int k) {
    constexpr float c1 = 0.92387953251128674f, s1 = 0.38268343236508977f, h = 0.70710678118654752f;
    const float C[16] = {1.f, c1, h, s1, 0.f, -s1, -h, -c1, -1.f, -c1, -h, -s1, 0.f, s1, h, c1};
    const float S[16] = {0.f, s1, h, c1, 1.f, c1, h, s1, 0.f, -s1, -h, -c1, -1.f, -c1, -h, -s1};
    return make_float2(C[k & 15], DIR * S[k & 15]);
}

// ---------------------------------------------------------------------------
// R-point DFTs in registers, A[q] = sum_r a[r] e^{DIR 2 pi i r q / R}, in place
// ---------------------------------------------------------------------------
template <int DIR>
__device__ __forceinline__ void dft2(float2* a) {
    float2 t = a[0];
    a[0] = cadd(t, a[1]);
    a[1] = csub(t, a[1]);
}

template <int DIR>
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
    float2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
    float2 t2 = cadd(a1, a3), t3 = mul_i<DIR>(csub(a1, a3));
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    a1 = cadd(t1, t3);
    a3 = csub(t1, t3);
}

template <int DIR>
__device__ __forceinline__ void dft4(float2* a) { dft4<DIR>(a[0], a[1], a[2], a[3]); }

// 8 = 2 x 4: n = 4 n1 + n2, k = k1 + 2 k2
template <int DIR>
__device__ __forceinline__ void dft8(float2* a) {
    float2 b[4][2];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
        b[n2][0] = cadd(a[n2], a[4 + n2]);
        b[n2][1] = csub(a[n2], a[4 + n2]);
    }
#pragma unroll
    for (int n2 = 1; n2 < 4; ++n2) b[n2][1] = cmul(b[n2][1], w16<DIR>(2 * n2));
#pragma unroll
    for (int k1 = 0; k1 < 2; ++k1) {
        dft4<DIR>(b[0][k1], b[1][k1], b[2][k1], b[3][k1]);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) a[k1 + 2 * k2] = b[k2][k1];
    }
}

// 16 = 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2
template <int DIR>
__device__ __forceinline__ void dft16(float2* a) {
    float2 b[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
        b[n2][0] = a[n2];
        b[n2][1] = a[4 + n2];
        b[n2][2] = a[8 + n2];
        b[n2][3] = a[12 + n2];
        dft4<DIR>(b[n2]);
    }
#pragma unroll
    for (int n2 = 1; n2 < 4; ++n2)
#pragma unroll
        for (int k1 = 1; k1 < 4; ++k1) b[n2][k1] = cmul(b[n2][k1], w16<DIR>(n2 * k1));
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        dft4<DIR>(b[0][k1], b[1][k1], b[2][k1], b[3][k1]);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) a[k1 + 4 * k2] = b[k2][k1];
    }
}

template <int R, int DIR>
__device__ __forceinline__ void dft(float2* a) {
    if constexpr (R == 2) dft2<DIR>(a);
    else if constexpr (R == 4) dft4<DIR>(a);
    else if constexpr (R == 8) dft8<DIR>(a);
    else dft16<DIR>(a);
}

// ---------------------------------------------------------------------------
// radix plans per line length
// ---------------------------------------------------------------------------
template <int N> struct Radix;
template <> struct Radix<16>  { static constexpr int S = 1, R0 = 16, R1 = 1; };
template <> struct Radix<32>  { static constexpr int S = 2, R0 = 8,  R1 = 4; };
template <> struct Radix<64>  { static constexpr int S = 2, R0 = 8,  R1 = 8; };
template <> struct Radix<128> { static constexpr int S = 2, R0 = 16, R1 = 8; };
template <> struct Radix<256> { static constexpr int S = 2, R0 = 16, R1 = 16; };

// LDS addressing: one float2 of padding after every 16 elements spreads
// power-of-two strides over the banks.
__host__ __device__ constexpr int pidx(int e) { return e + (e >> 4); }

struct NoPost {
    __device__ __forceinline__ void operator()(int, int, float2&) const {}
};

// One Stockham stage over LDS.  Lay maps a butterfly id b to its line start
// (Lay::base), its index j within the line (Lay::j) and gives the element
// stride of a line (Lay::stride).  NB butterflies are spread over NT threads,
// b = threadIdx.x + p NT.  Post(b, e, v) sees every output element e of the
// line before it is stored.
template <int N, int R, int L, int DIR, int NT, int NB, class Lay, class Post>
__device__ __forceinline__ void fft_stage(float2* __restrict__ lds, const float2* __restrict__ twl,
                                          Post& post) {
    constexpr int BPL = N / R;
    static_assert(NB % NT == 0, "butterflies must divide evenly over threads");
    constexpr int PER = NB / NT;
    // An opaque copy of the thread index: keeps the compiler from hoisting
    // every stage's address arithmetic out of the caller's loops (which
    // would hold hundreds of addresses live in registers).
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    tid &= 1023;  // non-negative: index divisions by powers of two stay shifts
    float2 v[PER][R];
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int b = tid + p * NT;
        const int base = Lay::base(b), j = Lay::j(b);
#pragma unroll
        for (int r = 0; r < R; ++r) v[p][r] = lds[pidx(base + (j + r * BPL) * Lay::stride)];
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int b = tid + p * NT;
        const int base = Lay::base(b), j = Lay::j(b);
        const int k = j % L;
        if constexpr (L > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                float2 t = twl[k * r * (N / (L * R))];
                if constexpr (DIR < 0) t.y = -t.y;
                v[p][r] = cmul(v[p][r], t);
            }
        }
        dft<R, DIR>(v[p]);
        const int ob = (j / L) * L * R + k;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int e = ob + q * L;
            post(b, e, v[p][q]);
            lds[pidx(base + e * Lay::stride)] = v[p][q];
        }
    }
    __syncthreads();
}

// A full 1-D transform of length N along the lines described by Lay.  The
// post-op runs on the outputs of the last stage only.
template <int N, int DIR, int NT, int NLINES, class Lay, class Post>
__device__ __forceinline__ void fft_lines(float2* lds, const float2* twl, Post& post) {
    using P = Radix<N>;
    NoPost none;
    if constexpr (P::S == 1) {
        fft_stage<N, P::R0, 1, DIR, NT, NLINES * (N / P::R0), Lay>(lds, twl, post);
    } else {
        fft_stage<N, P::R0, 1, DIR, NT, NLINES * (N / P::R0), Lay>(lds, twl, none);
        fft_stage<N, P::R1, P::R0, DIR, NT, NLINES * (N / P::R1), Lay>(lds, twl, post);
    }
}

}  // namespace sharp
