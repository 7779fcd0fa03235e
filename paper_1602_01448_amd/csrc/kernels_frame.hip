// Frame kernels: gather (Q), 2-D FFT (F), Fourier-modulus projection (P_a),
// inverse FFT (F*) and the RAAR / gradient epilogues, fused per frame.
//
// Paper references: frames z_i = w T_i psi (Sec. "Forward model", Eq.
// (overlap)); F (Sec. "Forward model"); P_a z = F*(Fz/|Fz|) a (Eq. (Pa));
// RAAR update (algorithm box, step 5, relaxed-averaged-alternating-
// reflections sign); eps_a (Eq. (amplitudemetric)); probe update (Eq.
// (standardprobe)).
//
// Two execution shapes:
//  * m <= 128: one workgroup owns a group of G whole frames in LDS (G m^2 =
//    16 NT) and runs gather -> F -> modulus -> F* -> epilogue without leaving
//    the CU.  HBM traffic per frame pixel: carry in 8 B, a 4 B, carry out 8 B,
//    merge input out 8 B.
//  * m = 256: a frame (512 KiB) exceeds LDS, so the transform is split into
//    a row pass (gather + row FFTs), a column pass (column FFTs + modulus +
//    inverse column FFTs) and a row pass (inverse row FFTs + epilogue), with
//    the row-transformed frames kept in an HBM stage buffer between passes.
#include <algorithm>

#include "fft_lds.hpp"
#include "reduce_fixed.hpp"
#include "sharp_internal.hpp"

namespace sharp {

// ---------------------------------------------------------------------------
// LDS layouts for fft_stage
// ---------------------------------------------------------------------------
template <int M>
struct RowLay {  // consecutive lines of length M (rows of the frames held)
    static constexpr int stride = 1;
    template <int BPL> __device__ static int base(int b) { return (b / BPL) * M; }
    template <int BPL> __device__ static int j(int b) { return b % BPL; }
};

template <int M>
struct ColLayFG {  // columns of G whole frames stored [f][y][x]; x fastest over lanes
    static constexpr int stride = M;
    template <int BPL> __device__ static int base(int b) { return ((b / M) / BPL) * M * M + b % M; }
    template <int BPL> __device__ static int j(int b) { return (b / M) % BPL; }
};

template <int CB>
struct ColLayCB {  // CB columns of one frame stored [y][c]
    static constexpr int stride = CB;
    template <int BPL> __device__ static int base(int b) { return b % CB; }
    template <int BPL> __device__ static int j(int b) { return b / CB; }
};

// fft_stage needs Lay::base/j as plain templates; adapt the member templates.
template <class Lay, int BPL> struct LayAt {
    static constexpr int stride = Lay::stride;
    __device__ static int base(int b) { return Lay::template base<BPL>(b); }
    __device__ static int j(int b) { return Lay::template j<BPL>(b); }
};

template <int N, int DIR, int NT, int NLINES, class Lay, class Post>
__device__ __forceinline__ void fft_1d(float2* lds, const float2* twl, Post& post) {
    using P = Radix<N>;
    NoPost none;
    if constexpr (P::S == 1) {
        fft_stage<N, P::R0, 1, DIR, NT, NLINES * (N / P::R0), LayAt<Lay, N / P::R0>>(lds, twl, post);
    } else {
        fft_stage<N, P::R0, 1, DIR, NT, NLINES * (N / P::R0), LayAt<Lay, N / P::R0>>(lds, twl, none);
        fft_stage<N, P::R1, P::R0, DIR, NT, NLINES * (N / P::R1), LayAt<Lay, N / P::R1>>(lds, twl, post);
    }
}

// ---------------------------------------------------------------------------
// shared pieces
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wrap(int v, int n) { return v >= n ? v - n : v; }

// Thread index the compiler cannot treat as loop-invariant: per-item address
// arithmetic stays inside the item instead of being hoisted (and held live)
// across the item loop.
// The mask (blocks have at most 1024 threads) tells the compiler that the
// value is non-negative, so index divisions by powers of two stay shifts.
__device__ __forceinline__ int opaque_tid() {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t & 1023;
}

// The threads of a transform line lie in one wavefront, whose LDS accesses
// are performed in program order: exchanges inside a line only need the
// compiler to keep that order.
__device__ __forceinline__ void line_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Memory access through a uniform base pointer plus a 32-bit element offset
// (the compiler then addresses with a scalar base and one vector offset).
__device__ __forceinline__ const char* byte_at(const void* p, unsigned elem, unsigned size) {
    return reinterpret_cast<const char*>(p) + elem * size;
}
__device__ __forceinline__ void ld2(const float2* __restrict__ p, unsigned i, float2& a, float2& b) {
    const float4 t = *reinterpret_cast<const float4*>(byte_at(p, i, 8u));
    a = make_float2(t.x, t.y);
    b = make_float2(t.z, t.w);
}
__device__ __forceinline__ void st2(float2* __restrict__ p, unsigned i, float2 a, float2 b) {
    *reinterpret_cast<float4*>(const_cast<char*>(byte_at(p, i, 8u))) = make_float4(a.x, a.y, b.x, b.y);
}
__device__ __forceinline__ float2 ldf2(const float* __restrict__ p, unsigned i) {
    return *reinterpret_cast<const float2*>(byte_at(p, i, 4u));
}
__device__ __forceinline__ void stf2(float* __restrict__ p, unsigned i, float a, float b) {
    *reinterpret_cast<float2*>(const_cast<char*>(byte_at(p, i, 4u))) = make_float2(a, b);
}
// Streaming forms (nontemporal hint) for arrays that a pass reads or writes
// once (the carry, the amplitudes, the stage buffer, the merge input of the
// large frames): when these arrays are larger than the last-level cache, the
// carry passes move measurably more bytes per second with them.
__device__ __forceinline__ void ld2s(const float2* __restrict__ p, unsigned i, float2& a, float2& b) {
    const sf4 t = __builtin_nontemporal_load(reinterpret_cast<const sf4*>(byte_at(p, i, 8u)));
    a = make_float2(t.x, t.y);
    b = make_float2(t.z, t.w);
}
__device__ __forceinline__ void st2s(float2* __restrict__ p, unsigned i, float2 a, float2 b) {
    const sf4 t = {a.x, a.y, b.x, b.y};
    __builtin_nontemporal_store(t, reinterpret_cast<sf4*>(const_cast<char*>(byte_at(p, i, 8u))));
}
__device__ __forceinline__ float2 ldf2s(const float* __restrict__ p, unsigned i) {
    const sf2 t = __builtin_nontemporal_load(reinterpret_cast<const sf2*>(byte_at(p, i, 4u)));
    return make_float2(t.x, t.y);
}
// NT selects the streaming form (a plan streams when its frame arrays exceed
// the last-level cache; below that, the cached form keeps them resident).
template <bool NT>
__device__ __forceinline__ void ld2t(const float2* __restrict__ p, unsigned i, float2& a, float2& b) {
    if constexpr (NT) ld2s(p, i, a, b);
    else ld2(p, i, a, b);
}
template <bool NT>
__device__ __forceinline__ void st2t(float2* __restrict__ p, unsigned i, float2 a, float2 b) {
    if constexpr (NT) st2s(p, i, a, b);
    else st2(p, i, a, b);
}
template <bool NT>
__device__ __forceinline__ float2 ldf2t(const float* __restrict__ p, unsigned i) {
    if constexpr (NT) return ldf2s(p, i);
    else return ldf2(p, i);
}
__device__ __forceinline__ float2 ldc(const float2* __restrict__ p, unsigned i) {
    return *reinterpret_cast<const float2*>(byte_at(p, i, 8u));
}

// g * w * psi for the gather of the m = 128 kernel, evaluated without
// contraction.
__device__ __forceinline__ float2 gather_z(float2 w, float2 p, float g) {
#pragma clang fp contract(off)
    return make_float2((w.x * p.x - w.y * p.y) * g, (w.x * p.y + w.y * p.x) * g);
}
__device__ __forceinline__ void stc(float2* __restrict__ p, unsigned i, float2 v) {
    *reinterpret_cast<float2*>(const_cast<char*>(byte_at(p, i, 8u))) = v;
}

// Gather of two horizontally adjacent object pixels for frame pixel (y, x), (y, x+1).
__device__ __forceinline__ void gather2(const FrameArgs& A, int frame, int y, int x, float2& p0, float2& p1) {
    const int py = A.pos[2 * frame], px = A.pos[2 * frame + 1];
    int gy = py + y, gx = px + x, gx1 = gx + 1;
    if (A.periodic) {
        gy = wrap(gy, A.ny);
        gx = wrap(gx, A.nx);
        gx1 = wrap(gx1, A.nx);
    }
    const unsigned row = (unsigned)gy * (unsigned)A.nx;
    p0 = ldc(A.psi, row + gx);
    p1 = ldc(A.psi, row + gx1);
}

// Prologue: the frame values z entering the transform (and T psi for GRAD).
// fb: element offset of a frame (group) base, uniform across the block;
// off: element offset from there; pix: pixel index inside the frame.
template <int MODE>
__device__ __forceinline__ void prologue2(const FrameArgs& A, int frame, int y, int x, size_t fb, unsigned off,
                                          unsigned pix, float2& z0, float2& z1, float2& t0, float2& t1) {
    if constexpr (MODE == FM_RAAR) {
        float2 p0, p1, w0, w1;
        ld2(A.u + fb, off, z0, z1);
        gather2(A, frame, y, x, p0, p1);
        ld2(A.w_g, pix, w0, w1);
        z0 = cadd(z0, cscale(cmul(w0, p0), A.g));
        z1 = cadd(z1, cscale(cmul(w1, p1), A.g));
    } else if constexpr (MODE == FM_PA || MODE == FM_F || MODE == FM_FINV) {
        ld2(A.in + fb, off, z0, z1);
    } else if constexpr (MODE == FM_GATHER) {
        float2 p0, p1, w0, w1;
        gather2(A, frame, y, x, p0, p1);
        ld2(A.w_g, pix, w0, w1);
        z0 = cmul(w0, p0);   // g is applied by the column pass
        z1 = cmul(w1, p1);
    } else {  // GRAD, SIM, Q
        float2 w0, w1;
        gather2(A, frame, y, x, t0, t1);
        ld2(A.w, pix, w0, w1);
        z0 = cmul(w0, t0);
        z1 = cmul(w1, t1);
    }
}

// Fourier-domain operation applied to the last forward stage's outputs.
// `addr_to_g` maps the LDS element address to (frame, global index).
template <int MODE, int M>
struct ModOp {
    const float* __restrict__ a;      // frame (group) base of the amplitudes
    float* __restrict__ out_f;        // frame (group) base of the intensity output
    float resid = 0.f;
    // v is the unscaled transform value at element offset i from the bases
    __device__ __forceinline__ void apply(bool ok, unsigned i, float2& v) {
        v = cscale(v, 1.0f / M);  // unitary scaling of F
        if constexpr (MODE == FM_RAAR || MODE == FM_PA || MODE == FM_GRAD) {
            const float av = ok ? a[i] : 0.f;
            v = modulus(v, av, ok);
        } else if constexpr (MODE == FM_SIM) {
            if (ok) out_f[i] = cabs2(v);
        }
    }
    // P_a on one value: a sgn(v), sgn(0) := 1; GRAD keeps v - a sgn(v).
    // One reciprocal square root gives both v / |v| and |v| (to an ulp or so).
    __device__ __forceinline__ float2 modulus(float2 v, float av, bool ok) {
        const float n2 = cabs2(v);
        float2 s = make_float2(1.f, 0.f);
        float mag = 0.f;
        if (n2 > 0.f) {
            const float r = rsqrtf(n2);
            s = cscale(v, r);
            mag = n2 * r;
        }
        const float d = mag - av;
        if (ok) resid += d * d;
        const float2 p = cscale(s, av);
        return (MODE == FM_GRAD) ? csub(v, p) : p;
    }
    // The same with selects instead of a branch on |v| > 0 (identical results;
    // fewer instructions where the branch would be taken per element, more
    // registers live, so only the kernels with registers to spare use it).
    __device__ __forceinline__ float2 modulus_sel(float2 v, float av) {
        const float n2 = cabs2(v);
        const bool nz = n2 > 0.f;
        const float r = rsqrtf(nz ? n2 : 1.f);
        const float2 s = nz ? cscale(v, r) : make_float2(1.f, 0.f);
        const float mag = nz ? n2 * r : 0.f;
        const float d = mag - av;
        resid += d * d;
        const float2 p = cscale(s, av);
        return (MODE == FM_GRAD) ? csub(v, p) : p;
    }
};

__device__ __forceinline__ float block_sum(float x, float* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = x;
    __syncthreads();
    float s = 0.f;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int i = 0; i < nw; ++i) s += red[i];
    }
    __syncthreads();
    return s;
}

// ---------------------------------------------------------------------------
// m <= 128: whole frames in LDS
// ---------------------------------------------------------------------------
// A workgroup of NT threads holds G frames, E elements per thread.  32^2 and
// 64^2 frames take one frame per workgroup of 128 and 512 threads (eight
// elements per thread): half the dependent work per thread of sixteen-element
// groups, and more workgroups (at 169 frames of 32^2, 169 instead of 43).  The
// 64^2 transforms are radix 8 x 8 (512 butterflies per stage and frame).
template <int M>
struct FG {
    static constexpr int NT = (M == 128) ? 1024 : (M == 32) ? 128 : (M == 64) ? 512 : 256;
    static constexpr int E = (M == 32 || M == 64) ? 8 : 16;
    static constexpr int G = NT * E / (M * M);
    static constexpr int FE = G * M * M;
    static constexpr int NP = E / 2;
    static constexpr int LDS = pidx(FE);
    static constexpr size_t SMEM = (size_t)(LDS + M) * sizeof(float2);
};

// fft_stage calls post(b, e, v); wrap to give the LDS element address instead.
template <class Lay, class P>
struct AddrPost {
    P* p;
    __device__ __forceinline__ void operator()(int b, int e, float2& v) const {
        (*p)(Lay::base(b) + e * Lay::stride, v);
    }
};

template <int N, int DIR, int NT, int NLINES, class Lay, class P>
__device__ __forceinline__ void fft_1d_post(float2* lds, const float2* twl, P& post) {
    using PR = Radix<N>;
    NoPost none;
    if constexpr (PR::S == 1) {
        using L0 = LayAt<Lay, N / PR::R0>;
        AddrPost<L0, P> ap{&post};
        fft_stage<N, PR::R0, 1, DIR, NT, NLINES * (N / PR::R0), L0>(lds, twl, ap);
    } else {
        using L0 = LayAt<Lay, N / PR::R0>;
        using L1 = LayAt<Lay, N / PR::R1>;
        AddrPost<L1, P> ap{&post};
        fft_stage<N, PR::R0, 1, DIR, NT, NLINES * (N / PR::R0), L0>(lds, twl, none);
        fft_stage<N, PR::R1, PR::R0, DIR, NT, NLINES * (N / PR::R1), L1>(lds, twl, ap);
    }
}

// One group of G frames: prologue -> F -> Fourier op -> F* -> epilogue.
// Every thread owns the element pairs e0 = 2 (tid + NT k) of the group for
// the prologue, the Fourier-domain operation and the epilogue, so all global
// accesses are coalesced and share one 32-bit offset per pair.  Ends with a
// barrier, so the caller may reuse the LDS right away.
template <int M, int MODE>
__device__ __forceinline__ void fg_group(const FrameArgs& A, int grp, float2* lds, const float2* twl, float& resid,
                                         float2* gacc) {
    const int tid = opaque_tid();
    using C = FG<M>;
    constexpr int NT = C::NT, G = C::G, NP = C::NP, MM = M * M;
    const int f0 = grp * G;
    const size_t fb = (size_t)f0 * MM;  // element offset of the group in frame stacks
    float2 z[2 * NP], t[2 * NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int e0 = 2 * (tid + NT * k);
        // with m^2 >= 2 NT the frame of pair k is (2 NT k) / m^2 for every
        // thread (2 tid < 2 NT <= m^2): uniform, so its position is loaded once
        // through the scalar cache instead of per thread
        const int f = (MM >= 2 * NT) ? (2 * NT * k) / MM : e0 / MM;
        const int rem = e0 - f * MM, y = rem / M, x = rem % M;
        const int frame = f0 + f;
        z[2 * k] = z[2 * k + 1] = t[2 * k] = t[2 * k + 1] = make_float2(0.f, 0.f);
        if (frame < A.K)
            prologue2<MODE>(A, frame, y, x, fb, e0, rem, z[2 * k], z[2 * k + 1], t[2 * k], t[2 * k + 1]);
        lds[pidx(e0)] = z[2 * k];
        lds[pidx(e0 + 1)] = z[2 * k + 1];
    }
    __syncthreads();

    constexpr int D1 = (MODE == FM_FINV) ? -1 : 1;
    NoPost none;
    fft_1d<M, D1, NT, G * M, RowLay<M>>(lds, twl, none);
    fft_1d<M, D1, NT, G * M, ColLayFG<M>>(lds, twl, none);

    // Fourier-domain operation on the same element pairs
    ModOp<MODE, M> op{A.a + fb, A.out_f + fb, 0.f};
    const float inv_m = 1.0f / M;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int e0 = 2 * (tid + NT * k);
        const bool ok = f0 + e0 / MM < A.K;
        float2 v0 = cscale(lds[pidx(e0)], inv_m), v1 = cscale(lds[pidx(e0 + 1)], inv_m);
        if constexpr (MODE == FM_RAAR || MODE == FM_PA || MODE == FM_GRAD) {
            const float2 av = ok ? ldf2(A.a + fb, e0) : make_float2(0.f, 0.f);
            lds[pidx(e0)] = op.modulus(v0, av.x, ok);
            lds[pidx(e0 + 1)] = op.modulus(v1, av.y, ok);
        } else if constexpr (MODE == FM_SIM) {
            if (ok) stf2(A.out_f + fb, e0, cabs2(v0), cabs2(v1));
        } else if constexpr (MODE == FM_F || MODE == FM_FINV) {
            if (ok) st2(A.out + fb, e0, v0, v1);
        }
    }
    resid += op.resid;
    __syncthreads();
    if constexpr (MODE == FM_SIM || MODE == FM_F || MODE == FM_FINV) return;

    fft_1d<M, -1, NT, G * M, RowLay<M>>(lds, twl, none);
    fft_1d<M, -1, NT, G * M, ColLayFG<M>>(lds, twl, none);
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int e0 = 2 * (tid + NT * k);
        const int f = e0 / MM, rem = e0 % MM, frame = f0 + f;
        if (frame >= A.K) continue;
        const float2 y0 = cscale(lds[pidx(e0)], inv_m), y1 = cscale(lds[pidx(e0 + 1)], inv_m);
        if constexpr (MODE == FM_RAAR) {
            // z is formed again (carry + gathered object term, as in the
            // prologue) instead of being held in registers across the four
            // transforms: 32 registers fewer, a wave per SIMD more
            float2 w0, w1, za, zb, ta, tb;
            prologue2<MODE>(A, frame, rem / M, rem % M, fb, e0, rem, za, zb, ta, tb);
            ld2(A.w, rem, w0, w1);
            const float b = A.beta, c = 1.f - 2.f * A.beta;
            st2(A.u + fb, e0, cadd(cscale(za, b), cscale(y0, c)), cadd(cscale(zb, b), cscale(y1, c)));
            st2(A.v + fb, e0, cconjmul(w0, csub(cscale(y0, 2.f), za)), cconjmul(w1, csub(cscale(y1, 2.f), zb)));
        } else if constexpr (MODE == FM_PA) {
            st2(A.out + fb, e0, y0, y1);
        } else if constexpr (MODE == FM_GRAD) {
            // T psi is gathered again (object reads hit the caches) rather than
            // held in registers across the transforms
            float2 w0, w1, t0, t1;
            ld2(A.w, rem, w0, w1);
            gather2(A, frame, rem / M, rem % M, t0, t1);
            const float2 r0 = cscale(y0, 2.f), r1 = cscale(y1, 2.f);
            st2(A.v + fb, e0, cconjmul(w0, r0), cconjmul(w1, r1));
            gacc[2 * k] = cadd(gacc[2 * k], cconjmul(t0, r0));
            gacc[2 * k + 1] = cadd(gacc[2 * k + 1], cconjmul(t1, r1));
        }
    }
    __syncthreads();
}

template <int M, int MODE>
__global__ void __launch_bounds__(FG<M>::NT) fg_kernel(FrameArgs A) {
    using C = FG<M>;
    constexpr int NT = C::NT, G = C::G, NP = C::NP, MM = M * M;
    extern __shared__ float2 smem[];
    __shared__ float red[NT / 64];
    float2* lds = smem;
    float2* twl = smem + C::LDS;
    for (int t = threadIdx.x; t < M; t += NT) twl[t] = A.tw[t];

    float resid = 0.f;
    if constexpr (MODE != FM_GRAD) {
        // grid = groups: one group per workgroup (no loop, so nothing is
        // hoisted across groups and held in registers)
        fg_group<M, MODE>(A, blockIdx.x, lds, twl, resid, nullptr);
        if constexpr (MODE == FM_RAAR || MODE == FM_PA) {
            const float s = block_sum(resid, red);
            if (threadIdx.x == 0) A.resid[blockIdx.x] = s;
        }
        return;
    }
    // GRAD: grid may be smaller than the groups (probe-gradient slots)
    float2 gacc[2 * NP];
#pragma unroll
    for (int i = 0; i < 2 * NP; ++i) gacc[i] = make_float2(0.f, 0.f);
    const int ngroups = (A.K + G - 1) / G;
    for (int grp = blockIdx.x; grp < ngroups; grp += gridDim.x) fg_group<M, MODE>(A, grp, lds, twl, resid, gacc);
    {
        const float s = block_sum(resid, red);
        if (threadIdx.x == 0) A.resid[blockIdx.x] = s;
    }
    if constexpr (MODE == FM_GRAD) {
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const int e0 = 2 * (threadIdx.x + NT * k);
            const int f = e0 / MM, rem = e0 % MM;
            st2(A.gw_part + (size_t)blockIdx.x * G * MM, f * MM + rem, gacc[2 * k], gacc[2 * k + 1]);
        }
    }
}

// ---------------------------------------------------------------------------
// m = 128, Fourier-domain carry: U = F u is kept per frame, so an iteration
// is Z = U + F(g w_g T psi), Y = a sgn Z, U' = beta Z + (1 - 2 beta) Y and
// v = conj(w) F*(2Y - Z) -- no frame-space iterate has to survive the
// transforms.  One 1024-thread workgroup per CU loops over frames.  A
// 128-point line lives in 8 threads (16 elements each): a radix-8 and a
// radix-16 Stockham stage in registers, the exchange between them inside the
// line's wavefront.  Rows -> columns -> rows go through one 128 KiB LDS frame
// buffer, two workgroup barriers per frame.  Plan A (radix 8, then 16) starts
// from element pairs 2t + h + 16 r, plan B (16, then 8) ends on them, so every
// global access moves two adjacent elements; U and a second copy of the
// amplitudes are stored transposed per frame ([kx][ky]) for the same reason
// on the column side.
// ---------------------------------------------------------------------------
static const Timer kNoTimer{};

// Argument block of scan `scan` in a batch launch: the by-value copy with the
// fields that change on the device between iterations taken from D.
__device__ __forceinline__ FrameArgs batch_args(const BatchArgs& CH, const FrameArgs* __restrict__ D, int scan) {
    FrameArgs A = CH.a[scan - CH.base];
    A.g = D[scan].g;
    A.beta = D[scan].beta;
    A.gather = D[scan].gather;
    return A;
}

// LDS position of frame element (y, x): XOR swizzle of the low five bits of
// x, chosen so that the row-thread and column-thread patterns below (8 lines
// of 8 threads per wavefront) hit distinct banks, except plan B's second-stage
// column reads (two-way).
__device__ __forceinline__ int sw128(int y, int x) {
    const int b0 = (y ^ (y >> 2)) & 1, b3 = (y ^ (y >> 4)) & 1, b4 = ((y >> 1) ^ (y >> 5)) & 1;
    return y * 128 + (x ^ (x >> 4) ^ b0 ^ (b3 << 3) ^ (b4 << 4));
}

// A copy of an index the compiler must treat as unknown (keeps address
// arithmetic local to the stage that uses it).
__device__ __forceinline__ int opaque(int x) {
    asm volatile("" : "+v"(x));
    return x & 1023;
}

template <bool COL>
__device__ __forceinline__ int l128_at(int line, int e) {
    return COL ? sw128(e, line) : sw128(line, e);
}

// Plan A: held v[2 r + h] = element 2t + h + 16 r.  Radix-8 butterflies
// 2t, 2t + 1 -> LDS elements 8 j + q; radix-16 butterfly t on elements
// t + 8 r with twiddles W^(t r).  Ends with v[q] = element t + 8 q.
template <int DIR, bool COL>
__device__ __forceinline__ void l128_planA(float2 (&v)[16], float2* lds, const float2* twl, int line, int t) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        float2 b[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) b[r] = v[2 * r + h];
        dft<8, DIR>(b);
#pragma unroll
        for (int q = 0; q < 8; ++q) lds[l128_at<COL>(line, 8 * (2 * t + h) + q)] = b[q];
    }
    line_sync();
    line = opaque(line);
    t = opaque(t);
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = lds[l128_at<COL>(line, t + 8 * r)];
#pragma unroll
    for (int r = 1; r < 16; ++r) {
        float2 w = twl[t * r];
        if constexpr (DIR < 0) w.y = -w.y;
        v[r] = cmul(v[r], w);
    }
    dft<16, DIR>(v);
}

// Plan B: held v[r] = element t + 8 r.  Radix-16 butterfly t -> LDS
// elements 16 t + q; radix-8 butterflies k = 2t, 2t + 1 on elements k + 16 r
// with twiddles W^(k r).  Ends with v[2 q + h] = element 2t + h + 16 q.
template <int DIR, bool COL>
__device__ __forceinline__ void l128_planB(float2 (&v)[16], float2* lds, const float2* twl, int line, int t) {
    dft<16, DIR>(v);
#pragma unroll
    for (int q = 0; q < 16; ++q) lds[l128_at<COL>(line, 16 * t + q)] = v[q];
    line_sync();
    line = opaque(line);
    t = opaque(t);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int k = 2 * t + h;
        float2 b[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) b[r] = lds[l128_at<COL>(line, k + 16 * r)];
#pragma unroll
        for (int r = 1; r < 8; ++r) {
            float2 w = twl[k * r];
            if constexpr (DIR < 0) w.y = -w.y;
            b[r] = cmul(b[r], w);
        }
        dft<8, DIR>(b);
#pragma unroll
        for (int q = 0; q < 8; ++q) v[2 * q + h] = b[q];
    }
}

enum Fc128Mode : int { FC_RAAR = 0, FC_TO_SPACE = 1, FC_TO_CARRY = 2, FC_GRAD = 3 };

template <int MODE>
using Fc128Op = ModOp<MODE == FC_GRAD ? FM_GRAD : FM_RAAR, 128>;

constexpr size_t kFc128Smem = (size_t)(128 * 128 + 128) * sizeof(float2);
constexpr int kFc128Groups = 256;

// Workgroup b takes frames s, s + G, s + 2G, ... with s = fc128_slot(b, G)
// and writes one residual partial; the batched form runs the same (scan, b)
// items, so both sum the residual in the same order.  Workgroups are spread
// over the XCDs round-robin (b mod 8), so the slot map gives each XCD a run of
// G/8 consecutive frames at a time: neighbouring frames gather overlapping
// object windows, which then hit that XCD's L2.
__host__ __device__ int fc128_groups(int K) { return K < 1 ? 1 : (K < kFc128Groups ? K : kFc128Groups); }
__host__ __device__ int fc128_slot(int b, int G) { return (G & 7) ? b : (b & 7) * (G >> 3) + (b >> 3); }


// One frame f.  RAAR: the carry-form step (reads A.u = U transposed, A.at =
// amplitudes transposed, gathers psi; writes U' and v = conj(w) y).
// FC_TO_SPACE: A.in (U transposed) -> A.out = F* U (natural layout).
// FC_TO_CARRY: A.in (natural) -> A.out = F A.in (transposed).  FC_GRAD:
// z = w T psi, r = 2 F*(Z - a sgn Z); writes r itself to A.v (the merge
// applies conj(w) for Q* r, and a chunked pass forms sum conj(T psi) r, so
// no per-workgroup probe-gradient slot is read and rewritten per frame; those
// slots are larger than the L2 and cost as much traffic as r).  Ends with
// the row threads done with their rows: the next frame's first LDS writes
// are made by the same threads, so frames need no barrier between them.
template <int MODE, bool NT>
__device__ __forceinline__ void fc128_frame(const FrameArgs& A, int f, float2* lds, const float2* twl,
                                            Fc128Op<MODE>& op) {
    constexpr int M = 128, MM = M * M;
    const size_t fb = (size_t)f * MM;
    const float inv_m = 1.0f / M;
    float2 v[16];
    if constexpr (MODE != FC_TO_SPACE) {   // rows: load, forward row transform (plan A)
        const int tid = opaque_tid();
        const int row = tid >> 3, t = tid & 7;
        if constexpr (MODE == FC_RAAR || MODE == FC_GRAD) {
            const float g = MODE == FC_GRAD ? 1.f : A.g;
            const int py = A.pos[2 * f], px = A.pos[2 * f + 1];
            int gy = py + row;
            if (A.periodic && gy >= A.ny) gy -= A.ny;
            const unsigned orow = (unsigned)gy * (unsigned)A.nx;
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const int x = 2 * t + 16 * r;
                int gx0 = px + x, gx1 = gx0 + 1;
                if (A.periodic) {
                    if (gx0 >= A.nx) gx0 -= A.nx;
                    if (gx1 >= A.nx) gx1 -= A.nx;
                }
                float2 w0, w1;
                ld2(A.w_g, (unsigned)(row * M + x), w0, w1);
                v[2 * r] = gather_z(w0, ldc(A.psi, orow + gx0), g);
                v[2 * r + 1] = gather_z(w1, ldc(A.psi, orow + gx1), g);
            }
        } else {
#pragma unroll
            for (int r = 0; r < 8; ++r) ld2(A.in + fb, (unsigned)(row * M + 2 * t + 16 * r), v[2 * r], v[2 * r + 1]);
        }
        l128_planA<1, false>(v, lds, twl, row, t);
        const int row2 = opaque(row), t2 = opaque(t);
#pragma unroll
        for (int q = 0; q < 16; ++q) lds[sw128(row2, t2 + 8 * q)] = v[q];
        __syncthreads();
    }
    {   // columns
        const int tid = opaque_tid();
        const int c = 8 * (tid >> 6) + (tid & 7), t = (tid >> 3) & 7;
        const unsigned cb = (unsigned)(c * M + 2 * t);   // transposed pair (c, 2t + 16 q)
        if constexpr (MODE == FC_TO_SPACE) {
#pragma unroll
            for (int q = 0; q < 8; ++q) ld2(A.in + fb, cb + 16 * q, v[2 * q], v[2 * q + 1]);
        } else {
            // amplitudes and the first half of the carry are fetched ahead of the
            // column transform (what the register budget allows)
            float2 av8[8], u8[8];
            if constexpr (MODE == FC_RAAR || MODE == FC_GRAD) {
#pragma unroll
                for (int q = 0; q < 8; ++q) av8[q] = ldf2t<NT>(A.at + fb, cb + 16 * q);
            }
            if constexpr (MODE == FC_RAAR) {
#pragma unroll
                for (int q = 0; q < 4; ++q) ld2t<NT>(A.u + fb, cb + 16 * q, u8[2 * q], u8[2 * q + 1]);
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) v[r] = lds[sw128(t + 8 * r, c)];
            l128_planB<1, true>(v, lds, twl, c, t);
            if constexpr (MODE == FC_TO_CARRY) {
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    st2(A.out + fb, cb + 16 * q, cscale(v[2 * q], inv_m), cscale(v[2 * q + 1], inv_m));
                return;
            } else if constexpr (MODE == FC_GRAD) {
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const float2 av = av8[q];
                    v[2 * q] = cscale(op.modulus(cscale(v[2 * q], inv_m), av.x, true), 2.f);
                    v[2 * q + 1] = cscale(op.modulus(cscale(v[2 * q + 1], inv_m), av.y, true), 2.f);
                }
            } else {
                const float b = A.beta, c1 = 1.f - 2.f * A.beta;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    float2 u0, u1;
                    if (q < 4) {
                        u0 = u8[2 * q];
                        u1 = u8[2 * q + 1];
                    } else {
                        ld2t<NT>(A.u + fb, cb + 16 * q, u0, u1);
                    }
                    const float2 av = av8[q];
                    const float2 z0 = cadd(u0, cscale(v[2 * q], inv_m)), z1 = cadd(u1, cscale(v[2 * q + 1], inv_m));
                    const float2 y0 = op.modulus(z0, av.x, true), y1 = op.modulus(z1, av.y, true);
                    st2t<NT>(A.u + fb, cb + 16 * q, cadd(cscale(z0, b), cscale(y0, c1)), cadd(cscale(z1, b), cscale(y1, c1)));
                    v[2 * q] = csub(cscale(y0, 2.f), z0);
                    v[2 * q + 1] = csub(cscale(y1, 2.f), z1);
                }
            }
        }
        l128_planA<-1, true>(v, lds, twl, c, t);
        const int c2 = opaque(c), t2 = opaque(t);   // fresh addresses, not the ones of the first reads
#pragma unroll
        for (int q = 0; q < 16; ++q) lds[sw128(t2 + 8 * q, c2)] = v[q];
    }
    __syncthreads();
    {   // rows: inverse row transform (plan B), store
        const int tid = opaque_tid();
        const int row = tid >> 3, t = tid & 7;
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = lds[sw128(row, t + 8 * r)];
        l128_planB<-1, false>(v, lds, twl, row, t);
        // RAAR: the probe row is requested before the first store of v (a load
        // issued after a store is waited for together with the store)
        float2 wr[16];
        if constexpr (MODE == FC_RAAR) {
#pragma unroll
            for (int q = 0; q < 8; ++q) ld2(A.w, (unsigned)(row * M + 2 * t + 16 * q), wr[2 * q], wr[2 * q + 1]);
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const unsigned o = (unsigned)(row * M + 2 * t + 16 * q);
            if constexpr (MODE == FC_RAAR) {
                const float2 w0 = wr[2 * q], w1 = wr[2 * q + 1];
                st2t<NT>(A.v + fb, o, cconjmul(w0, cscale(v[2 * q], inv_m)), cconjmul(w1, cscale(v[2 * q + 1], inv_m)));
            } else if constexpr (MODE == FC_GRAD) {
                st2t<NT>(A.v + fb, o, cscale(v[2 * q], inv_m), cscale(v[2 * q + 1], inv_m));
            } else {
                st2(A.out + fb, o, cscale(v[2 * q], inv_m), cscale(v[2 * q + 1], inv_m));
            }
        }
    }
}

template <int MODE, bool NT>
__global__ void __launch_bounds__(1024) fc128_kernel(FrameArgs A) {
    extern __shared__ float2 smem[];
    __shared__ float red[16];
    float2* lds = smem;
    float2* twl = smem + 128 * 128;
    for (int t = threadIdx.x; t < 128; t += 1024) twl[t] = A.tw[t];
    __syncthreads();
    Fc128Op<MODE> op{nullptr, nullptr, 0.f};
    const int first = fc128_slot(blockIdx.x, gridDim.x);
    for (int f = first; f < A.K; f += gridDim.x) {
        fc128_frame<MODE, NT>(A, f, lds, twl, op);
        if constexpr (MODE == FC_TO_SPACE || MODE == FC_TO_CARRY)
            __syncthreads();   // conversions start or end on the column side
    }
    if constexpr (MODE == FC_RAAR || MODE == FC_GRAD) {
        const float s = block_sum(op.resid, red);
        if (threadIdx.x == 0) A.resid[blockIdx.x] = s;
    }
}

template <int MODE, bool NT>
static hipError_t launch_fc128_nt(const FrameArgs& A, int grid, hipStream_t s) {
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)fc128_kernel<MODE, NT>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFc128Smem);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL((fc128_kernel<MODE, NT>), dim3(grid), dim3(1024), kFc128Smem, s, A);
    return hipGetLastError();
}

template <int MODE>
static hipError_t launch_fc128_mode(const FrameArgs& A, hipStream_t s) {
    return A.stream ? launch_fc128_nt<MODE, true>(A, fc128_groups(A.K), s)
                    : launch_fc128_nt<MODE, false>(A, fc128_groups(A.K), s);
}

hipError_t launch_fc128(const FrameArgs& A, hipStream_t s, const Timer* tp, int* blocks_used) {
    const Timer& t = tp ? *tp : kNoTimer;
    t.begin(TC_FRAME);
    hipError_t e = launch_fc128_mode<FC_RAAR>(A, s);
    t.end(TC_FRAME);
    *blocks_used = fc128_groups(A.K);
    return e;
}

hipError_t launch_fc128_convert(const FrameArgs& A, int to_space, hipStream_t s) {
    // the conversions use none of the streaming accesses
    return to_space ? launch_fc128_nt<FC_TO_SPACE, false>(A, fc128_groups(A.K), s)
                    : launch_fc128_nt<FC_TO_CARRY, false>(A, fc128_groups(A.K), s);
}

hipError_t launch_fc128_grad(const FrameArgs& A, int grid, hipStream_t s, const Timer* tp, int* blocks_used) {
    const Timer& t = tp ? *tp : kNoTimer;
    grid = std::max(1, std::min(grid, A.K));
    t.begin(TC_FRAME);
    const hipError_t e = A.stream ? launch_fc128_nt<FC_GRAD, true>(A, grid, s) : launch_fc128_nt<FC_GRAD, false>(A, grid, s);
    t.end(TC_FRAME);
    *blocks_used = grid;
    return e;
}

__global__ void __launch_bounds__(1024) batch_fc128_kernel(const BatchArgs CH, const FrameArgs* __restrict__ D,
                                                           const int2* __restrict__ items, int n) {
    extern __shared__ float2 smem[];
    __shared__ float red[16];
    float2* lds = smem;
    float2* twl = smem + 128 * 128;
    const int it = blockIdx.x;
    if (it >= n) return;
    const int2 w = items[it];
    const FrameArgs A = batch_args(CH, D, w.x);
    for (int t = threadIdx.x; t < 128; t += 1024) twl[t] = A.tw[t];
    __syncthreads();
    const int G = fc128_groups(A.K);
    Fc128Op<FC_RAAR> op{nullptr, nullptr, 0.f};
    if (A.stream)
        for (int f = fc128_slot(w.y, G); f < A.K; f += G) fc128_frame<FC_RAAR, true>(A, f, lds, twl, op);
    else
        for (int f = fc128_slot(w.y, G); f < A.K; f += G) fc128_frame<FC_RAAR, false>(A, f, lds, twl, op);
    const float s = block_sum(op.resid, red);
    if (threadIdx.x == 0) A.resid[w.y] = s;
}

hipError_t batch_fc128_prepare(int* blocks_per_cu) {
    hipError_t e = hipFuncSetAttribute((const void*)batch_fc128_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)kFc128Smem);
    *blocks_per_cu = 1;
    return e;
}

hipError_t launch_batch_fc128(const BatchArgs& C, const FrameArgs* D, const int2* items, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(batch_fc128_kernel, dim3(n), dim3(1024), kFc128Smem, s, C, D, items, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// m = 256: three passes through an HBM stage buffer
// ---------------------------------------------------------------------------
template <int M, int NT_ = 256>
struct MP {
    static constexpr int NT = NT_, E = 16, NP = E / 2;
    static constexpr int RB = NT * E / M;  // rows per row-pass workgroup
    static constexpr int CB = NT * E / M;  // columns per column-pass workgroup
    static constexpr int NRB = M / RB, NCB = M / CB;
    static constexpr int LDS = pidx(NT * E);
    static constexpr size_t SMEM = (size_t)(LDS + M) * sizeof(float2);
};

// Row pass forward on item it = frame * NRB + row block: prologue + row FFTs -> stage
template <int M, int MODE, int NTB = 256>
__device__ __forceinline__ void mp_row_fwd_item(const FrameArgs& A, int it, float2* lds, const float2* twl) {
    const int tid = opaque_tid();
    using C = MP<M, NTB>;
    constexpr int NT = C::NT, NP = C::NP, RB = C::RB, MM = M * M, NRB = C::NRB;
    const int frame = it / NRB, rb = it % NRB;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int e0 = 2 * (tid + NT * k);
        const int y = rb * RB + e0 / M, x = e0 % M, rem = y * M + x;
        float2 z0, z1, t0, t1;
        prologue2<MODE>(A, frame, y, x, (size_t)frame * MM, rem, rem, z0, z1, t0, t1);
        lds[pidx(e0)] = z0;
        lds[pidx(e0 + 1)] = z1;
    }
    __syncthreads();
    constexpr int D1 = (MODE == FM_FINV) ? -1 : 1;
    NoPost none;
    fft_1d<M, D1, NT, RB, RowLay<M>>(lds, twl, none);
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int e0 = 2 * (tid + NT * k);
        const int y = rb * RB + e0 / M, x = e0 % M;
        st2(A.stage + (size_t)frame * MM, y * M + x, lds[pidx(e0)], lds[pidx(e0 + 1)]);
    }
    __syncthreads();
}

template <int M, int MODE, int NTB = 256>
__global__ void __launch_bounds__(NTB) mp_row_fwd(FrameArgs A) {
    using C = MP<M, NTB>;
    extern __shared__ float2 smem[];
    float2* lds = smem;
    float2* twl = smem + C::LDS;
    for (int t = threadIdx.x; t < M; t += C::NT) twl[t] = A.tw[t];
    const int items = A.K * C::NRB;
    for (int it = blockIdx.x; it < items; it += gridDim.x) mp_row_fwd_item<M, MODE, NTB>(A, it, lds, twl);
}

template <int M, int MODE, int NTB = 256>
struct CBPost {
    ModOp<MODE, M> op;  // bases point at the frame (amplitudes: column-block layout)
    int x0;             // first column of this block
    __device__ __forceinline__ void operator()(int addr, float2& v) {
        constexpr int CB = MP<M, NTB>::CB;
        const unsigned y = addr / CB, x = x0 + addr % CB;
        op.apply(true, MODE == FM_SIM ? y * M + x : cb256(y, x), v);
    }
};

// Column pass on item it = frame * NCB + column block: column FFTs + Fourier op
// (+ inverse column FFTs); returns this thread's residual contribution.
template <int M, int MODE, int NTB = 256>
__device__ __forceinline__ float mp_col_item(const FrameArgs& A, int it, float2* lds, const float2* twl) {
    const int tid = opaque_tid();
    using C = MP<M, NTB>;
    constexpr int NT = C::NT, NP = C::NP, CB = C::CB, MM = M * M, NCB = C::NCB;
    const int frame = it / NCB, cb = it % NCB;
    const size_t fb = (size_t)frame * MM;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int e0 = 2 * (tid + NT * k);
        const int y = e0 / CB, c = e0 % CB;
        float2 a0, a1;
        ld2(A.stage + fb, y * M + cb * CB + c, a0, a1);
        lds[pidx(e0)] = a0;
        lds[pidx(e0 + 1)] = a1;
    }
    __syncthreads();
    constexpr int D1 = (MODE == FM_FINV) ? -1 : 1;
    CBPost<M, MODE, NTB> post{{A.a + fb, A.out_f + fb, 0.f}, cb * CB};
    fft_1d_post<M, D1, NT, CB, ColLayCB<CB>>(lds, twl, post);
    if constexpr (MODE == FM_SIM) return post.op.resid;
    float2* dst = A.stage;
    if constexpr (MODE == FM_F || MODE == FM_FINV) {
        dst = A.out;
    } else {
        NoPost none;
        fft_1d<M, -1, NT, CB, ColLayCB<CB>>(lds, twl, none);
    }
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int e0 = 2 * (tid + NT * k);
        const int y = e0 / CB, c = e0 % CB;
        st2(dst + fb, y * M + cb * CB + c, lds[pidx(e0)], lds[pidx(e0 + 1)]);
    }
    __syncthreads();
    return post.op.resid;
}

template <int M, int MODE, int NTB = 256>
__global__ void __launch_bounds__(NTB) mp_col(FrameArgs A) {
    using C = MP<M, NTB>;
    extern __shared__ float2 smem[];
    __shared__ float red[C::NT / 64];
    float2* lds = smem;
    float2* twl = smem + C::LDS;
    for (int t = threadIdx.x; t < M; t += C::NT) twl[t] = A.tw[t];
    float resid = 0.f;
    const int items = A.K * C::NCB;
    for (int it = blockIdx.x; it < items; it += gridDim.x) resid += mp_col_item<M, MODE, NTB>(A, it, lds, twl);
    if constexpr (MODE == FM_RAAR || MODE == FM_PA || MODE == FM_GRAD) {
        const float s = block_sum(resid, red);
        if (threadIdx.x == 0) A.resid[blockIdx.x] = s;
    }
}

// Row pass inverse on item it: inverse row FFTs + epilogue
template <int M, int MODE, int NTB = 256>
__device__ __forceinline__ void mp_row_inv_item(const FrameArgs& A, int it, float2* lds, const float2* twl,
                                                float2* gacc) {
    const int tid = opaque_tid();
    using C = MP<M, NTB>;
    constexpr int NT = C::NT, NP = C::NP, RB = C::RB, MM = M * M, NRB = C::NRB;
    const int frame = it / NRB, rb = it % NRB;
    const size_t fb = (size_t)frame * MM;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int e0 = 2 * (tid + NT * k);
        const int y = rb * RB + e0 / M, x = e0 % M;
        float2 a0, a1;
        ld2(A.stage + fb, y * M + x, a0, a1);
        lds[pidx(e0)] = a0;
        lds[pidx(e0 + 1)] = a1;
    }
    __syncthreads();
    NoPost none;
    fft_1d<M, -1, NT, RB, RowLay<M>>(lds, twl, none);
    const float inv_m = 1.0f / M;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int e0 = 2 * (tid + NT * k);
        const int y = rb * RB + e0 / M, x = e0 % M, rem = y * M + x;
        const float2 y0 = cscale(lds[pidx(e0)], inv_m), y1 = cscale(lds[pidx(e0 + 1)], inv_m);
        if constexpr (MODE == FM_RAAR) {
            float2 z0, z1, t0, t1, w0, w1;
            prologue2<MODE>(A, frame, y, x, fb, rem, rem, z0, z1, t0, t1);
            ld2(A.w, rem, w0, w1);
            const float b = A.beta, c = 1.f - 2.f * A.beta;
            st2(A.u + fb, rem, cadd(cscale(z0, b), cscale(y0, c)), cadd(cscale(z1, b), cscale(y1, c)));
            st2(A.v + fb, rem, cconjmul(w0, csub(cscale(y0, 2.f), z0)), cconjmul(w1, csub(cscale(y1, 2.f), z1)));
        } else if constexpr (MODE == FM_PA) {
            st2(A.out + fb, rem, y0, y1);
        } else if constexpr (MODE == FM_GRAD) {
            float2 t0, t1, w0, w1;
            gather2(A, frame, y, x, t0, t1);
            ld2(A.w, rem, w0, w1);
            const float2 r0 = cscale(y0, 2.f), r1 = cscale(y1, 2.f);
            st2(A.v + fb, rem, cconjmul(w0, r0), cconjmul(w1, r1));
            gacc[2 * k] = cadd(gacc[2 * k], cconjmul(t0, r0));
            gacc[2 * k + 1] = cadd(gacc[2 * k + 1], cconjmul(t1, r1));
        }
    }
    __syncthreads();
}

template <int M, int MODE, int NTB = 256>
__global__ void __launch_bounds__(NTB) mp_row_inv(FrameArgs A) {
    using C = MP<M, NTB>;
    constexpr int NT = C::NT, NP = C::NP, RB = C::RB, MM = M * M, NRB = C::NRB;
    extern __shared__ float2 smem[];
    float2* lds = smem;
    float2* twl = smem + C::LDS;
    for (int t = threadIdx.x; t < M; t += NT) twl[t] = A.tw[t];
    float2 gacc[2 * NP];
#pragma unroll
    for (int i = 0; i < 2 * NP; ++i) gacc[i] = make_float2(0.f, 0.f);
    const int items = A.K * NRB;
    for (int it = blockIdx.x; it < items; it += gridDim.x) mp_row_inv_item<M, MODE, NTB>(A, it, lds, twl, gacc);
    if constexpr (MODE == FM_GRAD) {
        // gridDim.x is a multiple of NRB, so this block only saw row block blockIdx.x % NRB.
        const int slot = blockIdx.x / NRB, rb = blockIdx.x % NRB;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const int e0 = 2 * (threadIdx.x + NT * k);
            const int y = rb * RB + e0 / M, x = e0 % M;
            st2(A.gw_part + (size_t)slot * MM, y * M + x, gacc[2 * k], gacc[2 * k + 1]);
        }
    }
}

// ---------------------------------------------------------------------------
// Q alone for any m (no transform): out = w T psi
// ---------------------------------------------------------------------------
template <int M>
__global__ void __launch_bounds__(256) q_kernel(FrameArgs A) {
    constexpr int MM = M * M;
    const size_t npairs = (size_t)A.K * MM / 2;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < npairs; i += (size_t)gridDim.x * 256) {
        const size_t e0 = 2 * i;
        const int frame = (int)(e0 / MM), rem = (int)(e0 % MM), y = rem / M, x = rem % M;
        float2 z0, z1, t0, t1;
        prologue2<FM_Q>(A, frame, y, x, 0, 0, rem, z0, z1, t0, t1);
        st2(A.out + e0, 0, z0, z1);
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <int M, int MODE>
static hipError_t launch_fg(const FrameArgs& A, int grid, hipStream_t s, const Timer& t) {
    using C = FG<M>;
    auto k = fg_kernel<M, MODE>;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)C::SMEM);
        if (e != hipSuccess) return e;
        attr = true;
    }
    t.begin(TC_FRAME);
    hipLaunchKernelGGL(k, dim3(grid), dim3(C::NT), C::SMEM, s, A);
    t.end(TC_FRAME);
    return hipGetLastError();
}

template <int M, int MODE, int NTB = 256>
static hipError_t launch_mp(const FrameArgs& A, int grid_rows, int grid_cols, int grid_inv, hipStream_t s,
                            const Timer& t) {
    using C = MP<M, NTB>;
    t.begin(TC_FRAME);
    hipLaunchKernelGGL((mp_row_fwd<M, MODE, NTB>), dim3(grid_rows), dim3(NTB), C::SMEM, s, A);
    t.end(TC_FRAME);
    t.begin(TC_COLS);
    hipLaunchKernelGGL((mp_col<M, MODE, NTB>), dim3(grid_cols), dim3(NTB), C::SMEM, s, A);
    t.end(TC_COLS);
    if constexpr (MODE == FM_RAAR || MODE == FM_PA || MODE == FM_GRAD) {
        t.begin(TC_FRAME_OUT);
        hipLaunchKernelGGL((mp_row_inv<M, MODE, NTB>), dim3(grid_inv), dim3(NTB), C::SMEM, s, A);
        t.end(TC_FRAME_OUT);
    }
    return hipGetLastError();
}

// RAAR frame phase for m = 256 with a chosen pass block (threads 128, 256 or
// 512: 8, 16 or 32 rows / columns per workgroup).
hipError_t launch_raar_mp256(const FrameArgs& A, int threads, hipStream_t s, const Timer* tp, int* blocks_used) {
    const Timer& t = tp ? *tp : kNoTimer;
    switch (threads) {
        case 128: {
            const int items = A.K * MP<256, 128>::NRB;
            *blocks_used = A.K * MP<256, 128>::NCB;
            return launch_mp<256, FM_RAAR, 128>(A, items, *blocks_used, items, s, t);
        }
        case 512: {
            const int items = A.K * MP<256, 512>::NRB;
            *blocks_used = A.K * MP<256, 512>::NCB;
            return launch_mp<256, FM_RAAR, 512>(A, items, *blocks_used, items, s, t);
        }
        default: {
            const int items = A.K * MP<256, 256>::NRB;
            *blocks_used = A.K * MP<256, 256>::NCB;
            return launch_mp<256, FM_RAAR, 256>(A, items, *blocks_used, items, s, t);
        }
    }
}

template <int M>
static hipError_t dispatch_m(int mode, const FrameArgs& A, int grid_hint, hipStream_t s, int* blocks_used,
                             const Timer& t) {
    if (mode == FM_Q) {
        const size_t npairs = (size_t)A.K * M * M / 2;
        int grid = (int)std::min<size_t>((npairs + 255) / 256, 65536);
        hipLaunchKernelGGL(q_kernel<M>, dim3(grid), dim3(256), 0, s, A);
        if (blocks_used) *blocks_used = 0;
        return hipGetLastError();
    }
    if constexpr (M <= 128) {
        using C = FG<M>;
        const int ngroups = (A.K + C::G - 1) / C::G;
        int grid = ngroups;
        if (mode == FM_GRAD && grid_hint > 0) grid = std::min(ngroups, grid_hint);
        if (blocks_used) *blocks_used = grid;
        switch (mode) {
            case FM_RAAR: return launch_fg<M, FM_RAAR>(A, grid, s, t);
            case FM_PA: return launch_fg<M, FM_PA>(A, grid, s, t);
            case FM_GRAD: return launch_fg<M, FM_GRAD>(A, grid, s, t);
            case FM_SIM: return launch_fg<M, FM_SIM>(A, grid, s, t);
            case FM_F: return launch_fg<M, FM_F>(A, grid, s, t);
            case FM_FINV: return launch_fg<M, FM_FINV>(A, grid, s, t);
        }
        return hipErrorInvalidValue;
    } else {
        using C = MP<M>;
        const int items = A.K * (M / C::RB);
        int ginv = items;
        if (mode == FM_GRAD && grid_hint > 0) {
            const int nrb = M / C::RB;
            ginv = std::max(nrb, std::min(items, (grid_hint / nrb) * nrb));
        }
        if (blocks_used) *blocks_used = (mode == FM_GRAD) ? ginv : items;
        switch (mode) {
            case FM_RAAR: return launch_mp<M, FM_RAAR>(A, items, items, ginv, s, t);
            case FM_PA: return launch_mp<M, FM_PA>(A, items, items, ginv, s, t);
            case FM_GRAD: return launch_mp<M, FM_GRAD>(A, items, items, ginv, s, t);
            case FM_SIM: return launch_mp<M, FM_SIM>(A, items, items, ginv, s, t);
            case FM_F: return launch_mp<M, FM_F>(A, items, items, ginv, s, t);
            case FM_FINV: return launch_mp<M, FM_FINV>(A, items, items, ginv, s, t);
        }
        return hipErrorInvalidValue;
    }
}

hipError_t launch_frame(int mode, const FrameArgs& A, int grid_hint, hipStream_t s, int* blocks_used,
                        const Timer* tp) {
    const Timer& t = tp ? *tp : kNoTimer;
    switch (A.M) {
        case 16: return dispatch_m<16>(mode, A, grid_hint, s, blocks_used, t);
        case 32: return dispatch_m<32>(mode, A, grid_hint, s, blocks_used, t);
        case 64: return dispatch_m<64>(mode, A, grid_hint, s, blocks_used, t);
        case 128: return dispatch_m<128>(mode, A, grid_hint, s, blocks_used, t);
        case 256: return dispatch_m<256>(mode, A, grid_hint, s, blocks_used, t);
    }
    return hipErrorInvalidValue;
}

int fg_groups(int M) {
    switch (M) {
        case 16: return FG<16>::G;
        case 32: return FG<32>::G;
        case 64: return FG<64>::G;
        case 128: return FG<128>::G;
    }
    return 1;
}

int frame_partial_slots(int M, int mode, int blocks) {
    if (mode != FM_GRAD) return 0;
    switch (M) {
        case 16: return blocks * FG<16>::G;
        case 32: return blocks * FG<32>::G;
        case 64: return blocks * FG<64>::G;
        case 128: return blocks * FG<128>::G;
        case 256: return blocks / (256 / MP<256>::RB);
    }
    return 0;
}

// ---------------------------------------------------------------------------
// probe update (Eq. (standardprobe)): per frame-chunk partial sums of
// conj(T psi_l) z and |T psi_l|^2 with z = u' + beta w T psi_v, then w = num/den
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) probe_partial_kernel(int M, int K, const int* __restrict__ pos, int nx,
                                                            int ny, int periodic, const float2* __restrict__ u,
                                                            const float2* __restrict__ w,
                                                            const float2* __restrict__ psi_v,
                                                            const float2* __restrict__ psi_l, float beta,
                                                            int chunks, float2* __restrict__ num,
                                                            float* __restrict__ den) {
    const int MM = M * M;
    const int p = blockIdx.y * 256 + threadIdx.x;  // pixel index in the frame
    if (p >= MM) return;
    const int c = blockIdx.x;
    const int f0 = (int)((long long)K * c / chunks), f1 = (int)((long long)K * (c + 1) / chunks);
    const int y = p / M, x = p % M;
    const float2 wp = w[p];
    float2 acc = make_float2(0.f, 0.f);
    float d = 0.f;
    for (int f = f0; f < f1; ++f) {
        int gy = pos[2 * f] + y, gx = pos[2 * f + 1] + x;
        if (periodic) {
            gy = wrap(gy, ny);
            gx = wrap(gx, nx);
        }
        const size_t o = (size_t)gy * nx + gx;
        const float2 zf = cadd(u[(size_t)f * MM + p], cscale(cmul(wp, psi_v[o]), beta));
        const float2 t = psi_l[o];
        acc = cadd(acc, cconjmul(t, zf));
        d += cabs2(t);
    }
    num[(size_t)c * MM + p] = acc;
    den[(size_t)c * MM + p] = d;
}

// Probe gradient of the frame-residual form (Eq. (standardprobe)'s numerator
// with r in place of z): per frame chunk, sum over its frames (ascending) of
// conj(T psi) r at every frame pixel; chunk partials are then added in fixed
// order by gw_finish_kernel.
__global__ void __launch_bounds__(256) grad_probe_partial_kernel(int M, int K, const int* __restrict__ pos, int nx,
                                                                 int ny, int periodic, const float2* __restrict__ r,
                                                                 const float2* __restrict__ psi, int chunks,
                                                                 float2* __restrict__ part) {
    const int MM = M * M;
    const int p = blockIdx.y * 256 + threadIdx.x;  // pixel index in the frame
    if (p >= MM) return;
    const int c = blockIdx.x;
    const int f0 = (int)((long long)K * c / chunks), f1 = (int)((long long)K * (c + 1) / chunks);
    const int y = p / M, x = p % M;
    float2 acc = make_float2(0.f, 0.f);
    for (int f = f0; f < f1; ++f) {
        int gy = pos[2 * f] + y, gx = pos[2 * f + 1] + x;
        if (periodic) {
            gy = wrap(gy, ny);
            gx = wrap(gx, nx);
        }
        acc = cadd(acc, cconjmul(psi[(size_t)gy * nx + gx], r[(size_t)f * MM + p]));
    }
    part[(size_t)c * MM + p] = acc;
}

// Fixed-order sums over C chunk partials ([C][MM] arrays), 32 pixels per
// 256-thread workgroup: thread (g, q) = (t / 32, t mod 32) adds chunks g,
// g + 8, g + 16, ... of pixel q in ascending order (independent loads, all in
// flight), then the eight partials of the pixel are added in g order.  The
// order depends on C only, never on scheduling.
constexpr int kSumPix = 32, kSumWays = 8;

__global__ void __launch_bounds__(256) probe_finish_kernel(int MM, int chunks, const float2* __restrict__ num,
                                                           const float* __restrict__ den, float2* __restrict__ w_gat,
                                                           float2* __restrict__ w_cur) {
    __shared__ float2 sn[kSumWays][kSumPix];
    __shared__ float sd[kSumWays][kSumPix];
    const int q = threadIdx.x % kSumPix, g = threadIdx.x / kSumPix;
    const int p = blockIdx.x * kSumPix + q;
    float2 n = make_float2(0.f, 0.f);
    float d = 0.f;
    if (p < MM)
        for (int c = g; c < chunks; c += kSumWays) {
            n = cadd(n, num[(size_t)c * MM + p]);
            d += den[(size_t)c * MM + p];
        }
    sn[g][q] = n;
    sd[g][q] = d;
    __syncthreads();
    if (g != 0 || p >= MM) return;
    for (int k = 1; k < kSumWays; ++k) {
        n = cadd(n, sn[k][q]);
        d += sd[k][q];
    }
    const float2 old = w_cur[p];
    w_gat[p] = old;
    w_cur[p] = d > 0.f ? cscale(n, 1.0f / d) : make_float2(0.f, 0.f);
}

// Probe constraint in the Fourier domain (algorithm box, step 7): kind 1
// multiplies by the mask, kind 2 keeps the phase and sets the magnitude
// (sgn(0) := 1).
__global__ void __launch_bounds__(256) probe_fourier_kernel(float2* __restrict__ W, const float* __restrict__ vals,
                                                            int MM, int kind) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= MM) return;
    const float2 v = W[p];
    const float c = vals[p];
    if (kind == 1) {
        W[p] = cscale(v, c);
    } else {
        const float n2 = cabs2(v);
        float2 s = make_float2(1.f, 0.f);
        if (n2 > 0.f) s = cscale(v, rsqrtf(n2));
        W[p] = cscale(s, c);
    }
}

// Centre-of-mass correction (algorithm box, step 7): one workgroup forms the
// centroid of |w|^2 (fixed-order FP32 sums), then rolls w circularly by
// s = floor(m/2 - centroid + 1/2) per axis through tmp.
__global__ void __launch_bounds__(1024) probe_center_kernel(float2* __restrict__ w, float2* __restrict__ tmp, int m) {
    __shared__ float red[3][16];
    __shared__ int shift[2];
    const int MM = m * m, tid = threadIdx.x;
    float t = 0.f, sy = 0.f, sx = 0.f;
    for (int p = tid; p < MM; p += 1024) {
        const float q = cabs2(w[p]);
        t += q;
        sy += (float)(p / m) * q;
        sx += (float)(p % m) * q;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        t += __shfl_xor(t, o, 64);
        sy += __shfl_xor(sy, o, 64);
        sx += __shfl_xor(sx, o, 64);
    }
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = t;
        red[1][tid >> 6] = sy;
        red[2][tid >> 6] = sx;
    }
    __syncthreads();
    if (tid == 0) {
        float T = 0.f, Y = 0.f, X = 0.f;
        for (int i = 0; i < 16; ++i) {
            T += red[0][i];
            Y += red[1][i];
            X += red[2][i];
        }
        int a = 0, b = 0;
        if (T > 0.f) {
            const float half = (float)(m / 2);
            a = (int)floorf(half - Y / T + 0.5f);
            b = (int)floorf(half - X / T + 0.5f);
        }
        shift[0] = a;
        shift[1] = b;
    }
    __syncthreads();
    const int a = shift[0], b = shift[1];
    if (a == 0 && b == 0) return;
    for (int p = tid; p < MM; p += 1024) {
        int y = (p / m + a) % m, x = (p % m + b) % m;
        if (y < 0) y += m;
        if (x < 0) x += m;
        tmp[y * m + x] = w[p];
    }
    __syncthreads();
    for (int p = tid; p < MM; p += 1024) w[p] = tmp[p];
}

hipError_t launch_probe_fourier(float2* W, const float* vals, int M, int kind, hipStream_t s) {
    hipLaunchKernelGGL(probe_fourier_kernel, dim3((M * M + 255) / 256), dim3(256), 0, s, W, vals, M * M, kind);
    return hipGetLastError();
}

hipError_t launch_probe_center(float2* w, float2* tmp, int M, hipStream_t s) {
    hipLaunchKernelGGL(probe_center_kernel, dim3(1), dim3(1024), 0, s, w, tmp, M);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) gw_finish_kernel(int MM, int slots, const float2* __restrict__ part,
                                                        float2* __restrict__ gw) {
    __shared__ float2 sp[kSumWays][kSumPix];   // same fixed order as probe_finish_kernel
    const int q = threadIdx.x % kSumPix, g = threadIdx.x / kSumPix;
    const int p = blockIdx.x * kSumPix + q;
    float2 acc = make_float2(0.f, 0.f);
    if (p < MM)
        for (int c = g; c < slots; c += kSumWays) acc = cadd(acc, part[(size_t)c * MM + p]);
    sp[g][q] = acc;
    __syncthreads();
    if (g != 0 || p >= MM) return;
    for (int k = 1; k < kSumWays; ++k) acc = cadd(acc, sp[k][q]);
    gw[p] = acc;
}

hipError_t launch_probe_partial(int M, int K, const int* pos, int nx, int ny, int periodic, const float2* u,
                                const float2* w, const float2* psi_v, const float2* psi_l, float beta, int chunks,
                                float2* num, float* den, hipStream_t s) {
    dim3 grid(chunks, (M * M + 255) / 256);
    hipLaunchKernelGGL(probe_partial_kernel, grid, dim3(256), 0, s, M, K, pos, nx, ny, periodic, u, w, psi_v, psi_l,
                       beta, chunks, num, den);
    return hipGetLastError();
}

hipError_t launch_grad_probe_partial(int M, int K, const int* pos, int nx, int ny, int periodic, const float2* r,
                                     const float2* psi, int chunks, float2* part, hipStream_t s) {
    dim3 grid(chunks, (M * M + 255) / 256);
    hipLaunchKernelGGL(grad_probe_partial_kernel, grid, dim3(256), 0, s, M, K, pos, nx, ny, periodic, r, psi, chunks,
                       part);
    return hipGetLastError();
}

hipError_t launch_probe_finish(int M, int chunks, const float2* num, const float* den, float2* w_gat, float2* w_cur,
                               hipStream_t s) {
    hipLaunchKernelGGL(probe_finish_kernel, dim3((M * M + kSumPix - 1) / kSumPix), dim3(256), 0, s, M * M, chunks,
                       num, den, w_gat, w_cur);
    return hipGetLastError();
}

hipError_t launch_gw_finish(int M, int slots, const float2* part, float2* gw, hipStream_t s) {
    hipLaunchKernelGGL(gw_finish_kernel, dim3((M * M + kSumPix - 1) / kSumPix), dim3(256), 0, s, M * M, slots, part, gw);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched execution: items (scan, local item) over a device table of scans.
// Each item runs exactly the arithmetic of the single-scan kernels and writes
// its residual partial where the single-scan launch (one item per block)
// would, so a batched iteration reproduces the single-scan one bit for bit.
// The grid is sized to the resident capacity and strides over the item list.
// ---------------------------------------------------------------------------
template <int M>
__global__ void __launch_bounds__(FG<M>::NT) batch_fg_kernel(const BatchArgs CH, const FrameArgs* __restrict__ D,
                                                             const int2* __restrict__ items, int n) {
    using C = FG<M>;
    extern __shared__ float2 smem[];
    __shared__ float red[C::NT / 64];
    float2* lds = smem;
    float2* twl = smem + C::LDS;
    const int it = blockIdx.x;
    if (it >= n) return;
    const int2 w = items[it];
    const FrameArgs A = batch_args(CH, D, w.x);
    for (int t = threadIdx.x; t < M; t += C::NT) twl[t] = A.tw[t];
    float resid = 0.f;
    fg_group<M, FM_RAAR>(A, w.y, lds, twl, resid, nullptr);
    const float s = block_sum(resid, red);
    if (threadIdx.x == 0) A.resid[w.y] = s;
}

template <int M, int PHASE>
__global__ void __launch_bounds__(256) batch_mp_kernel(const BatchArgs CH, const FrameArgs* __restrict__ D,
                                                       const int2* __restrict__ items, int n) {
    using C = MP<M>;
    extern __shared__ float2 smem[];
    __shared__ float red[C::NT / 64];
    float2* lds = smem;
    float2* twl = smem + C::LDS;
    const int it = blockIdx.x;
    if (it >= n) return;
    const int2 w = items[it];
    const FrameArgs A = batch_args(CH, D, w.x);
    for (int t = threadIdx.x; t < M; t += C::NT) twl[t] = A.tw[t];
    if constexpr (PHASE == 0) {
        mp_row_fwd_item<M, FM_RAAR>(A, w.y, lds, twl);
    } else if constexpr (PHASE == 1) {
        const float s = block_sum(mp_col_item<M, FM_RAAR>(A, w.y, lds, twl), red);
        if (threadIdx.x == 0) A.resid[w.y] = s;
    } else {
        mp_row_inv_item<M, FM_RAAR>(A, w.y, lds, twl, nullptr);
    }
}

template <class K>
static int occupancy(K k, int threads, size_t smem) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, threads, smem) != hipSuccess) return 1;
    return nb > 0 ? nb : 1;
}

template <int M>
static hipError_t prep_batch_fg() {
    return hipFuncSetAttribute((const void*)batch_fg_kernel<M>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)FG<M>::SMEM);
}

hipError_t batch_frame_prepare(int M, int phase, int* blocks_per_cu) {
    hipError_t e = hipSuccess;
    switch (M) {
        case 16: e = prep_batch_fg<16>(); *blocks_per_cu = occupancy(batch_fg_kernel<16>, FG<16>::NT, FG<16>::SMEM); break;
        case 32: e = prep_batch_fg<32>(); *blocks_per_cu = occupancy(batch_fg_kernel<32>, FG<32>::NT, FG<32>::SMEM); break;
        case 64: e = prep_batch_fg<64>(); *blocks_per_cu = occupancy(batch_fg_kernel<64>, FG<64>::NT, FG<64>::SMEM); break;
        case 128: e = prep_batch_fg<128>(); *blocks_per_cu = occupancy(batch_fg_kernel<128>, FG<128>::NT, FG<128>::SMEM); break;
        case 256:
            if (phase == 0) *blocks_per_cu = occupancy(batch_mp_kernel<256, 0>, 256, MP<256>::SMEM);
            else if (phase == 1) *blocks_per_cu = occupancy(batch_mp_kernel<256, 1>, 256, MP<256>::SMEM);
            else *blocks_per_cu = occupancy(batch_mp_kernel<256, 2>, 256, MP<256>::SMEM);
            break;
        default: return hipErrorInvalidValue;
    }
    return e;
}

hipError_t launch_batch_frame(int M, int phase, const BatchArgs& C, const FrameArgs* D, const int2* items, int n,
                              hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const dim3 g(n);
    switch (M) {
        case 16: hipLaunchKernelGGL(batch_fg_kernel<16>, g, dim3(FG<16>::NT), FG<16>::SMEM, s, C, D, items, n); break;
        case 32: hipLaunchKernelGGL(batch_fg_kernel<32>, g, dim3(FG<32>::NT), FG<32>::SMEM, s, C, D, items, n); break;
        case 64: hipLaunchKernelGGL(batch_fg_kernel<64>, g, dim3(FG<64>::NT), FG<64>::SMEM, s, C, D, items, n); break;
        case 128: hipLaunchKernelGGL(batch_fg_kernel<128>, g, dim3(FG<128>::NT), FG<128>::SMEM, s, C, D, items, n); break;
        case 256:
            if (phase == 0) hipLaunchKernelGGL((batch_mp_kernel<256, 0>), g, dim3(256), MP<256>::SMEM, s, C, D, items, n);
            else if (phase == 1) hipLaunchKernelGGL((batch_mp_kernel<256, 1>), g, dim3(256), MP<256>::SMEM, s, C, D, items, n);
            else hipLaunchKernelGGL((batch_mp_kernel<256, 2>), g, dim3(256), MP<256>::SMEM, s, C, D, items, n);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// m = 256 with the RAAR carry kept in the Fourier domain.
//
// With U = F u the iterate's spectrum is Z = U + F(g w_g T psi_v), so the
// row pass only transforms the gathered object term, the column pass forms
// Z, the projection Y = a sgn Z, the new carry U' = b Z + (1 - 2b) Y and the
// spectrum of the merge input V = 2Y - Z (then inverse column FFTs), and the
// last pass inverse-transforms rows of V straight into the overlap merge.
// The carry and the amplitudes are stored column-block-major (cb256), so the
// column pass reads and writes one contiguous block per workgroup.
// ---------------------------------------------------------------------------
template <bool STREAM>
__device__ float col_carry_item(const FrameArgs& A, int it, float2* lds, const float2* twl) {
    const int tid = opaque_tid();
    constexpr int M = 256;
    using C = MP<M, 256>;
    constexpr int NT = C::NT, NP = C::NP, CB = C::CB, MM = M * M, NCB = C::NCB;
    static_assert(CB == 16, "column block must match the cb256 layout");
    const int frame = it / NCB, cb = it % NCB;
    const size_t fb = (size_t)frame * MM;
    // LDS element e0 = y * 16 + c is also the offset of (y, 16 cb + c) inside
    // this block of the cb256 layout: the carry and amplitudes of the block are
    // fetched with the stage columns, ahead of the column FFTs
    const size_t blk = fb + (size_t)cb * M * CB;
    float2 uc[2 * NP], ac[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int e0 = 2 * (tid + NT * k);
        const int y = e0 / CB, c = e0 % CB;
        float2 a0, a1;
        ld2t<STREAM>(A.stage + fb, y * M + cb * CB + c, a0, a1);
        lds[pidx(e0)] = a0;
        lds[pidx(e0 + 1)] = a1;
    }
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int e0 = 2 * (tid + NT * k);
        ld2t<STREAM>(A.u + blk, e0, uc[2 * k], uc[2 * k + 1]);
        ac[k] = ldf2t<STREAM>(A.a + blk, e0);
    }
    __syncthreads();
    NoPost none;
    fft_1d<M, 1, NT, CB, ColLayCB<CB>>(lds, twl, none);
    // pointwise in the Fourier domain; the stage holds the transform of the
    // unscaled gather w_g T psi_v, so the coefficient g joins the 1/m of F
    const float gm = A.g * (1.0f / M), b = A.beta, c1 = 1.f - 2.f * A.beta;
    ModOp<FM_RAAR, M> op{nullptr, nullptr, 0.f};
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int e0 = 2 * (tid + NT * k);
        const float2 u0 = uc[2 * k], u1 = uc[2 * k + 1];
        const float2 av = ac[k];
        const float2 z0 = cadd(u0, cscale(lds[pidx(e0)], gm));
        const float2 z1 = cadd(u1, cscale(lds[pidx(e0 + 1)], gm));
        const float2 y0 = op.modulus(z0, av.x, true), y1 = op.modulus(z1, av.y, true);
        st2t<STREAM>(A.u + blk, e0, cadd(cscale(z0, b), cscale(y0, c1)), cadd(cscale(z1, b), cscale(y1, c1)));
        lds[pidx(e0)] = csub(cscale(y0, 2.f), z0);
        lds[pidx(e0 + 1)] = csub(cscale(y1, 2.f), z1);
    }
    __syncthreads();
    fft_1d<M, -1, NT, CB, ColLayCB<CB>>(lds, twl, none);
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int e0 = 2 * (tid + NT * k);
        const int y = e0 / CB, c = e0 % CB;
        st2t<STREAM>(A.stage + fb, y * M + cb * CB + c, lds[pidx(e0)], lds[pidx(e0 + 1)]);
    }
    __syncthreads();
    return op.resid;
}

template <bool NT>
__global__ void __launch_bounds__(256) col_carry_kernel(FrameArgs A) {
    using C = MP<256, 256>;
    extern __shared__ float2 smem[];
    __shared__ float red[C::NT / 64];
    float2* lds = smem;
    float2* twl = smem + C::LDS;
    for (int t = threadIdx.x; t < 256; t += C::NT) twl[t] = A.tw[t];
    const int items = A.K * C::NCB;
    for (int it = blockIdx.x; it < items; it += gridDim.x) {
        const float s = block_sum(col_carry_item<NT>(A, it, lds, twl), red);
        if (threadIdx.x == 0) A.resid[it] = s;
    }
}

// ---------------------------------------------------------------------------
// m = 256, form 3: the column pass forms its own row transform.
//
// The row transform of the gathered frame g = w_g T psi_v factors with
// x = 16 n1 + n2 and kx = k1 + 16 k2 as
//   G[y][k1 + 16 k2] = sum_n2 W16^(k2 n2) W256^(k1 n2) sum_n1 g[y][16 n1 + n2] W16^(k1 n1),
// so the 64 columns with k1 in {4q, .., 4q + 3} need only the four inner sums
// k1 = 4q + i of every (y, n2).  One 1024-thread workgroup takes one quarter
// q of one frame: it gathers the whole frame (the object window and the probe
// come from the caches), forms those inner sums (four radix-4 DFTs over n1 / 4
// and a four-term combination), twiddles them, runs the sixteen-point DFTs
// over n2, and then does what the column pass of the two-pass form does on its
// 64 columns: column FFTs, Z = U + (g / m) G, eps_a partials, Y = a sgn Z,
// U' = beta Z + (1 - 2 beta) Y, V = 2Y - Z, inverse column FFTs.  The merge
// input leaves in octet rows: element (k1, k2) of a row at 128 (k2 / 8) + 8 k1
// + k2 mod 8, so a quarter writes two runs of 256 bytes per row and a thread
// of the strip pass's line transforms (one k1, all k2) reads two runs of 64
// bytes, its 16 neighbours in the line the adjacent runs.  The four
// workgroups of a frame each repeat the gather and the n1 sums (the price of
// dropping the row-transformed frame's trip through memory).
//
// LDS: one 128 KiB buffer, laid out three ways in turn (inner sums, columns,
// rows of the result); the XOR swizzles keep the wavefront access patterns
// of each phase at two-way bank sharing (the minimum for 64-bit accesses).
// ---------------------------------------------------------------------------
// The swizzles follow this GPU's LDS banking, measured with the bank-conflict
// counter: 64 banks of 4 bytes, and a 64-bit access served per half
// wavefront (32 lanes), each half taking as many cycles as its most
// requested bank has distinct words -- so a half wavefront's 32 float2 must
// fall on 32 distinct slots modulo 32 float2.
namespace colg {
constexpr int M = 256, NT = 1024, QE = 64 * M;  // quarter: 64 columns x 256 rows
// inner sums S'(y, i, n2): written by 8 n2-pairs x 4 rows (y bits 5, 6) per
// half wavefront, read by 32 consecutive rows
__device__ __forceinline__ int l1(int y, int i, int n2) {
    const int f = (y & 31) ^ ((y >> 5) & 1) ^ (((y >> 6) & 1) << 4);
    return y * 64 + ((i * 16 + n2) ^ f);
}
// column c (0..63), position p (0..255) along the column
__device__ __forceinline__ int l2(int c, int p) { return c * M + (p ^ ((p >> 4) & 15) ^ ((c & 3) << 4)); }
// result rows: row y, column c; written by 2 columns x 16 rows, read in
// 16-byte pairs (2 c', 2 c' + 1) of one row (the XOR keeps a pair adjacent,
// swapped when bit 0 of the mask is set -- it never is: the mask is even)
__device__ __forceinline__ int l3(int y, int c) { return y * 64 + (c ^ ((y & 15) << 1)); }
// per-thread twiddles W^(j r) of the column lines: T[j][r] at 17 j + r
constexpr int TW17 = 16 * 17;
}  // namespace colg

// 256-point line held as v[r] = element j + 16 r by the 16 threads (j) of a
// line (one wavefront holds four lines): two radix-16 stages with one
// exchange through the line's LDS positions; ends with v[q] = element
// j + 16 q of the transform.  `at(p)` maps a line position to LDS.
template <int DIR, class At>
__device__ __forceinline__ void colg_line(float2 (&v)[16], float2* lds, const float2* tw17, int j_in, At at) {
    // the LDS addresses are formed again in each call instead of being held
    // live (in registers) from one transform to the next
    const int j = opaque(j_in) & 15;
    dft<16, DIR>(v);
    line_sync();   // every thread of the line has read its inputs
#pragma unroll
    for (int q = 0; q < 16; ++q) lds[at(16 * j + q)] = v[q];
    line_sync();
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = lds[at(j + 16 * r)];
#pragma unroll
    for (int r = 1; r < 16; ++r) {
        float2 t = tw17[17 * j + r];
        if constexpr (DIR < 0) t.y = -t.y;
        v[r] = cmul(v[r], t);
    }
    dft<16, DIR>(v);
}

// Gather and inner sums of the column pass with its own row transform: for
// every row y and n2 the four sums S(k1) = sum_n1 g[y][16 n1 + n2] W16^(k1 n1),
// k1 = 4 quarter + i, times W256^(k1 n2), into LDS.  A thread takes the pair
// n2 = 2h, 2h + 1 of two rows: 16-byte requests for the object and the probe
// (the object window starts anywhere, so its pairs are 8-byte aligned).  With
// n1 = 4a + b the 16 terms of each sum are taken b by b, four requests of
// each kind in flight per step.
template <bool PERIODIC>
__device__ __forceinline__ void colg_inner_sums(const FrameArgs& A, int py, int px, int quarter, float2* lds,
                                                const float2* twl) {
    using namespace colg;
    typedef float f4a8 __attribute__((ext_vector_type(4), aligned(8)));
    const int tid = opaque_tid();
    const int h = tid & 7, rr = (tid >> 3) & 7, wv = tid >> 6;
    const int nx = A.nx, ny = A.ny;
#pragma unroll 1
    for (int half = 0; half < 2; ++half) {
        const int y = (rr << 5) | (opaque(half) << 4) | wv;
        int gy = py + y;
        if constexpr (PERIODIC) gy = wrap(gy, ny);
        const float2* prow = A.psi + (size_t)gy * nx;
        const float2* wrow = A.w_g + y * M + 2 * h;
        float2 sacc[2][4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            float2 x[2][4];   // [n2 of the pair][a]
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const int n1 = 4 * a + b;
                const int gx = px + 16 * n1 + 2 * h;
                float2 p0, p1;
                if constexpr (!PERIODIC) {
                    const f4a8 t = *reinterpret_cast<const f4a8*>(prow + gx);
                    p0 = make_float2(t.x, t.y);
                    p1 = make_float2(t.z, t.w);
                } else {
                    const int g0 = wrap(gx, nx);   // gx < 2 nx
                    p0 = prow[g0];
                    p1 = prow[g0 + 1 == nx ? 0 : g0 + 1];
                }
                float2 w0, w1;
                ld2(wrow, 16 * n1, w0, w1);
                x[0][a] = cmul(w0, p0);
                x[1][a] = cmul(w1, p1);
            }
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                // T[b][i] = sum_a x[4a + b] W4^(a i), then the b term of each k1 sum
                dft4<1>(x[e][0], x[e][1], x[e][2], x[e][3]);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float2 term = b == 0 ? x[e][i] : cmul(x[e][i], w16<1>(b * (4 * quarter + i)));
                    sacc[e][i] = b == 0 ? term : cadd(sacc[e][i], term);
                }
            }
        }
#pragma unroll
        for (int e = 0; e < 2; ++e)
#pragma unroll
            for (int i = 0; i < 4; ++i)   // times W256^(k1 n2)
                lds[l1(y, i, 2 * h + e)] = cmul(sacc[e][i], twl[((4 * quarter + i) * (2 * h + e)) & 255]);
    }
}

// One quarter-frame item; writes its residual partial A.resid[4 frame + quarter]
// (wave sums in red[], added by thread 0 in wave order once the barrier after
// the inverse column transforms has made them visible).  The workgroup takes
// no further item, so it ends without a closing barrier.
template <bool STREAM>
__device__ void colg_item(const FrameArgs& A, int frame, int quarter, float2* lds, const float2* twl, float* red) {
    using namespace colg;
    const int tid = opaque_tid();
    const int py = A.pos[2 * frame], px = A.pos[2 * frame + 1];
    const int nx = A.nx, ny = A.ny;
    const unsigned MM = M * M;
    // ---- gather and the inner sums over n1 for k1 = 4 quarter + i ----------
    if (A.periodic) colg_inner_sums<true>(A, py, px, quarter, lds, twl);
    else colg_inner_sums<false>(A, py, px, quarter, lds, twl);
    __syncthreads();
    // carry and amplitudes of rows j + 16 q of column col (q256 layout: the
    // pair q, q + 1 of every thread of the column lies side by side, so a
    // request of the 16 threads covers 256 contiguous bytes); the amplitudes
    // and the first half of the carry are requested here, ahead of the DFTs
    // over n2 and the forward column transform (earlier, during the inner
    // sums, they do not fit the register budget), the second half in the
    // pointwise loop
    const int col = tid >> 4, j = tid & 15;
    const size_t qb = (size_t)frame * MM + (size_t)quarter * QE;
    const unsigned cofs = (unsigned)col * M + 2u * j;
    float2 uc[8];
    float ac[16];
#pragma unroll
    for (int q = 0; q < 16; q += 2) {
        const float2 t = ldf2t<STREAM>(A.at + qb, cofs + 16 * q);
        ac[q] = t.x;
        ac[q + 1] = t.y;
    }
#pragma unroll
    for (int q = 0; q < 8; q += 2) ld2t<STREAM>(A.u + qb, cofs + 16 * q, uc[q], uc[q + 1]);
    // ---- sixteen-point DFTs over n2: G[y][4 quarter + i + 16 k2] ------------
    {
        const int y = tid & 255, i = tid >> 8;
        float2 v[16];
#pragma unroll
        for (int n2 = 0; n2 < 16; ++n2) v[n2] = lds[l1(y, i, n2)];
        __syncthreads();   // the inner sums are read before the columns take the buffer
        dft<16, 1>(v);
#pragma unroll
        for (int k2 = 0; k2 < 16; ++k2) lds[l2(i * 16 + k2, y)] = v[k2];
    }
    __syncthreads();
    // ---- columns ------------------------------------------------------------
    auto at = [col](int p) { return colg::l2(col, p); };
    float2 v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = lds[at(j + 16 * r)];
    colg_line<1>(v, lds, twl + 256, j, at);
    const float gm = A.g * (1.0f / M), b = A.beta, c1 = 1.f - 2.f * A.beta;
    ModOp<FM_RAAR, M> op{nullptr, nullptr, 0.f};
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        if (half == 1) {
#pragma unroll
            for (int q = 0; q < 8; q += 2) ld2t<STREAM>(A.u + qb, cofs + 16 * (8 + q), uc[q], uc[q + 1]);
        }
#pragma unroll
        for (int q = 0; q < 8; q += 2) {
            const int e = 8 * half + q;
            float2 un[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const float2 z = cadd(uc[q + h], cscale(v[e + h], gm));
                const float2 yv = op.modulus_sel(z, ac[e + h]);
                un[h] = cadd(cscale(z, b), cscale(yv, c1));
                v[e + h] = csub(cscale(yv, 2.f), z);
            }
            st2t<STREAM>(A.u + qb, cofs + 16 * e, un[0], un[1]);
        }
    }
    {
        float r = op.resid;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) r += __shfl_xor(r, o, 64);
        if ((tid & 63) == 0) red[tid >> 6] = r;
    }
    colg_line<-1>(v, lds, twl + 256, j, at);
    __syncthreads();   // every column is done with the buffer; the wave sums are in red[]
    if (threadIdx.x == 0) {
        float s = 0.f;
        for (int i = 0; i < NT / 64; ++i) s += red[i];
        A.resid[4 * frame + quarter] = s;
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) lds[colg::l3(j + 16 * q, col)] = v[q];
    __syncthreads();
    // ---- rows of the result in octet rows: 2 x 256 contiguous bytes per row ---
    {
        const int c2 = tid & 31;
        // columns c = 2 c2, 2 c2 + 1: k1 = 4 quarter + c / 16, k2 = c mod 16 (even, odd)
        const int i2 = c2 >> 3, k2 = 2 * (c2 & 7);
        float2* dst = A.stage + (size_t)frame * MM + 128 * (k2 >> 3) + 8 * (4 * quarter + i2) + (k2 & 7);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int y = (tid >> 5) + 32 * k;
            const float4 pr = *reinterpret_cast<const float4*>(lds + colg::l3(y, 2 * c2));   // 16-byte read
            st2t<STREAM>(dst, (unsigned)y * M, make_float2(pr.x, pr.y), make_float2(pr.z, pr.w));
        }
    }
}

// Item b (of 32 ceil(K / 8)): XCD b mod 8 takes frames [x F, (x + 1) F) in order
// (F = ceil(K / 8)), the four quarters of a frame one after another, so that a
// frame's object window and its neighbours' stay in that XCD's L2 while they
// are reused.  Items past the last frame do nothing.
__device__ __forceinline__ void colg_run(const FrameArgs& A, int item, float2* lds, float* red) {
    float2* twl = lds + colg::QE;   // W^t, t < 256, then the padded table T[j][r] = W^(j r) at 256 + 17 j + r
    for (int t = threadIdx.x; t < 256; t += 1024) twl[t] = A.tw[t];
    for (int t = threadIdx.x; t < colg::TW17; t += 1024) {
        const int j = t / 17, r = t % 17;
        twl[256 + t] = A.tw[(j * r) & 255];
    }
    const int fpx = (A.K + 7) >> 3;
    const int xcd = item & 7, local = item >> 3;
    const int frame = xcd * fpx + (local >> 2), quarter = local & 3;
    if (frame >= A.K) return;
    __syncthreads();
    if (A.stream) colg_item<true>(A, frame, quarter, lds, twl, red);
    else colg_item<false>(A, frame, quarter, lds, twl, red);
}

__global__ void __launch_bounds__(1024) colg_kernel(FrameArgs A) {
    extern __shared__ float2 smem[];
    __shared__ float red[16];
    colg_run(A, blockIdx.x, smem, red);
}

// Batched form: one (scan, item) per workgroup, the single-scan arithmetic and
// item mapping.
__global__ void __launch_bounds__(1024) batch_colg_kernel(const BatchArgs CH, const FrameArgs* __restrict__ D,
                                                          const int2* __restrict__ items, int n) {
    extern __shared__ float2 smem[];
    __shared__ float red[16];
    const int it = blockIdx.x;
    if (it >= n) return;
    const int2 w = items[it];
    const FrameArgs A = batch_args(CH, D, w.x);
    colg_run(A, w.y, smem, red);
}

size_t colg_smem() { return (size_t)(colg::QE + 256 + colg::TW17) * sizeof(float2); }

// Inverse row FFTs of the frame rows that land in object strip s (SH rows),
// multiplied by conj(w) and summed in ascending frame order into the strip,
// then psi_v = D^+ * sum (the 1/m of F* is applied to the sum).  Thread t owns the strip pixels whose column is
// congruent to t modulo 256, so the per-pixel order of the sum is the frame
// order and no two threads touch one pixel.
//
// Lines are taken LINES = 16 at a time (16 / SH frames).  The 256-point
// transforms keep one line in 16 threads (thread t: line t / 16, j = t mod 16)
// and run the two radix-16 Stockham stages in registers: the first stage
// takes its 16 inputs (elements j + 16 r) straight from global memory, one
// LDS exchange feeds the second stage, whose twiddles W^(j r) are fixed per
// thread and held in registers for the whole strip.  Butterflies, twiddles
// and their order are those of the LDS transforms of the row passes; results
// agree with them to rounding (the compiler may fuse multiplies and adds
// differently in the two code shapes).  The transform threads also multiply
// their elements by conj(w) of the line's frame row (read contiguously), so
// the sum only adds.
//
// Lane l of every wave also holds the record (frame, frame row, frame x) of
// line l of a batch for the column-owned sum.  When every frame's columns map
// onto residues without wrap trouble (no periodic wrap, or nx a multiple of
// 256) thread t reads, for each line, the one frame column x with px + x = t
// (mod 256); otherwise (periodic wrap with nx not a multiple of 256) a thread
// walks its own columns.

constexpr int kStripLines = 16;

__device__ __forceinline__ int4 strip_records(const StripArgs& S, int i, int e, int lane) {
    int4 rec = make_int4(-1, 0, 0, 0);
    const int fk = S.SH == 2 ? (lane >> 1) : lane;
    if (lane < kStripLines && i + fk < e) rec = S.lines[(unsigned)i * S.SH + lane];
    return rec;
}

// The record of the line this thread transforms (line = tid / 16).
__device__ __forceinline__ int4 strip_my_record(const StripArgs& S, int i, int e, int line) {
    return strip_records(S, i, e, line);
}

// First radix-16 stage of a 256-point line held as v[r] = element j + 16 r;
// outputs go to LDS elements 16 j + q of the line.
template <int DIR>
__device__ __forceinline__ void line_stage1(float2 (&v)[16], float2* lds, int line, int j) {
    dft<16, DIR>(v);
#pragma unroll
    for (int q = 0; q < 16; ++q) lds[pidx(line * 256 + 16 * j + q)] = v[q];
}

// Second stage for butterfly k = j: inputs k + 16 r from LDS, twiddles
// W^(k r) (conjugated for the inverse), outputs v[q] = element k + 16 q.
template <int DIR>
__device__ __forceinline__ void line_stage2(float2 (&v)[16], const float2* lds, int line, int k,
                                            const float2 (&tw)[15]) {
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = lds[pidx(line * 256 + k + 16 * r)];
#pragma unroll
    for (int r = 1; r < 16; ++r) {
        float2 t = tw[r - 1];
        if constexpr (DIR < 0) t.y = -t.y;
        v[r] = cmul(v[r], t);
    }
    dft<16, DIR>(v);
}

// The next iteration's frames are z = beta w T psi_v + u (carry form, Fourier
// side), and the row pass of that iteration only gathers w T psi_v and
// row-transforms it (the column pass applies beta).  Frame row r of frame f reads object row py + r only, so
// the strip that has just finished psi_v on its rows forms those gathered,
// row-transformed lines itself (the row pass's transform, equal to rounding)
// and writes them where the row pass would: the next iteration starts at the
// column pass.  Lines are independent here, so a wavefront runs through its
// own lines without workgroup barriers.
__device__ void strip_gather_next(const FrameArgs& A, const StripArgs& S, int b, int e, float2* lds,
                                  const float2 (&tw)[15], const float2* psi_rows) {
    constexpr int M = 256, LINES = kStripLines, MM = M * M;
    const int tid = opaque_tid(), line = tid >> 4, j = tid & 15;
    const int SH = S.SH, FPB = LINES / SH, nx = A.nx;
    const int sr = SH == 2 ? (line & 1) : 0;
    float2 ww[16];
    // an absent line (record frame -1) has row 0 and x 0: its values stay in
    // bounds and are never stored
    auto loadw = [&](const int4& rec) {
#pragma unroll
        for (int r = 0; r < 16; ++r) ww[r] = ldc(A.w, (unsigned)rec.y * M + j + 16 * r);
    };
    // Memory requests complete in order among loads, but loads and stores are
    // not ordered with each other, so waiting for a load while stores are in
    // flight waits for the stores too.  The loop therefore issues everything
    // early and consumes it a batch later: records two batches ahead, probe
    // rows one batch ahead, and the transformed lines of a batch wait in their
    // LDS slots until the next batch has used its probe rows, then are stored.
    int4 cur = strip_my_record(S, b, e, line);
    int4 nxt = strip_my_record(S, b + FPB, e, line);
    int4 held = make_int4(-1, 0, 0, 0);   // record of the lines waiting in LDS
    loadw(cur);
    __builtin_amdgcn_s_waitcnt(0);        // nothing in flight when the loop starts
    auto store_held = [&]() {
        if (held.x >= 0) {
            float2* dst = A.stage + (size_t)held.x * MM + (size_t)held.y * M;
#pragma unroll
            for (int q = 0; q < 16; ++q) dst[j + 16 * q] = lds[pidx(line * M + j + 16 * q)];
        }
    };
    for (int i = b; i < e; i += FPB) {
        float2 v[16];
        const float2* prow = psi_rows + sr * nx;
        if (!A.periodic) {
            const float2* p = prow + cur.z + j;
#pragma unroll
            for (int r = 0; r < 16; ++r) v[r] = cmul(ww[r], p[16 * r]);
        } else {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                int gx = cur.z + j + 16 * r;
                if (gx >= nx) gx -= nx;
                v[r] = cmul(ww[r], prow[gx]);
            }
        }
        store_held();
        if (i + FPB < e) loadw(nxt);
        const int4 after = strip_my_record(S, i + 2 * FPB, e, line);
        line_sync();   // the held lines are read before stage 1 rewrites the slots
        line_stage1<1>(v, lds, line, j);
        line_sync();
        line_stage2<1>(v, lds, line, j, tw);
        line_sync();   // stage-2 inputs are read before the results take the slots
#pragma unroll
        for (int q = 0; q < 16; ++q) lds[pidx(line * M + j + 16 * q)] = v[q];
        held = cur;
        cur = nxt;
        nxt = after;
    }
    line_sync();
    store_held();
    __syncthreads();
}

template <bool OCT>
__device__ void strip_merge_item(const FrameArgs& A, const StripArgs& S, int strip, float2* lds, const float2* twl,
                                 float2* acc) {
    constexpr int M = 256, NT = 256, LINES = kStripLines, MM = M * M;
    const int tid = opaque_tid(), lane = tid & 63, line = tid >> 4, j = tid & 15;
    const int SH = S.SH, FPB = LINES / SH, nx = A.nx, ny = A.ny;
    const int y0 = strip * SH;
    for (int i = tid; i < SH * nx; i += NT) acc[i] = make_float2(0.f, 0.f);
    const int b = S.ptr[strip], e = S.ptr[strip + 1];
    const float inv_m = 1.0f / M;
    float2 tw[15];
#pragma unroll
    for (int r = 1; r < 16; ++r) tw[r - 1] = twl[j * r];
    const bool owned = !A.periodic || (nx & (M - 1)) == 0;
    float2 v[16];
    // an absent line (record frame -1, row 0, x 0) reads frame 0 row 0: in
    // bounds, and its transform is never summed
    // element j + 16 r of a line (k1 = j, k2 = r): natural order (stride 16),
    // or octet rows (two runs of eight at 128 (r / 8) + 8 j)
    auto load_line = [&](const int4& rec) {
        if constexpr (OCT) {
            const float2* src = A.stage + (size_t)(rec.x < 0 ? 0 : rec.x) * MM + (size_t)rec.y * M + 8 * j;
#pragma unroll
            for (int r = 0; r < 16; ++r) v[r] = src[128 * (r >> 3) + (r & 7)];
        } else {
            const float2* src = A.stage + (size_t)(rec.x < 0 ? 0 : rec.x) * MM + (size_t)rec.y * M + j;
#pragma unroll
            for (int r = 0; r < 16; ++r) v[r] = src[16 * r];
        }
    };
    // records are fetched two batches ahead, so that the lines of the next
    // batch can be requested at once (no wait for a record load in between)
    int4 mine = strip_my_record(S, b, e, line);
    int4 mine_next = strip_my_record(S, b + FPB, e, line);
    int4 cur = strip_records(S, b, e, lane);
    load_line(mine);
    for (int i = b; i < e; i += FPB) {
        line_stage1<-1>(v, lds, line, j);
        // conj(w) of the line (applied below) is requested before the next
        // batch's lines: memory requests complete in order, so waiting for it
        // then leaves the next batch in flight
        float2 ww[16];
        {
            const float2* wrow = A.w + (unsigned)mine.y * M + j;
#pragma unroll
            for (int q = 0; q < 16; ++q) ww[q] = wrow[16 * q];
        }
        __builtin_amdgcn_sched_barrier(0);       // keeps that order
        // next batch in flight during this one; requested unconditionally (past
        // the last batch the record is absent and frame 0's row 0 is read and
        // not used), so the count of requests in flight does not depend on the
        // branch and the wait for conj(w) stays partial
        load_line(mine_next);
        const int4 mine_after = strip_my_record(S, i + 2 * FPB, e, line);
        const int4 next = strip_records(S, i + FPB, e, lane);
        line_sync();
        {
            // a thread reads and writes the same 16 elements of its line here
            float2 t[16];
            line_stage2<-1>(t, lds, line, j, tw);
#pragma unroll
            for (int q = 0; q < 16; ++q) lds[pidx(line * M + j + 16 * q)] = cconjmul(ww[q], t[q]);
        }
        __syncthreads();
        if (owned) {
#pragma unroll
            for (int l = 0; l < LINES; ++l) {
                if (__builtin_amdgcn_readlane(cur.x, l) < 0) continue;
                const int px = __builtin_amdgcn_readlane(cur.z, l);
                const int x = (tid - px) & (M - 1);
                int gx = px + x;
                if (gx >= nx) gx -= nx;
                float2& a = acc[(SH == 2 ? (l & 1) : 0) * nx + gx];
                a = cadd(a, lds[pidx(l * M + x)]);
            }
        } else {
            for (int l = 0; l < LINES; ++l) {
                if (__builtin_amdgcn_readlane(cur.x, l) < 0) continue;
                const int px = __builtin_amdgcn_readlane(cur.z, l);
                const int sr = SH == 2 ? (l & 1) : 0;
                for (int gx = tid; gx < nx; gx += NT) {
                    int x = gx - px;
                    if (x < 0) x += nx;
                    if ((unsigned)x >= (unsigned)M) continue;
                    float2& a = acc[sr * nx + gx];
                    a = cadd(a, lds[pidx(l * M + x)]);
                }
            }
        }
        __syncthreads();
        mine = mine_next;
        mine_next = mine_after;
        cur = next;
    }
    for (int sr = 0; sr < SH; ++sr) {
        const int y = y0 + sr;
        if (y >= ny) break;
        for (int gx = tid; gx < nx; gx += NT) {
            const unsigned o = (unsigned)y * (unsigned)nx + gx;
            const float2 pv = cscale(acc[sr * nx + gx], S.Dinv[o] * inv_m);   // 1/m of F* applied once
            S.out[o] = pv;
            acc[sr * nx + gx] = pv;
        }
    }
    __syncthreads();
    if (S.next_gather) strip_gather_next(A, S, b, e, lds, tw, acc);
}

// The last workgroup (the lightest strip in the heaviest-first order) also
// forms eps_a when E.partials is set.
__global__ void __launch_bounds__(256, 3) strip_merge_kernel(FrameArgs A, StripArgs S, EpsArgs E) {
    extern __shared__ float2 smem[];
    float2* lds = smem;
    float2* twl = smem + pidx(16 * 256);
    float2* acc = twl + 256;
    for (int t = threadIdx.x; t < 256; t += 256) twl[t] = A.tw[t];
    __syncthreads();
    const int slot = S.strip0 + blockIdx.x;
    const int strip = S.order ? S.order[slot] : slot;
    if (S.octet_rows) strip_merge_item<true>(A, S, strip, lds, twl, acc);
    else strip_merge_item<false>(A, S, strip, lds, twl, acc);
    if (E.partials && blockIdx.x == gridDim.x - 1) eps_epilogue(E);
}

// Batched form: phase 0 gather + row FFTs, 1 column pass with the carry,
// 2 strip merge; items (scan, local item), identical arithmetic.  One item
// per workgroup (grid = items) and the scans' argument blocks by value, as in
// the single-scan launches: a persistent loop over items and argument blocks
// read from memory each kept about 20 more registers live (a wave per SIMD).
template <int PHASE>
__global__ void __launch_bounds__(256, PHASE == 2 ? 3 : 1) batch_carry_kernel(const BatchArgs CH,
                                                          const FrameArgs* __restrict__ D,
                                                          const int2* __restrict__ items, int n) {
    using C = MP<256, 256>;
    extern __shared__ float2 smem[];
    __shared__ float red[4];
    float2* lds = smem;
    float2* twl = smem + (PHASE == 2 ? pidx(16 * 256) : C::LDS);
    const int it = blockIdx.x;
    if (it >= n) return;
    const int2 w = items[it];
    const FrameArgs A = batch_args(CH, D, w.x);
    for (int t = threadIdx.x; t < 256; t += 256) twl[t] = A.tw[t];
    __syncthreads();
    if constexpr (PHASE == 0) {
        if (A.gather) mp_row_fwd_item<256, FM_GATHER, 256>(A, w.y, lds, twl);
    } else if constexpr (PHASE == 1) {
        const float r = A.stream ? col_carry_item<true>(A, w.y, lds, twl) : col_carry_item<false>(A, w.y, lds, twl);
        const float s = block_sum(r, red);
        if (threadIdx.x == 0) A.resid[w.y] = s;
    } else {
        const StripArgs& S = CH.s[w.x - CH.base];
        if (S.octet_rows) strip_merge_item<true>(A, S, w.y, lds, twl, twl + 256);
        else strip_merge_item<false>(A, S, w.y, lds, twl, twl + 256);
    }
}

size_t carry_phase_smem() { return MP<256, 256>::SMEM; }

// Allows `f` all of a CU's 160 KiB of LDS that its static shared arrays leave
// for dynamic shared memory (the runtime rejects a larger limit).
static hipError_t allow_full_lds(const void* f) {
    hipFuncAttributes fa{};
    hipError_t e = hipFuncGetAttributes(&fa, f);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(160 * 1024 - fa.sharedSizeBytes));
}

hipError_t batch_carry_prepare(int phase, size_t smem, int* blocks_per_cu) {
    hipError_t e = hipSuccess;
    int nb = 0;
    if (phase == 0) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_carry_kernel<0>, 256, smem);
    else if (phase == 1) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_carry_kernel<1>, 256, smem);
    else {
        e = allow_full_lds((const void*)batch_carry_kernel<2>);
        if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_carry_kernel<2>, 256, smem);
    }
    *blocks_per_cu = nb > 0 ? nb : 1;
    return e;
}

hipError_t launch_batch_carry(int phase, const BatchArgs& C, const FrameArgs* D, const int2* items, int n,
                              size_t smem, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (phase == 0) hipLaunchKernelGGL(batch_carry_kernel<0>, dim3(n), dim3(256), smem, s, C, D, items, n);
    else if (phase == 1) hipLaunchKernelGGL(batch_carry_kernel<1>, dim3(n), dim3(256), smem, s, C, D, items, n);
    else hipLaunchKernelGGL(batch_carry_kernel<2>, dim3(n), dim3(256), smem, s, C, D, items, n);
    return hipGetLastError();
}

// Carry <-> space: u = F* U (column pass then row pass) and U = F u.
// Column transforms of the carry conversions; `layout` is that of the carry
// (CL_CB256 or CL_Q256).
__global__ void __launch_bounds__(256) carry_cols_kernel(FrameArgs A, int dir, int layout) {
    using C = MP<256, 256>;
    constexpr int M = 256, NT = C::NT, NP = C::NP, CB = C::CB, MM = M * M, NCB = C::NCB;
    extern __shared__ float2 smem[];
    float2* lds = smem;
    float2* twl = smem + C::LDS;
    for (int t = threadIdx.x; t < M; t += NT) twl[t] = A.tw[t];
    const int items = A.K * NCB;
    for (int it = blockIdx.x; it < items; it += gridDim.x) {
        const int tid = opaque_tid();
        const int frame = it / NCB, cb = it % NCB;
        const size_t fb = (size_t)frame * MM, blk = fb + (size_t)cb * M * CB;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const int e0 = 2 * (tid + NT * k);
            const int y = e0 / CB, c = e0 % CB;
            float2 a0, a1;
            if (dir < 0 && layout == CL_Q256) {                           // carry, q256
                a0 = A.in[fb + q256(y, cb * CB + c)];
                a1 = A.in[fb + q256(y, cb * CB + c + 1)];
            } else if (dir < 0) {
                ld2(A.in + blk, e0, a0, a1);                              // carry block
            } else {
                ld2(A.stage + fb, y * M + cb * CB + c, a0, a1);           // row-transformed frame
            }
            lds[pidx(e0)] = a0;
            lds[pidx(e0 + 1)] = a1;
        }
        __syncthreads();
        NoPost none;
        if (dir < 0) fft_1d<M, -1, NT, CB, ColLayCB<CB>>(lds, twl, none);
        else fft_1d<M, 1, NT, CB, ColLayCB<CB>>(lds, twl, none);
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const int e0 = 2 * (tid + NT * k);
            const int y = e0 / CB, c = e0 % CB;
            const float2 v0 = lds[pidx(e0)], v1 = lds[pidx(e0 + 1)];
            if (dir < 0) {
                st2(A.stage + fb, y * M + cb * CB + c, v0, v1);
            } else if (layout == CL_Q256) {
                A.out[fb + q256(y, cb * CB + c)] = cscale(v0, 1.0f / M);
                A.out[fb + q256(y, cb * CB + c + 1)] = cscale(v1, 1.0f / M);
            } else {
                st2(A.out + blk, e0, cscale(v0, 1.0f / M), cscale(v1, 1.0f / M));
            }
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) carry_rows_inv_kernel(FrameArgs A) {
    using C = MP<256, 256>;
    constexpr int M = 256, NT = C::NT, NP = C::NP, RB = C::RB, MM = M * M, NRB = C::NRB;
    extern __shared__ float2 smem[];
    float2* lds = smem;
    float2* twl = smem + C::LDS;
    for (int t = threadIdx.x; t < M; t += NT) twl[t] = A.tw[t];
    const int items = A.K * NRB;
    for (int it = blockIdx.x; it < items; it += gridDim.x) {
        const int tid = opaque_tid();
        const int frame = it / NRB, rb = it % NRB;
        const size_t fb = (size_t)frame * MM;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const int e0 = 2 * (tid + NT * k);
            float2 a0, a1;
            ld2(A.stage + fb, rb * RB * M + e0, a0, a1);
            lds[pidx(e0)] = a0;
            lds[pidx(e0 + 1)] = a1;
        }
        __syncthreads();
        NoPost none;
        fft_1d<M, -1, NT, RB, RowLay<M>>(lds, twl, none);
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const int e0 = 2 * (tid + NT * k);
            st2(A.out + fb, rb * RB * M + e0, cscale(lds[pidx(e0)], 1.0f / M), cscale(lds[pidx(e0 + 1)], 1.0f / M));
        }
        __syncthreads();
    }
}

size_t strip_smem_bytes(int SH, int nx) {
    return (size_t)(pidx(16 * 256) + 256 + SH * nx) * sizeof(float2);
}

hipError_t launch_row_gather_256(const FrameArgs& A, hipStream_t s, const Timer* tp) {
    const Timer& t = tp ? *tp : kNoTimer;
    using C = MP<256, 256>;
    t.begin(TC_FRAME, s);
    hipLaunchKernelGGL((mp_row_fwd<256, FM_GATHER, 256>), dim3(A.K * C::NRB), dim3(256), C::SMEM, s, A);
    t.end(TC_FRAME, s);
    return hipGetLastError();
}

hipError_t launch_col_carry_256(const FrameArgs& A, hipStream_t s, const Timer* tp) {
    const Timer& t = tp ? *tp : kNoTimer;
    using C = MP<256, 256>;
    if (A.K <= 0) return hipSuccess;
    t.begin(TC_COLS, s);
    if (A.stream) hipLaunchKernelGGL(col_carry_kernel<true>, dim3(A.K * C::NCB), dim3(256), C::SMEM, s, A);
    else hipLaunchKernelGGL(col_carry_kernel<false>, dim3(A.K * C::NCB), dim3(256), C::SMEM, s, A);
    t.end(TC_COLS, s);
    return hipGetLastError();
}

int colg_items(int K) { return 32 * ((K + 7) / 8); }

hipError_t batch_colg_prepare() {
    return hipFuncSetAttribute((const void*)batch_colg_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)colg_smem());
}

hipError_t launch_batch_colg(const BatchArgs& C, const FrameArgs* D, const int2* items, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(batch_colg_kernel, dim3(n), dim3(1024), colg_smem(), s, C, D, items, n);
    return hipGetLastError();
}

hipError_t launch_colg_256(const FrameArgs& A, hipStream_t s, const Timer* tp) {
    const Timer& t = tp ? *tp : kNoTimer;
    if (A.K <= 0) return hipSuccess;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)colg_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)colg_smem());
        if (e != hipSuccess) return e;
        attr = true;
    }
    t.begin(TC_COLS, s);
    hipLaunchKernelGGL(colg_kernel, dim3(colg_items(A.K)), dim3(1024), colg_smem(), s, A);
    t.end(TC_COLS, s);
    return hipGetLastError();
}

hipError_t launch_strip_256(const FrameArgs& A, const StripArgs& S, int s0, int s1, hipStream_t s,
                            const Timer* tp, const EpsArgs* eps) {
    const Timer& t = tp ? *tp : kNoTimer;
    if (s1 <= s0) return hipSuccess;
    static bool attr = false;
    if (!attr) {
        hipError_t e = allow_full_lds((const void*)strip_merge_kernel);
        if (e != hipSuccess) return e;
        attr = true;
    }
    StripArgs S2 = S;
    S2.strip0 = s0;
    t.begin(TC_MERGE, s);
    const EpsArgs E = eps ? *eps : EpsArgs{};
    hipLaunchKernelGGL(strip_merge_kernel, dim3(s1 - s0), dim3(256), strip_smem_bytes(S.SH, A.nx), s, A, S2, E);
    t.end(TC_MERGE, s);
    return hipGetLastError();
}

// u = F* U for the K frames of A.in (carry blocks) into A.out (natural layout)
hipError_t launch_carry_to_space(const FrameArgs& A, hipStream_t s, int layout) {
    using C = MP<256, 256>;
    hipLaunchKernelGGL(carry_cols_kernel, dim3(A.K * C::NCB), dim3(256), C::SMEM, s, A, -1, layout);
    hipLaunchKernelGGL(carry_rows_inv_kernel, dim3(A.K * C::NRB), dim3(256), C::SMEM, s, A);
    return hipGetLastError();
}

// U = F u for the K frames of A.in (natural layout) into A.out (carry blocks)
hipError_t launch_space_to_carry(const FrameArgs& A, hipStream_t s, int layout) {
    using C = MP<256, 256>;
    hipLaunchKernelGGL((mp_row_fwd<256, FM_F, 256>), dim3(A.K * C::NRB), dim3(256), C::SMEM, s, A);
    hipLaunchKernelGGL(carry_cols_kernel, dim3(A.K * C::NCB), dim3(256), C::SMEM, s, A, 1, layout);
    return hipGetLastError();
}

}  // namespace sharp
