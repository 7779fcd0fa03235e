// Internal interfaces between the host plan code (sharp_api.cpp) and the
// kernels (kernels_frame.hip, kernels_merge.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace sharp {

constexpr int kHistCap = 4096;  // eps_a history ring (entries)

// Frame-kernel modes
enum FrameMode : int {
    FM_RAAR = 0,  // z = u + g w_g T psi_v; P_a; u' = b z + (1-2b) y; v' = conj(w)(2y - z)
    FM_PA = 1,    // in -> P_a in
    FM_GRAD = 2,  // z = w T psi; r = 2 (z - P_a z); v = conj(w) r; gw partial += conj(T psi) r
    FM_SIM = 3,   // I = |F w T psi|^2
    FM_F = 4,     // in -> F in
    FM_FINV = 5,  // in -> F* in
    FM_Q = 6,     // psi -> w T psi
    FM_GATHER = 7,  // z = g w_g T psi_v (Fourier-carry RAAR row pass, m = 256)
};

// Layouts of the m = 256 Fourier-domain carry (and of the amplitudes read with it)
enum CarryLayout : int { CL_CB256 = 0, CL_Q256 = 1 };

// For m = 256 the amplitudes (and the Fourier-domain carry) are stored
// column-block-major: element (y, x) of a frame at ((x / 16) * 256 + y) * 16
// + x % 16, so that a column-pass workgroup (16 columns) reads one
// contiguous 32 KiB block.
__host__ __device__ __forceinline__ unsigned cb256(unsigned y, unsigned x) {
    return ((x >> 4) << 12) + (y << 4) + (x & 15u);
}

// Layout of the Fourier-domain carry and the second amplitude copy of the
// m = 256 form whose column pass forms its own row transform: the frame's
// columns kx = k1 + 16 k2 fall into four quarters by k1 / 4 (one column-pass
// workgroup each, 64 columns); inside a quarter, column c = 16 (k1 mod 4) + k2
// holds its 256 rows ky = j + 16 r at c * 256 + 32 (r / 2) + 2 j + r mod 2:
// the thread that owns rows j + 16 r of a column reads pairs (r, r + 1), and
// the 16 threads of the column read 16 such pairs side by side.
__host__ __device__ __forceinline__ unsigned q256(unsigned ky, unsigned kx) {
    const unsigned k1 = kx & 15u, k2 = kx >> 4, j = ky & 15u, r = ky >> 4;
    return ((k1 >> 2) << 14) + ((((k1 & 3u) << 4) + k2) << 8) + ((r >> 1) << 5) + (j << 1) + (r & 1u);
}

// Merge-kernel kinds
enum MergeKind : int {
    MK_V = 0,     // psi_v = Dinv sum v
    MK_VU = 1,    // psi_v = Dinv sum v;  psi_l = [Dinv>0] (Dinv sum conj(w) u + g psi_v)
    MK_U = 2,     // out = [Dinv>0] (Dinv sum conj(w) u + g psi_v)
    MK_RAW = 3,   // out = sum v
    MK_RAWW = 4,  // out = sum conj(w) u
    MK_OBJ = 5,   // out = Dinv sum conj(w) u
    MK_DENS = 6,  // D = sum |w|^2, Dinv = D > eps ? 1/D : 0
};

struct FrameArgs {
    int K, M, nx, ny, periodic;
    const int* __restrict__ pos;        // [K][2] (y, x)
    const float2* __restrict__ tw;      // [M] e^{2 pi i t / M}
    const float* __restrict__ a;        // [K][M][M] amplitudes
    const float2* __restrict__ w_g;     // gather probe
    const float* __restrict__ at;       // m = 128 carry form: amplitudes, per frame transposed
    const float2* __restrict__ w;       // current probe
    const float2* __restrict__ psi;     // gathered object (psi_v, or psi for GRAD/SIM/Q)
    const float2* __restrict__ in;      // input frames (PA/F/FINV)
    float2* __restrict__ u;             // carry (RAAR, in/out)
    float2* __restrict__ v;             // merge input (RAAR, GRAD)
    float2* __restrict__ out;           // output frames (PA/F/FINV/Q)
    float* __restrict__ out_f;          // output intensities (SIM)
    float2* __restrict__ stage;         // multi-pass intermediate [K][M][M]
    float* __restrict__ resid;          // per-block residual partials
    float2* __restrict__ gw_part;       // per-block probe-gradient partials
    float g, beta;
    int gather;                         // batched m = 256 carry form: run the gather pass
    int stream;                         // frame arrays exceed the last-level cache: streaming accesses
};

struct MergeArgs {
    int M, nx, ny, periodic, T, tiles_x, split;
    const int* __restrict__ tile_ptr;
    const int* __restrict__ tile_frames;
    const int* __restrict__ pos;
    const float2* __restrict__ v;       // frames (pre-multiplied by conj(w))
    const float2* __restrict__ u;       // frames multiplied by conj(w) on the fly
    const float2* __restrict__ w;
    const float* __restrict__ Dinv;
    const float2* __restrict__ psi_v_in;   // MK_U: g psi_v term
    float2* __restrict__ out;           // psi_v / out
    float2* __restrict__ out2;          // psi_l (MK_VU)
    float* __restrict__ D_out;          // MK_DENS
    float* __restrict__ Dinv_out;       // MK_DENS
    float4* __restrict__ part;          // split partials [tiles][split][T*T] (x2 for VU)
    float g, eps_D;
};

// Optional per-launch timing hook (HIP events recorded on the launch stream).
enum TimerCat : int { TC_FRAME = 0, TC_COLS = 1, TC_FRAME_OUT = 2, TC_MERGE = 3, TC_REDUCE = 4, TC_PROBE = 5,
                      TC_COPY = 6, TC_N = 8 };
struct Timer {
    void* ctx = nullptr;
    void (*mark)(void* ctx, int cat, int begin, hipStream_t s) = nullptr;  // s = nullptr: the plan's stream
    void begin(int c, hipStream_t s = nullptr) const { if (mark) mark(ctx, c, 1, s); }
    void end(int c, hipStream_t s = nullptr) const { if (mark) mark(ctx, c, 0, s); }
};

// launchers (kernels_frame.hip)
hipError_t launch_frame(int mode, const FrameArgs& a, int grid_hint, hipStream_t s, int* blocks_used,
                        const Timer* t = nullptr);
int frame_partial_slots(int M, int mode, int blocks);  // gw partial slots per launch
int fg_groups(int M);                                   // frames per frame-kernel workgroup, m <= 128
// device read-rate reference (kernels_merge.hip); sink holds kReadRefBlocks floats
constexpr int kReadRefBlocks = 2048;
hipError_t launch_read_reference(const void* src, size_t bytes, float* sink, hipStream_t s);
hipError_t launch_probe_partial(int M, int K, const int* pos, int nx, int ny, int periodic,
                                const float2* u, const float2* w, const float2* psi_v,
                                const float2* psi_l, float beta, int chunks, float2* num, float* den,
                                hipStream_t s);
hipError_t launch_probe_finish(int M, int chunks, const float2* num, const float* den, float2* w_gat,
                               float2* w_cur, hipStream_t s);
hipError_t launch_gw_finish(int M, int slots, const float2* part, float2* gw, hipStream_t s);
// sum over frames of conj(T psi) r per frame pixel, in `chunks` frame-chunk partials (part: [chunks][M*M])
hipError_t launch_grad_probe_partial(int M, int K, const int* pos, int nx, int ny, int periodic, const float2* r,
                                     const float2* psi, int chunks, float2* part, hipStream_t s);

// launchers (kernels_merge.hip)
// eps_a of an iteration (Eq. (amplitudemetric)) formed by one workgroup of a
// merge launch instead of a launch of its own: the fixed-order sum of the
// residual partials (the order of the separate reduction, bit for bit),
// sqrt(sum / ||a||^2) into hist[idx] -- or, without norm_a2, the sum itself
// (the gradient's loss) -- and flag[0] = 1 when not finite
struct EpsArgs {
    const float* __restrict__ partials;   // nullptr: no eps
    int n;
    const float* __restrict__ norm_a2;    // nullptr: write the sum
    float* __restrict__ hist;
    int idx;
    int* __restrict__ flag;
};
hipError_t launch_merge(int kind, const MergeArgs& a, int tiles, hipStream_t s, const EpsArgs* eps = nullptr);
// a2: optional second amplitude copy, 128 x 128 frames transposed (a2_q256 = 0)
// or 256 x 256 frames in the q256 layout (a2_q256 = 1)
hipError_t launch_set_data(const float* I, float* a, size_t n, float* partials, int* flag,
                           hipStream_t s, int* blocks_used, int blocked256, float* a2, int a2_q256);
hipError_t launch_reduce(const float* partials, int n, float* out, hipStream_t s);
hipError_t launch_loss(const float* partials, int n, float* out, int* flag, hipStream_t s);
hipError_t launch_mean_amp(const float* a, int K, int M, float2* out, hipStream_t s);
hipError_t launch_roll_probe(const float2* src, int M, float2* w_cur, float2* w_gat, hipStream_t s);
hipError_t launch_fill(void* p, size_t bytes, hipStream_t s);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);

// m = 256 RAAR frame phase in three launches with a chosen pass block size
hipError_t launch_raar_mp256(const FrameArgs& A, int threads, hipStream_t s, const Timer* t, int* blocks_used);
// m = 256 RAAR with the carry in the Fourier domain and the merge fused into
// the last row pass (kernels_frame.hip).  Strip merge arguments:
struct StripArgs {
    const int* __restrict__ ptr;     // [nstrips + 1] entries (frames) per strip
    const int4* __restrict__ lines;  // [entries * SH]: (frame, frame row, frame x, 0) of the frame
                                     // row landing on each strip row, frame -1 when none; frames
                                     // ascending within a strip
    const float* __restrict__ Dinv;
    float2* __restrict__ out;        // psi_v
    int SH;                          // object rows per strip
    int next_gather;                 // also form the next iteration's gathered, row-transformed
                                     // frame rows (w * T psi_v) in the stage buffer
    int strip0;                      // first launch slot (workgroup b takes slot strip0 + b)
    int octet_rows;                  // stage rows hold element k1 + 16 k2 at 128 (k2 / 8) + 8 k1 + k2 mod 8
                                     // (else natural order)
    const int* __restrict__ order;   // [nstrips] strip of each launch slot, the strips with the most frame
                                     // rows first (nullptr: slot = strip)
};
size_t carry_phase_smem();
// m = 128 with the RAAR carry kept in the Fourier domain
__host__ __device__ int fc128_groups(int K);
hipError_t launch_fc128(const FrameArgs& A, hipStream_t s, const Timer* t, int* blocks_used);
// to_space: A.out = F* A.in (A.in transposed carry); else A.out (transposed) = F A.in
hipError_t launch_fc128_convert(const FrameArgs& A, int to_space, hipStream_t s);
// probe constraints of the probe update: Fourier-domain mask / amplitudes, centre of mass
hipError_t launch_probe_fourier(float2* W, const float* vals, int M, int kind, hipStream_t s);
hipError_t launch_probe_center(float2* w, float2* tmp, int M, hipStream_t s);
// amplitude-loss gradient at m = 128 (carry-form plans, which hold the transposed amplitudes)
hipError_t launch_fc128_grad(const FrameArgs& A, int grid, hipStream_t s, const Timer* t, int* blocks_used);
hipError_t batch_fc128_prepare(int* blocks_per_cu);
hipError_t batch_carry_prepare(int phase, size_t smem, int* blocks_per_cu);
// The batch kernels take the argument blocks of up to kBatchChunk scans by
// value (kernel arguments): pointers read from there are known to address
// global memory (read from device memory they are not, and every access
// becomes a flat one), which keeps the kernels at the registers, occupancy and
// instruction forms of the single-scan launches.  Fields that change between
// iterations on the device (g, beta, gather) are still read from D.
constexpr int kBatchChunk = 12;
struct BatchArgs {
    FrameArgs a[kBatchChunk];   // scans base .. base + kBatchChunk - 1
    StripArgs s[kBatchChunk];
    int base;
};
static_assert(sizeof(BatchArgs) <= 4000, "kernel arguments are limited to 4 KiB");
struct BatchMergeArgs {
    MergeArgs a[kBatchChunk];   // scans base .. base + kBatchChunk - 1
    int base;
};
static_assert(sizeof(BatchMergeArgs) <= 4000, "kernel arguments are limited to 4 KiB");
// items: (scan, item) of scans base .. base + kBatchChunk - 1, one workgroup each
hipError_t launch_batch_carry(int phase, const BatchArgs& C, const FrameArgs* D, const int2* items, int n,
                              size_t smem, hipStream_t s);
// items: (scan, frame group slot) of the chunk's scans, one workgroup each
hipError_t launch_batch_fc128(const BatchArgs& C, const FrameArgs* D, const int2* items, int n, hipStream_t s);
// items: (scan, item < colg_items(K)) of the chunk's form-3 scans, one workgroup each
hipError_t batch_colg_prepare();
hipError_t launch_batch_colg(const BatchArgs& C, const FrameArgs* D, const int2* items, int n, hipStream_t s);
size_t strip_smem_bytes(int SH, int nx);
// m = 256 Fourier-carry form: gather + row transforms (first iteration only),
// column pass over the K frames of A, strip pass over strips [s0, s1)
hipError_t launch_row_gather_256(const FrameArgs& A, hipStream_t s, const Timer* t);
hipError_t launch_col_carry_256(const FrameArgs& A, hipStream_t s, const Timer* t);
hipError_t launch_strip_256(const FrameArgs& A, const StripArgs& S, int s0, int s1, hipStream_t s, const Timer* t,
                            const EpsArgs* eps = nullptr);
hipError_t launch_carry_to_space(const FrameArgs& A, hipStream_t s, int layout = CL_CB256);
hipError_t launch_space_to_carry(const FrameArgs& A, hipStream_t s, int layout = CL_CB256);
// m = 256, form 3: column pass that forms its own gathered row transform
// (quarter-frame workgroups, carry and amplitudes in the q256 layout), writing
// the merge input in octet rows to the stage buffer; one residual partial
// per (frame, quarter), at 4 frame + quarter
hipError_t launch_colg_256(const FrameArgs& A, hipStream_t s, const Timer* t);
int colg_items(int K);   // workgroups (items) of one launch over K frames

// batched execution (kernels_frame.hip, kernels_merge.hip)
constexpr int kMaxBatch = 256;
struct EpsDesc {
    const float* partials;
    int n;
    int hist_idx;
    const float* norm_a2;
    float* hist;
    int* flag;
};
struct BatchBegin {
    int n;
    float g[kMaxBatch];
    int hist[kMaxBatch];
    int gather[kMaxBatch];  // m = 256 carry form: stage does not hold the first iteration's gather
};
hipError_t batch_frame_prepare(int M, int phase, int* blocks_per_cu);
// items: (scan, frame group or pass block) of the chunk's scans, one workgroup each
hipError_t launch_batch_frame(int M, int phase, const BatchArgs& C, const FrameArgs* D, const int2* items, int n,
                              hipStream_t s);
// items (scan, tile, chunk) and finish items (scan, tile) of the chunk's scans, one workgroup each
hipError_t launch_batch_merge(int T, const BatchMergeArgs& C, const int4* items, int n, const int2* fin, int nfin,
                              hipStream_t s);
hipError_t launch_batch_eps(EpsDesc* E, FrameArgs* D, int nscans, float beta, hipStream_t s);
hipError_t launch_batch_begin(FrameArgs* D, EpsDesc* E, const BatchBegin& b, float beta, hipStream_t s);

}  // namespace sharp
