// Private: the plan object shared by the C ABI implementation files.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <utility>
#include <vector>

#include "../../include/sharp.h"
#include "sharp_internal.hpp"

namespace sharp {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

inline bool supported_m(int m) { return m == 16 || m == 32 || m == 64 || m == 128 || m == 256; }

struct Offsets {
    size_t tw, pos, tile_ptr, tile_frames, a, a_t, u, v, stage, psi_v, psi_l, tmp_obj, D, Dinv;
    size_t w_cur, w_gat, tmp_w, tmp_w2, pcons, mpart, pnum, pden, gwpart, resid, hist, scal, flag, sptr, sln, sord, total;
};

}  // namespace sharp

struct sharp_plan_s {
    int nx = 0, ny = 0, m = 0, K = 0;
    sharp_options opt{};
    std::vector<int32_t> pos;
    int T = 32, tiles_x = 0, tiles_y = 0, ntiles = 0, split = 1, grad_groups = 0, probe_chunks = 1;
    int frame_launch = 1;     // 1 = carry in frame space; 2 = carry in the Fourier domain (m = 128: one
                              // frame kernel + tile merge; m = 256: column pass + strip pass); 3 (m = 256):
                              // Fourier carry, column pass forming its own row transform + strip pass
    int SH = 0, nstrips = 0;  // strip merge: object rows per strip (0 = form unavailable)
    std::vector<int32_t> strip_ptr, strip_lines;  // strip_lines: 4 ints per (entry, strip row)
    std::vector<int32_t> strip_order;             // strips by descending frame-row count (launch order)
    int fft_block = 256;      // m = 256, three launches: threads per pass workgroup
    std::vector<int32_t> tile_ptr, tile_frames;
    sharp::Offsets off{};
    size_t resid_cap = 0, gw_slots = 0;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    unsigned long long ws_generation = 0;  // bumped by every sharp_set_workspace (batches check it)
    hipStream_t stream = nullptr;
    bool has_ws = false, has_data = false, has_probe = false, has_object = false;
    float g = 1.f;
    long long iter = 0, hist_count = 0;
    bool gat_stale = false, last_probe_updated = false;
    int pcons_kind = 0;         // probe constraint: 0 none, 1 Fourier mask, 2 Fourier amplitudes
    bool stage_gather = false;  // carry form: stage holds the next iteration's gathered, row-transformed frames

    // kernel timing (diagnostics): pending (start, stop) event pairs per category
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pairs[sharp::TC_N];
    std::vector<hipEvent_t> ev_open[sharp::TC_N];
    sharp::Timer timer{};
    ~sharp_plan_s() {
        for (auto e : ev_pool) (void)hipEventDestroy(e);
        for (int c = 0; c < sharp::TC_N; ++c) {
            for (auto& pr : ev_pairs[c]) {
                (void)hipEventDestroy(pr.first);
                (void)hipEventDestroy(pr.second);
            }
            for (auto e : ev_open[c]) (void)hipEventDestroy(e);
        }
    }
    const sharp::Timer* tm() const { return timing ? &timer : nullptr; }

    template <class T> T* at(size_t o) const { return reinterpret_cast<T*>(ws + o); }
    bool carry_form() const { return (m == 128 && frame_launch == 2) || (m == 256 && frame_launch >= 2); }
    bool strip_form() const { return m == 256 && frame_launch >= 2; }   // merge fused into the strip pass
    bool colg_form() const { return m == 256 && frame_launch == 3; }    // column pass forms its own row transform
    int carry_layout() const { return colg_form() ? sharp::CL_Q256 : sharp::CL_CB256; }
    // frame arrays (K m^2 complex values) larger than the GPU's last-level
    // cache (256 MiB on this part) are read and written with streaming
    // accesses; smaller ones stay cacheable, since a pass often finds them there
    static constexpr size_t kLastLevelCache = size_t(256) << 20;
    // frame chunks of the probe-gradient pass of the m = 128 Fourier-carry form
    // frame chunks of the probe-gradient partial sums (m = 128 Fourier-carry form): at 1024 frames
    // 32 chunks took 0.147 ms per gradient call against 0.149 (64), 0.152 (128), 0.153 (16), 0.161 (256)
    int grad_chunks() const { return K < 32 ? K : 32; }
    bool streams() const { return (size_t)K * m * m * sizeof(float2) > kLastLevelCache; }
    size_t frame_elems() const { return (size_t)K * m * m; }
    size_t obj_elems() const { return (size_t)nx * ny; }
};

namespace sharp {
// argument blocks of a plan's kernels (sharp_api.cpp)
FrameArgs frame_args(const sharp_plan_s& p);
MergeArgs merge_args(const sharp_plan_s& p);
// sharp_apply with its scratch segments taken from `scratch` (device memory of
// at least apply_scratch(p, op).total bytes, 256-byte aligned) instead of the
// workspace when it is not null
struct ApplyScratch {
    size_t stage, resid, tmp_obj, mpart, total;
};
ApplyScratch apply_scratch(const sharp_plan_s& p, int op);
// host-side argument and readiness checks of sharp_apply (no device work)
int apply_check(const sharp_plan_s& p, int op, const void* d_in, const void* d_out);
int apply_into(sharp_plan_s& p, int op, const void* d_in, void* d_out, char* scratch);
// number of per-block residual partials an iteration's frame launch writes
int resid_blocks(const sharp_plan_s& p);
// the same for the default launch shape (used by batched execution)
int resid_blocks_default(const sharp_plan_s& p);
}  // namespace sharp
