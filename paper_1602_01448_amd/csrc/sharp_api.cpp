// Host side of the C ABI declared in include/sharp.h: argument validation,
// the tile -> frame incidence lists of the overlap merge (the per-block
// contributing-frame lists of Sec. "Computational Methodology"), workspace
// layout, and the launch sequences of one RAAR iteration (algorithm box,
// steps 5-7).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/sharp.h"
#include "plan_impl.hpp"
#include "sharp_internal.hpp"

using namespace sharp;

static void timer_mark(void* ctx, int cat, int begin, hipStream_t s) {
    sharp_plan_s& p = *static_cast<sharp_plan_s*>(ctx);
    hipEvent_t e = nullptr;
    if (!p.ev_pool.empty()) {
        e = p.ev_pool.back();
        p.ev_pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
        return;
    }
    if (hipEventRecord(e, s ? s : p.stream) != hipSuccess) {
        p.ev_pool.push_back(e);
        return;
    }
    if (begin) {
        p.ev_open[cat].push_back(e);
    } else if (!p.ev_open[cat].empty()) {
        p.ev_pairs[cat].emplace_back(p.ev_open[cat].back(), e);
        p.ev_open[cat].pop_back();
    } else {
        p.ev_pool.push_back(e);
    }
}

static_assert(sharp::kReadRefBlocks == SHARP_READ_REFERENCE_SINK, "read-reference sink size");

extern "C" int sharp_read_reference(const void* d_src, size_t bytes, float* d_sink, void* stream) {
    if (!d_src || !d_sink || bytes == 0 || bytes % 16 || reinterpret_cast<uintptr_t>(d_src) % 16)
        return SHARP_ERR_INVALID_ARG;
    return sharp::launch_read_reference(d_src, bytes, d_sink, static_cast<hipStream_t>(stream)) == hipSuccess
               ? SHARP_OK
               : SHARP_ERR_HIP;
}

extern "C" const char* sharp_status_string(int s) {
    switch (s) {
        case SHARP_OK: return "ok";
        case SHARP_ERR_INVALID_ARG: return "invalid argument";
        case SHARP_ERR_UNSUPPORTED_SIZE: return "unsupported size";
        case SHARP_ERR_POSITION_OUT_OF_RANGE: return "frame position out of range";
        case SHARP_ERR_NOT_READY: return "not ready (workspace, data, probe or object missing)";
        case SHARP_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
        case SHARP_ERR_NONFINITE: return "non-finite value in data or iterate";
        case SHARP_ERR_HIP: return "HIP runtime error";
        case SHARP_ERR_HOST_ALLOC: return "host allocation failed";
        case SHARP_ERR_SCRATCH_LIMIT:
            return "the operator needs more scratch than the allocation-free entry point holds "
                   "(SHARP_NOALLOC_SCRATCH_BYTES)";
    }
    return "unknown status";
}

// ---------------------------------------------------------------------------
// plan creation
// ---------------------------------------------------------------------------
static void build_csr(sharp_plan_s& p) {
    const int T = p.T, m = p.m;
    p.tiles_x = (p.nx + T - 1) / T;
    p.tiles_y = (p.ny + T - 1) / T;
    p.ntiles = p.tiles_x * p.tiles_y;
    // tile rows / columns touched by a frame (two wrapped segments at most)
    auto spans = [&](int start, int n, int ntl, std::vector<int>& out) {
        out.clear();
        for (int r = 0; r < m; ++r) {
            int v = start + r;
            if (v >= n) v -= n;  // periodic only; non-periodic never exceeds n-1
            const int t = v / T;
            if (out.empty() || out.back() != t) {
                if (std::find(out.begin(), out.end(), t) == out.end()) out.push_back(t);
            }
        }
        (void)ntl;
    };
    std::vector<int> count(p.ntiles, 0), rows, cols;
    for (int i = 0; i < p.K; ++i) {
        spans(p.pos[2 * i], p.ny, p.tiles_y, rows);
        spans(p.pos[2 * i + 1], p.nx, p.tiles_x, cols);
        for (int ty : rows)
            for (int tx : cols) ++count[ty * p.tiles_x + tx];
    }
    p.tile_ptr.assign(p.ntiles + 1, 0);
    for (int t = 0; t < p.ntiles; ++t) p.tile_ptr[t + 1] = p.tile_ptr[t] + count[t];
    p.tile_frames.assign(p.tile_ptr[p.ntiles], 0);
    std::vector<int> fill(p.tile_ptr.begin(), p.tile_ptr.end() - 1);
    for (int i = 0; i < p.K; ++i) {  // ascending frame order inside every tile
        spans(p.pos[2 * i], p.ny, p.tiles_y, rows);
        spans(p.pos[2 * i + 1], p.nx, p.tiles_x, cols);
        for (int ty : rows)
            for (int tx : cols) p.tile_frames[fill[ty * p.tiles_x + tx]++] = i;
    }
}

// Frames touching each strip of SH object rows, ascending (strip merge), and
// for each (frame, strip row) the frame row that lands there.
static void build_strips(sharp_plan_s& p) {
    p.nstrips = (p.ny + p.SH - 1) / p.SH;
    std::vector<int> count(p.nstrips, 0), hit;
    auto strips_of = [&](int i, std::vector<int>& out) {
        out.clear();
        const int py = p.pos[2 * i];
        for (int r = 0; r < p.m; ++r) {
            int y = py + r;
            if (y >= p.ny) y -= p.ny;  // periodic only
            const int sidx = y / p.SH;
            if (std::find(out.begin(), out.end(), sidx) == out.end()) out.push_back(sidx);
        }
    };
    for (int i = 0; i < p.K; ++i) {
        strips_of(i, hit);
        for (int sidx : hit) ++count[sidx];
    }
    p.strip_ptr.assign(p.nstrips + 1, 0);
    for (int t = 0; t < p.nstrips; ++t) p.strip_ptr[t + 1] = p.strip_ptr[t] + count[t];
    std::vector<int> frames(p.strip_ptr[p.nstrips], 0);
    std::vector<int> fill(p.strip_ptr.begin(), p.strip_ptr.end() - 1);
    for (int i = 0; i < p.K; ++i) {
        strips_of(i, hit);
        for (int sidx : hit) frames[fill[sidx]++] = i;
    }
    p.strip_lines.assign(frames.size() * p.SH * 4, 0);
    for (int sidx = 0; sidx < p.nstrips; ++sidx)
        for (int j = p.strip_ptr[sidx]; j < p.strip_ptr[sidx + 1]; ++j)
            for (int sr = 0; sr < p.SH; ++sr) {
                const int f = frames[j], y = sidx * p.SH + sr;
                int r = y - p.pos[2 * f];
                if (r < 0) r += p.ny;  // periodic only (else the frame does not reach y)
                int32_t* rec = &p.strip_lines[((size_t)j * p.SH + sr) * 4];
                const bool hit_row = y < p.ny && r < p.m;
                rec[0] = hit_row ? f : -1;
                rec[1] = hit_row ? r : 0;
                rec[2] = hit_row ? p.pos[2 * f + 1] : 0;
            }
    // launch order: strips with more frame rows first (longest-processing-time
    // order), so that the light strips at the object's edges fill the last
    // workgroup slots instead of a heavy strip starting last
    p.strip_order.resize(p.nstrips);
    for (int t = 0; t < p.nstrips; ++t) p.strip_order[t] = t;
    std::stable_sort(p.strip_order.begin(), p.strip_order.end(), [&](int a, int b) {
        return p.strip_ptr[a + 1] - p.strip_ptr[a] > p.strip_ptr[b + 1] - p.strip_ptr[b];
    });
}

static void choose_tuning(sharp_plan_s& p) {
    // tile side: 32 while that still gives >= 1024 tiles (workgroups enough
    // for the merge without a frame-chunk split and its finishing pass),
    // else 16
    if (p.opt.tile) p.T = p.opt.tile;
    else p.T = ((p.nx + 31) / 32) * ((p.ny + 31) / 32) >= 1024 ? 32 : 16;
    build_csr(p);
    int maxf = 0;
    for (int t = 0; t < p.ntiles; ++t) maxf = std::max(maxf, p.tile_ptr[t + 1] - p.tile_ptr[t]);
    if (p.opt.merge_split) p.split = p.opt.merge_split;
    else {
        // aim for >= 1024 workgroups in the first merge pass, >= 4 frames per chunk
        int s = (1024 + p.ntiles - 1) / p.ntiles;
        s = std::min(s, std::max(1, maxf / 4));
        p.split = std::max(1, s);
    }
    const int groups = (p.m == 256) ? p.K * 16 : (p.K + fg_groups(p.m) - 1) / fg_groups(p.m);
    if (p.opt.grad_groups) p.grad_groups = p.opt.grad_groups;
    else p.grad_groups = (p.m == 256) ? 1024 : std::min(groups, p.m == 128 ? 256 : 512);
    if (p.m == 256) p.grad_groups = std::max(16, p.grad_groups / 16 * 16);
    // frame chunks of the probe-update partial sums: at 841 frames of 64^2, 64
    // chunks took 0.0693 ms per probe iteration against 0.0726 (32 and 128) and 0.0780 (256)
    p.probe_chunks = std::min(p.K, 64);
    p.fft_block = p.opt.fft_block ? p.opt.fft_block : 256;
    // m = 256: Fourier-domain carry with the merge fused into the last row pass
    // unless asked otherwise; needs a strip of the object in LDS
    p.SH = p.m != 256 || p.nx > 8192 ? 0 : (p.opt.strip_rows == 2 && 2 * p.nx <= 8192) ? 2 : 1;
    // m = 256 default: the column pass with its own row transform once the
    // frames are many enough for its 4 K quarter-frame workgroups to fill the
    // GPU for several rounds (measured on parts of the 2025-frame scan: form 2
    // 5 % faster at 270 frames, form 3 5 % faster at 495 and 15 % at 990),
    // else the column pass reading the prepared gather
    p.frame_launch = p.opt.frame_launch ? p.opt.frame_launch
                                        : (p.m == 256 && p.K >= 400) ? 3 : (p.m >= 128 ? 2 : 1);
    if (p.m == 256 && p.frame_launch >= 2 && !p.SH) p.frame_launch = 1;
    if (p.m < 128) p.frame_launch = 1;
    if (p.m == 128 && p.frame_launch == 3) p.frame_launch = 2;
    if (p.strip_form()) build_strips(p);
}

static void layout(sharp_plan_s& p) {
    Offsets& o = p.off;
    size_t cur = 0;
    auto take = [&](size_t bytes) {
        size_t at = cur;
        cur = align_up(cur + bytes);
        return at;
    };
    const size_t FE = p.frame_elems(), OE = p.obj_elems(), MM = (size_t)p.m * p.m;
    o.tw = take(p.m * sizeof(float2));
    o.pos = take((size_t)p.K * 2 * sizeof(int32_t));
    o.tile_ptr = take((p.ntiles + 1) * sizeof(int32_t));
    o.tile_frames = take(std::max<size_t>(p.tile_frames.size(), 1) * sizeof(int32_t));
    o.a = take(FE * sizeof(float));
    o.a_t = take((p.m == 128 && p.carry_form()) || p.colg_form() ? FE * sizeof(float) : 0);
    o.u = take(FE * sizeof(float2));
    o.v = take(FE * sizeof(float2));
    o.stage = take(p.m == 256 ? FE * sizeof(float2) : 0);
    o.psi_v = take(OE * sizeof(float2));
    o.psi_l = take(OE * sizeof(float2));
    o.tmp_obj = take(OE * sizeof(float2));
    o.D = take(OE * sizeof(float));
    o.Dinv = take(OE * sizeof(float));
    o.w_cur = take(MM * sizeof(float2));
    o.w_gat = take(MM * sizeof(float2));
    o.tmp_w = take(MM * sizeof(float2));
    o.tmp_w2 = take(MM * sizeof(float2));
    o.pcons = take(MM * sizeof(float));
    o.mpart = take(p.split > 1 ? (size_t)p.ntiles * p.split * p.T * p.T * 2 * sizeof(float4) : 0);
    o.pnum = take((size_t)p.probe_chunks * MM * sizeof(float2));
    o.pden = take((size_t)p.probe_chunks * MM * sizeof(float));
    p.gw_slots = frame_partial_slots(p.m, FM_GRAD, p.grad_groups);
    if (p.m == 128 && p.carry_form()) p.gw_slots = std::max<size_t>(p.gw_slots, p.grad_chunks());
    o.gwpart = take(std::max<size_t>(p.gw_slots, 1) * MM * sizeof(float2));
    const size_t groups = (p.m == 256) ? (size_t)p.K * 32 : (size_t)(p.K + fg_groups(p.m) - 1) / fg_groups(p.m);
    p.resid_cap = std::max<size_t>(groups, 2048);
    o.resid = take(p.resid_cap * sizeof(float));
    o.hist = take(kHistCap * sizeof(float));
    o.scal = take(16 * sizeof(float));
    o.flag = take(16 * sizeof(int));
    o.sptr = take((p.strip_ptr.size() + 1) * sizeof(int32_t));
    o.sln = take((p.strip_lines.size() + 4) * sizeof(int32_t));
    o.sord = take((p.strip_order.size() + 1) * sizeof(int32_t));
    o.total = cur;
}

extern "C" int sharp_plan_create(sharp_plan* out, int nx, int ny, int m, int K, const int32_t* h_pos,
                                 const sharp_options* opt) {
    if (!out || !h_pos) return SHARP_ERR_INVALID_ARG;
    *out = nullptr;
    if (K < 1 || nx < 1 || ny < 1) return SHARP_ERR_INVALID_ARG;
    if (!supported_m(m) || m > nx || m > ny) return SHARP_ERR_UNSUPPORTED_SIZE;
    // frame stacks index with 32-bit element counts; objects with 32-bit byte offsets
    if ((long long)K * m * m > 2147483647LL || (long long)nx * ny > (1LL << 28)) return SHARP_ERR_UNSUPPORTED_SIZE;
    sharp_options o{};
    if (opt) {
        o = *opt;
        for (int r : o.reserved)
            if (r != 0) return SHARP_ERR_INVALID_ARG;
        if (o.periodic < 0 || o.periodic > 1 || o.probe_every < 0 || o.probe_start < 0 || !(o.eps_D >= 0.f) ||
            !(o.tile == 0 || o.tile == 16 || o.tile == 32 || o.tile == 64) || o.merge_split < 0 ||
            o.merge_split > 4096 || o.grad_groups < 0 || o.frame_launch < 0 || o.frame_launch > 3 ||
            !(o.fft_block == 0 || o.fft_block == 128 || o.fft_block == 256 || o.fft_block == 512) ||
            o.strip_rows < 0 || o.strip_rows > 2 || o.probe_center < 0 || o.probe_center > 1)
            return SHARP_ERR_INVALID_ARG;
    }
    if (o.probe_start == 0) o.probe_start = 1;
    for (int i = 0; i < K; ++i) {
        const int y = h_pos[2 * i], x = h_pos[2 * i + 1];
        const bool ok = o.periodic ? (y >= 0 && y < ny && x >= 0 && x < nx)
                                   : (y >= 0 && y <= ny - m && x >= 0 && x <= nx - m);
        if (!ok) return SHARP_ERR_POSITION_OUT_OF_RANGE;
    }
    sharp_plan_s* p = new (std::nothrow) sharp_plan_s();
    if (!p) return SHARP_ERR_HOST_ALLOC;
    try {
        p->nx = nx;
        p->ny = ny;
        p->m = m;
        p->K = K;
        p->opt = o;
        p->pos.assign(h_pos, h_pos + 2 * (size_t)K);
        choose_tuning(*p);
        layout(*p);
    } catch (...) {
        delete p;
        return SHARP_ERR_HOST_ALLOC;
    }
    *out = p;
    return SHARP_OK;
}

extern "C" void sharp_plan_destroy(sharp_plan p) { delete p; }

extern "C" size_t sharp_workspace_bytes(sharp_plan p) { return p ? p->off.total : 0; }

#define HIPCHK(x)                                   \
    do {                                            \
        hipError_t e_ = (x);                        \
        if (e_ != hipSuccess) return SHARP_ERR_HIP; \
    } while (0)

extern "C" int sharp_set_stream(sharp_plan p, void* stream) {
    if (!p) return SHARP_ERR_INVALID_ARG;
    p->stream = (hipStream_t)stream;
    return SHARP_OK;
}

static int density(sharp_plan_s& p);

extern "C" int sharp_set_workspace(sharp_plan p, void* d, size_t bytes) {
    if (!p || !d || ((uintptr_t)d % kAlign) != 0) return SHARP_ERR_INVALID_ARG;
    p->stage_gather = false;  // the stage buffer is about to be reused or the gather is out of date
    if (bytes < p->off.total) return SHARP_ERR_WORKSPACE_TOO_SMALL;
    p->ws = (char*)d;
    p->ws_bytes = bytes;
    p->ws_generation++;
    p->has_ws = true;
    p->has_data = p->has_probe = p->has_object = false;
    p->pcons_kind = 0;
    std::vector<float2> tw(p->m);
    for (int t = 0; t < p->m; ++t) {
        const double ang = 2.0 * M_PI * t / p->m;
        tw[t] = make_float2((float)std::cos(ang), (float)std::sin(ang));
    }
    hipStream_t s = p->stream;
    HIPCHK(hipMemcpyAsync(p->ws + p->off.tw, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(p->ws + p->off.pos, p->pos.data(), p->pos.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(p->ws + p->off.tile_ptr, p->tile_ptr.data(), p->tile_ptr.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice, s));
    if (!p->tile_frames.empty())
        HIPCHK(hipMemcpyAsync(p->ws + p->off.tile_frames, p->tile_frames.data(),
                              p->tile_frames.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIPCHK(launch_fill(p->ws + p->off.flag, 16 * sizeof(int), s));
    if (!p->strip_ptr.empty()) {
        HIPCHK(hipMemcpyAsync(p->ws + p->off.sptr, p->strip_ptr.data(), p->strip_ptr.size() * sizeof(int32_t),
                              hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(p->ws + p->off.sln, p->strip_lines.data(), p->strip_lines.size() * sizeof(int32_t),
                              hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(p->ws + p->off.sord, p->strip_order.data(), p->strip_order.size() * sizeof(int32_t),
                              hipMemcpyHostToDevice, s));
    }
    HIPCHK(launch_fill(p->ws + p->off.hist, kHistCap * sizeof(float), s));
    // host vectors are locals: finish the uploads before returning
    HIPCHK(hipStreamSynchronize(s));
    return SHARP_OK;
}

// ---------------------------------------------------------------------------
// argument blocks
// ---------------------------------------------------------------------------
FrameArgs sharp::frame_args(const sharp_plan_s& p) {
    FrameArgs A{};
    A.K = p.K;
    A.M = p.m;
    A.nx = p.nx;
    A.ny = p.ny;
    A.periodic = p.opt.periodic;
    A.pos = p.at<int>(p.off.pos);
    A.tw = p.at<float2>(p.off.tw);
    A.a = p.at<float>(p.off.a);
    A.at = p.at<float>(p.off.a_t);
    A.w_g = p.at<float2>(p.off.w_gat);
    A.w = p.at<float2>(p.off.w_cur);
    A.psi = p.at<float2>(p.off.psi_v);
    A.u = p.at<float2>(p.off.u);
    A.v = p.at<float2>(p.off.v);
    A.stage = p.m == 256 ? p.at<float2>(p.off.stage) : nullptr;
    A.resid = p.at<float>(p.off.resid);
    A.gw_part = p.at<float2>(p.off.gwpart);
    A.g = p.g;
    A.beta = 0.75f;
    A.stream = p.streams();
    return A;
}

MergeArgs sharp::merge_args(const sharp_plan_s& p) {
    MergeArgs A{};
    A.M = p.m;
    A.nx = p.nx;
    A.ny = p.ny;
    A.periodic = p.opt.periodic;
    A.T = p.T;
    A.tiles_x = p.tiles_x;
    A.split = p.split;
    A.tile_ptr = p.at<int>(p.off.tile_ptr);
    A.tile_frames = p.at<int>(p.off.tile_frames);
    A.pos = p.at<int>(p.off.pos);
    A.v = p.at<float2>(p.off.v);
    A.u = p.at<float2>(p.off.u);
    A.w = p.at<float2>(p.off.w_cur);
    A.Dinv = p.at<float>(p.off.Dinv);
    A.psi_v_in = p.at<float2>(p.off.psi_v);
    A.out = p.at<float2>(p.off.psi_v);
    A.out2 = p.at<float2>(p.off.psi_l);
    A.D_out = p.at<float>(p.off.D);
    A.Dinv_out = p.at<float>(p.off.Dinv);
    A.part = p.at<float4>(p.off.mpart);
    A.g = p.g;
    A.eps_D = p.opt.eps_D;
    return A;
}

int sharp::resid_blocks_default(const sharp_plan_s& p) {
    if (p.m == 128 && p.carry_form()) return fc128_groups(p.K);
    if (p.colg_form()) return p.K * 4;
    return p.m == 256 ? p.K * 16 : (p.K + fg_groups(p.m) - 1) / fg_groups(p.m);
}

int sharp::resid_blocks(const sharp_plan_s& p) {
    if (p.m == 256 && !p.carry_form()) return p.K * (4096 / p.fft_block);
    return resid_blocks_default(p);
}

static int density(sharp_plan_s& p) {
    MergeArgs A = merge_args(p);
    HIPCHK(launch_merge(MK_DENS, A, p.ntiles, p.stream));
    return SHARP_OK;
}

// ---------------------------------------------------------------------------
// inputs
// ---------------------------------------------------------------------------
extern "C" int sharp_set_data(sharp_plan p, const float* d_I) {
    if (!p || !d_I) return SHARP_ERR_INVALID_ARG;
    if (!p->has_ws) return SHARP_ERR_NOT_READY;
    int blocks = 0;
    const bool second = (p->m == 128 && p->carry_form()) || p->colg_form();
    HIPCHK(launch_set_data(d_I, p->at<float>(p->off.a), p->frame_elems(), p->at<float>(p->off.resid),
                           p->at<int>(p->off.flag), p->stream, &blocks, p->m == 256,
                           second ? p->at<float>(p->off.a_t) : nullptr, p->colg_form() ? 1 : 0));
    HIPCHK(launch_reduce(p->at<float>(p->off.resid), blocks, p->at<float>(p->off.scal), p->stream));
    p->has_data = true;
    return SHARP_OK;
}

extern "C" int sharp_set_probe(sharp_plan p, const void* d_w) {
    if (!p || !d_w) return SHARP_ERR_INVALID_ARG;
    p->stage_gather = false;  // the stage buffer is about to be reused or the gather is out of date
    if (!p->has_ws) return SHARP_ERR_NOT_READY;
    const size_t bytes = (size_t)p->m * p->m * sizeof(float2);
    HIPCHK(launch_copy(p->ws + p->off.w_cur, d_w, bytes, p->stream));
    HIPCHK(launch_copy(p->ws + p->off.w_gat, d_w, bytes, p->stream));
    int st = density(*p);
    if (st) return st;
    p->has_probe = true;
    p->has_object = false;
    return SHARP_OK;
}

extern "C" int sharp_init_probe(sharp_plan p) {
    if (!p) return SHARP_ERR_INVALID_ARG;
    p->stage_gather = false;  // the stage buffer is about to be reused or the gather is out of date
    if (!p->has_ws || !p->has_data) return SHARP_ERR_NOT_READY;
    hipStream_t s = p->stream;
    HIPCHK(launch_mean_amp(p->at<float>(p->off.a), p->K, p->m, p->at<float2>(p->off.tmp_w), s));
    FrameArgs A = frame_args(*p);
    A.K = 1;
    A.in = p->at<float2>(p->off.tmp_w);
    A.out = p->at<float2>(p->off.tmp_w2);
    HIPCHK(launch_frame(FM_FINV, A, 0, s, nullptr));
    HIPCHK(launch_roll_probe(p->at<float2>(p->off.tmp_w2), p->m, p->at<float2>(p->off.w_cur),
                             p->at<float2>(p->off.w_gat), s));
    int st = density(*p);
    if (st) return st;
    p->has_probe = true;
    p->has_object = false;
    return SHARP_OK;
}

extern "C" int sharp_set_probe_constraint(sharp_plan p, int kind, const float* d_values) {
    if (!p || kind < 0 || kind > 2 || (kind != 0 && !d_values)) return SHARP_ERR_INVALID_ARG;
    if (!p->has_ws) return SHARP_ERR_NOT_READY;
    if (kind) HIPCHK(launch_copy(p->ws + p->off.pcons, d_values, (size_t)p->m * p->m * sizeof(float), p->stream));
    p->pcons_kind = kind;
    return SHARP_OK;
}

extern "C" int sharp_set_object(sharp_plan p, const void* d_psi) {
    if (!p || !d_psi) return SHARP_ERR_INVALID_ARG;
    p->stage_gather = false;  // the stage buffer is about to be reused or the gather is out of date
    if (!p->has_ws || !p->has_probe) return SHARP_ERR_NOT_READY;
    hipStream_t s = p->stream;
    HIPCHK(launch_copy(p->ws + p->off.psi_v, d_psi, p->obj_elems() * sizeof(float2), s));
    HIPCHK(launch_fill(p->ws + p->off.u, p->frame_elems() * sizeof(float2), s));
    HIPCHK(launch_copy(p->ws + p->off.w_gat, p->ws + p->off.w_cur, (size_t)p->m * p->m * sizeof(float2), s));
    p->g = 1.f;  // z^(0) = Q psi0: carry 0, gather coefficient 1
    p->iter = 0;
    p->hist_count = 0;
    p->gat_stale = false;
    p->last_probe_updated = false;
    p->has_object = true;
    return SHARP_OK;
}

// ---------------------------------------------------------------------------
// iteration
// ---------------------------------------------------------------------------
// Fourier-domain carry -> frame space (u = F* U), into dst [K][m][m]
static hipError_t carry_to_space(sharp_plan_s& p, float2* dst) {
    FrameArgs A = frame_args(p);
    A.in = p.at<float2>(p.off.u);
    A.out = dst;
    if (p.m == 128) return launch_fc128_convert(A, 1, p.stream);
    return launch_carry_to_space(A, p.stream, p.carry_layout());
}
// frame space -> Fourier-domain carry (U = F u)
static hipError_t space_to_carry(sharp_plan_s& p, const float2* src) {
    FrameArgs A = frame_args(p);
    A.in = src;
    A.out = p.at<float2>(p.off.u);
    if (p.m == 128) return launch_fc128_convert(A, 0, p.stream);
    return launch_space_to_carry(A, p.stream, p.carry_layout());
}
// Algorithm box, step 7, after Eq. (standardprobe): the Fourier mask or
// Fourier amplitude constraint, then the centre-of-mass correction.
static hipError_t constrain_probe(sharp_plan_s& p) {
    hipStream_t s = p.stream;
    float2* w = p.at<float2>(p.off.w_cur);
    float2* tmp = p.at<float2>(p.off.tmp_w);
    if (p.pcons_kind) {
        FrameArgs A = frame_args(p);
        A.K = 1;
        A.in = w;
        A.out = tmp;
        hipError_t e = launch_frame(FM_F, A, 0, s, nullptr);
        if (e == hipSuccess) e = launch_probe_fourier(tmp, p.at<float>(p.off.pcons), p.m, p.pcons_kind, s);
        A.in = tmp;
        A.out = w;
        if (e == hipSuccess) e = launch_frame(FM_FINV, A, 0, s, nullptr);
        if (e != hipSuccess) return e;
    }
    if (p.opt.probe_center) return launch_probe_center(w, tmp, p.m, s);
    return hipSuccess;
}

static int one_iteration(sharp_plan_s& p, float beta) {
    hipStream_t s = p.stream;
    const long long it = p.iter + 1;
    const bool probe_due = p.opt.probe_every > 0 && it >= p.opt.probe_start &&
                           (it - p.opt.probe_start) % p.opt.probe_every == 0;
    FrameArgs A = frame_args(p);
    A.beta = beta;
    int blocks = 0;
    const Timer* t = p.tm();
    // eps_a of the iteration: formed by a workgroup of the merge launch that
    // follows the frame phase (the separate reduction's sum, bit for bit)
    auto eps_args = [&](int n) {
        return EpsArgs{p.at<float>(p.off.resid), n, p.at<float>(p.off.scal), p.at<float>(p.off.hist),
                       (int)(p.hist_count % kHistCap), p.at<int>(p.off.flag)};
    };
    if (p.colg_form()) {
        // column pass with its own gather and row transform, then the strip
        // merge of its octet rows; psi_v is final afterwards
        const StripArgs S{p.at<int>(p.off.sptr), p.at<int4>(p.off.sln), p.at<float>(p.off.Dinv),
                          p.at<float2>(p.off.psi_v), p.SH, 0, 0, 1, p.at<int>(p.off.sord)};
        blocks = p.K * 4;
        const EpsArgs E = eps_args(blocks);
        HIPCHK(launch_colg_256(A, s, t));
        HIPCHK(launch_strip_256(A, S, 0, p.nstrips, s, t, &E));
    } else if (p.strip_form()) {
        // frame phase and merge in one sequence; psi_v is final afterwards.  The
        // strip pass also prepares the next iteration's gather unless a probe
        // update (which reuses the stage buffer) follows.
        const StripArgs S{p.at<int>(p.off.sptr), p.at<int4>(p.off.sln), p.at<float>(p.off.Dinv),
                          p.at<float2>(p.off.psi_v), p.SH, probe_due ? 0 : 1, 0, 0, p.at<int>(p.off.sord)};
        blocks = p.K * 16;
        const EpsArgs E = eps_args(blocks);
        if (!p.stage_gather) HIPCHK(launch_row_gather_256(A, s, t));
        HIPCHK(launch_col_carry_256(A, s, t));
        HIPCHK(launch_strip_256(A, S, 0, p.nstrips, s, t, &E));
        p.stage_gather = !probe_due;
    } else if (p.carry_form()) {
        HIPCHK(launch_fc128(A, s, t, &blocks));
    } else if (p.m == 256) {
        HIPCHK(launch_raar_mp256(A, p.fft_block, s, t, &blocks));
    } else {
        HIPCHK(launch_frame(FM_RAAR, A, 0, s, &blocks, t));
    }
    if (p.gat_stale) {
        // the frames above were gathered with the probe before the last
        // update; later gathers use the current one.  A probe iteration's
        // update writes the gather probe itself (the probe it replaces, which
        // is the current one) and nothing reads it before, so the copy is only
        // needed when this iteration updates no probe.
        if (!probe_due)
            HIPCHK(launch_copy(p.ws + p.off.w_gat, p.ws + p.off.w_cur, (size_t)p.m * p.m * sizeof(float2), s));
        p.gat_stale = false;
    }
    const EpsArgs E = eps_args(blocks);   // tile-merge forms
    p.hist_count++;
    p.g = beta;
    MergeArgs Mg = merge_args(p);
    const float2* u_space = p.at<float2>(p.off.u);
    if (p.carry_form()) {
        if (!p.strip_form()) {  // m = 128: the frame kernel wrote v; tile merge
            if (t) t->begin(TC_MERGE);
            HIPCHK(launch_merge(MK_V, Mg, p.ntiles, s, &E));
            if (t) t->end(TC_MERGE);
        }
        if (probe_due) {
            // psi^(l) and the probe update need the carry in frame space
            if (t) t->begin(TC_PROBE);
            HIPCHK(carry_to_space(p, p.at<float2>(p.off.v)));
            Mg.u = p.at<float2>(p.off.v);
            Mg.out = p.at<float2>(p.off.psi_l);
            HIPCHK(launch_merge(MK_U, Mg, p.ntiles, s));
            u_space = p.at<float2>(p.off.v);
            if (t) t->end(TC_PROBE);
        }
    } else {
        if (t) t->begin(TC_MERGE);
        HIPCHK(launch_merge(probe_due ? MK_VU : MK_V, Mg, p.ntiles, s, &E));
        if (t) t->end(TC_MERGE);
    }
    if (probe_due) {
        if (t) t->begin(TC_PROBE);
        HIPCHK(launch_probe_partial(p.m, p.K, p.at<int>(p.off.pos), p.nx, p.ny, p.opt.periodic, u_space,
                                    p.at<float2>(p.off.w_cur), p.at<float2>(p.off.psi_v), p.at<float2>(p.off.psi_l),
                                    beta, p.probe_chunks, p.at<float2>(p.off.pnum), p.at<float>(p.off.pden), s));
        HIPCHK(launch_probe_finish(p.m, p.probe_chunks, p.at<float2>(p.off.pnum), p.at<float>(p.off.pden),
                                   p.at<float2>(p.off.w_gat), p.at<float2>(p.off.w_cur), s));
        HIPCHK(constrain_probe(p));
        int st = density(p);
        if (st) return st;
        if (t) t->end(TC_PROBE);
        p.gat_stale = true;
    }
    p.last_probe_updated = probe_due;
    p.iter = it;
    return SHARP_OK;
}

extern "C" int sharp_raar_iterate(sharp_plan p, int n, float beta) {
    if (!p || n < 0 || !(beta > 0.f && beta <= 1.f)) return SHARP_ERR_INVALID_ARG;
    if (!p->has_ws || !p->has_data || !p->has_probe || !p->has_object) return SHARP_ERR_NOT_READY;
    for (int l = 0; l < n; ++l) {
        int st = one_iteration(*p, beta);
        if (st) return st;
    }
    return SHARP_OK;
}

// ---------------------------------------------------------------------------
// outputs
// ---------------------------------------------------------------------------
extern "C" int sharp_get_object(sharp_plan p, void* d_out) {
    if (!p || !d_out) return SHARP_ERR_INVALID_ARG;
    p->stage_gather = false;  // the stage buffer is about to be reused or the gather is out of date
    if (!p->has_ws || !p->has_probe || !p->has_object) return SHARP_ERR_NOT_READY;
    if (p->last_probe_updated) {
        HIPCHK(launch_copy(d_out, p->ws + p->off.psi_l, p->obj_elems() * sizeof(float2), p->stream));
        return SHARP_OK;
    }
    MergeArgs A = merge_args(*p);
    A.out = (float2*)d_out;
    if (p->carry_form()) {
        HIPCHK(carry_to_space(*p, p->at<float2>(p->off.v)));
        A.u = p->at<float2>(p->off.v);
    }
    HIPCHK(launch_merge(MK_U, A, p->ntiles, p->stream));
    return SHARP_OK;
}

extern "C" int sharp_get_probe(sharp_plan p, void* d_out) {
    if (!p || !d_out) return SHARP_ERR_INVALID_ARG;
    if (!p->has_ws || !p->has_probe) return SHARP_ERR_NOT_READY;
    HIPCHK(launch_copy(d_out, p->ws + p->off.w_cur, (size_t)p->m * p->m * sizeof(float2), p->stream));
    return SHARP_OK;
}

static int read_flag(sharp_plan_s& p) {
    int flag = 0;
    HIPCHK(hipMemcpyAsync(&flag, p.ws + p.off.flag, sizeof(flag), hipMemcpyDeviceToHost, p.stream));
    HIPCHK(hipStreamSynchronize(p.stream));
    return flag ? SHARP_ERR_NONFINITE : SHARP_OK;
}

extern "C" int sharp_sync(sharp_plan p) {
    if (!p) return SHARP_ERR_INVALID_ARG;
    if (!p->has_ws) return SHARP_ERR_NOT_READY;
    return read_flag(*p);
}

extern "C" int sharp_get_metrics(sharp_plan p, float* h_eps, int max_n, int* n_written) {
    if (!p || max_n < 0 || (max_n > 0 && !h_eps)) return SHARP_ERR_INVALID_ARG;
    if (!p->has_ws) return SHARP_ERR_NOT_READY;
    std::vector<float> hist(kHistCap);
    HIPCHK(hipMemcpyAsync(hist.data(), p->ws + p->off.hist, kHistCap * sizeof(float), hipMemcpyDeviceToHost,
                          p->stream));
    int st = read_flag(*p);  // synchronises
    const long long cnt = std::min<long long>(p->hist_count, kHistCap);
    const long long start = p->hist_count - cnt;
    const int nw = (int)std::min<long long>(cnt, max_n);
    for (int j = 0; j < nw; ++j) h_eps[j] = hist[(start + j) % kHistCap];
    if (n_written) *n_written = nw;
    return st;
}

// ---------------------------------------------------------------------------
// gradient, forward model, operators
// ---------------------------------------------------------------------------
extern "C" int sharp_grad(sharp_plan p, const void* d_psi, const void* d_w, float* d_loss, void* d_gpsi,
                          void* d_gw) {
    if (!p || !d_psi || !d_w || !d_loss) return SHARP_ERR_INVALID_ARG;
    p->stage_gather = false;  // the stage buffer is about to be reused or the gather is out of date
    if (!p->has_ws || !p->has_data) return SHARP_ERR_NOT_READY;
    hipStream_t s = p->stream;
    FrameArgs A = frame_args(*p);
    A.psi = (const float2*)d_psi;
    A.w = (const float2*)d_w;
    A.w_g = (const float2*)d_w;
    int blocks = 0;
    // m = 128 Fourier-carry plans: the frame kernel writes r; Q* r applies
    // conj(w) in the merge and the probe gradient is a chunked pass over r
    const bool residual_form = p->m == 128 && p->carry_form();
    if (residual_form) HIPCHK(launch_fc128_grad(A, p->grad_groups, s, p->tm(), &blocks));
    else HIPCHK(launch_frame(FM_GRAD, A, p->grad_groups, s, &blocks, p->tm()));
    // the loss: the fixed-order sum of the frame launch's partials, formed by
    // a workgroup of the object-gradient merge when there is one (same bits)
    const EpsArgs L{p->at<float>(p->off.resid), p->m == 256 ? p->K * 16 : blocks, nullptr, d_loss, 0,
                    p->at<int>(p->off.flag)};
    if (!d_gpsi) HIPCHK(launch_loss(L.partials, L.n, d_loss, L.flag, s));
    if (d_gpsi) {
        MergeArgs Mg = merge_args(*p);
        Mg.out = (float2*)d_gpsi;
        if (residual_form) {
            Mg.u = p->at<float2>(p->off.v);
            Mg.w = (const float2*)d_w;
        }
        if (p->timing) p->timer.begin(TC_MERGE);
        HIPCHK(launch_merge(residual_form ? MK_RAWW : MK_RAW, Mg, p->ntiles, s, &L));
        if (p->timing) p->timer.end(TC_MERGE);
    }
    if (d_gw) {
        if (residual_form) {
            if (p->timing) p->timer.begin(TC_PROBE);
            HIPCHK(launch_grad_probe_partial(p->m, p->K, p->at<int>(p->off.pos), p->nx, p->ny, p->opt.periodic,
                                             p->at<float2>(p->off.v), (const float2*)d_psi, p->grad_chunks(),
                                             p->at<float2>(p->off.gwpart), s));
            if (p->timing) p->timer.end(TC_PROBE);
        }
        const int slots = residual_form ? p->grad_chunks() : frame_partial_slots(p->m, FM_GRAD, blocks);
        HIPCHK(launch_gw_finish(p->m, slots, p->at<float2>(p->off.gwpart), (float2*)d_gw, s));
    }
    return SHARP_OK;
}

extern "C" int sharp_simulate(sharp_plan p, const void* d_psi, const void* d_w, float* d_I) {
    if (!p || !d_psi || !d_w || !d_I) return SHARP_ERR_INVALID_ARG;
    p->stage_gather = false;  // the stage buffer is about to be reused or the gather is out of date
    if (!p->has_ws) return SHARP_ERR_NOT_READY;
    FrameArgs A = frame_args(*p);
    A.psi = (const float2*)d_psi;
    A.w = (const float2*)d_w;
    A.out_f = d_I;
    HIPCHK(launch_frame(FM_SIM, A, 0, p->stream, nullptr));
    return SHARP_OK;
}

// Scratch the operators of sharp_apply use beyond their input and output:
// the row-transformed frames between the passes of the m = 256 frame kernels,
// the residual partials the data projector writes, the object temporary of
// P_Q and the frame-chunk partials of a split merge.  Offsets into one buffer.
ApplyScratch sharp::apply_scratch(const sharp_plan_s& p, int op) {
    ApplyScratch S{};
    size_t cur = 0;
    auto take = [&](size_t bytes) {
        size_t at = cur;
        cur = align_up(cur + bytes);
        return at;
    };
    const bool frame_op = op == SHARP_OP_F || op == SHARP_OP_FINV || op == SHARP_OP_PA;
    const bool merge_op = op == SHARP_OP_QSTAR || op == SHARP_OP_OBJECT || op == SHARP_OP_PQ;
    S.stage = take(frame_op && p.m == 256 ? p.frame_elems() * sizeof(float2) : 0);
    S.resid = take(op == SHARP_OP_PA ? p.resid_cap * sizeof(float) : 0);
    S.tmp_obj = take(op == SHARP_OP_PQ ? p.obj_elems() * sizeof(float2) : 0);
    S.mpart = take(merge_op && p.split > 1 ? (size_t)p.ntiles * p.split * p.T * p.T * 2 * sizeof(float4) : 0);
    S.total = cur;
    return S;
}

int sharp::apply_check(const sharp_plan_s& p, int op, const void* d_in, const void* d_out) {
    if (op < SHARP_OP_F || op > SHARP_OP_OBJECT || !d_in || !d_out || d_in == d_out) return SHARP_ERR_INVALID_ARG;
    if (!p.has_ws) return SHARP_ERR_NOT_READY;
    if (op != SHARP_OP_F && op != SHARP_OP_FINV && !p.has_probe) return SHARP_ERR_NOT_READY;
    if (op == SHARP_OP_PA && !p.has_data) return SHARP_ERR_NOT_READY;
    return SHARP_OK;
}

int sharp::apply_into(sharp_plan_s& pl, int op, const void* d_in, void* d_out, char* scratch) {
    sharp_plan_s* p = &pl;
    if (!d_in || !d_out || d_in == d_out) return SHARP_ERR_INVALID_ARG;
    p->stage_gather = false;  // the stage buffer is about to be reused or the gather is out of date
    const int chk = apply_check(*p, op, d_in, d_out);
    if (chk != SHARP_OK) return chk;
    hipStream_t s = p->stream;
    FrameArgs A = frame_args(*p);
    MergeArgs Mg = merge_args(*p);
    float2* tmp_obj = p->at<float2>(p->off.tmp_obj);
    if (scratch) {  // the caller's scratch replaces the workspace segments the operators use as scratch
        const ApplyScratch S = apply_scratch(*p, op);
        if (p->m == 256) A.stage = reinterpret_cast<float2*>(scratch + S.stage);
        A.resid = reinterpret_cast<float*>(scratch + S.resid);
        tmp_obj = reinterpret_cast<float2*>(scratch + S.tmp_obj);
        Mg.part = reinterpret_cast<float4*>(scratch + S.mpart);
    }
    switch (op) {
        case SHARP_OP_F:
        case SHARP_OP_FINV:
        case SHARP_OP_PA:
            A.in = (const float2*)d_in;
            A.out = (float2*)d_out;
            HIPCHK(launch_frame(op == SHARP_OP_F ? FM_F : op == SHARP_OP_FINV ? FM_FINV : FM_PA, A, 0, s, nullptr));
            return SHARP_OK;
        case SHARP_OP_Q:
            A.psi = (const float2*)d_in;
            A.out = (float2*)d_out;
            HIPCHK(launch_frame(FM_Q, A, 0, s, nullptr));
            return SHARP_OK;
        case SHARP_OP_QSTAR:
        case SHARP_OP_OBJECT:
            Mg.u = (const float2*)d_in;
            Mg.out = (float2*)d_out;
            HIPCHK(launch_merge(op == SHARP_OP_QSTAR ? MK_RAWW : MK_OBJ, Mg, p->ntiles, s));
            return SHARP_OK;
        case SHARP_OP_PQ:
            Mg.u = (const float2*)d_in;
            Mg.out = tmp_obj;
            HIPCHK(launch_merge(MK_OBJ, Mg, p->ntiles, s));
            A.psi = tmp_obj;
            A.out = (float2*)d_out;
            HIPCHK(launch_frame(FM_Q, A, 0, s, nullptr));
            return SHARP_OK;
    }
    return SHARP_ERR_INVALID_ARG;
}

extern "C" int sharp_apply(sharp_plan p, int op, const void* d_in, void* d_out) {
    if (!p) return SHARP_ERR_INVALID_ARG;
    return apply_into(*p, op, d_in, d_out, nullptr);
}

// ---------------------------------------------------------------------------
// checkpoint / resume
// ---------------------------------------------------------------------------
namespace {
struct StateHeader {
    long long magic, iter, hist_count;
    int nx, ny, m, K;
    float g;
    int gat_stale, last_probe_updated, pad;
};
constexpr long long kMagic = 0x5348415250535431LL;

struct StateLayout {
    size_t u, psi_v, psi_l, w_cur, w_gat, hist, header, total;
};
StateLayout state_layout(const sharp_plan_s& p) {
    StateLayout L{};
    size_t cur = 0;
    auto take = [&](size_t b) {
        size_t at = cur;
        cur = align_up(cur + b);
        return at;
    };
    const size_t MM = (size_t)p.m * p.m;
    L.u = take(p.frame_elems() * sizeof(float2));
    L.psi_v = take(p.obj_elems() * sizeof(float2));
    L.psi_l = take(p.obj_elems() * sizeof(float2));
    L.w_cur = take(MM * sizeof(float2));
    L.w_gat = take(MM * sizeof(float2));
    L.hist = take(kHistCap * sizeof(float));
    L.header = take(sizeof(StateHeader));
    L.total = cur;
    return L;
}
}  // namespace

extern "C" size_t sharp_state_bytes(sharp_plan p) { return p ? state_layout(*p).total : 0; }

extern "C" int sharp_get_state(sharp_plan p, void* d_state) {
    if (!p || !d_state) return SHARP_ERR_INVALID_ARG;
    p->stage_gather = false;  // the stage buffer is about to be reused or the gather is out of date
    if (!p->has_ws || !p->has_probe || !p->has_object) return SHARP_ERR_NOT_READY;
    const StateLayout L = state_layout(*p);
    char* d = (char*)d_state;
    hipStream_t s = p->stream;
    const size_t MM = (size_t)p->m * p->m;
    if (p->carry_form()) HIPCHK(carry_to_space(*p, (float2*)(d + L.u)));
    else HIPCHK(launch_copy(d + L.u, p->ws + p->off.u, p->frame_elems() * sizeof(float2), s));
    HIPCHK(launch_copy(d + L.psi_v, p->ws + p->off.psi_v, p->obj_elems() * sizeof(float2), s));
    HIPCHK(launch_copy(d + L.psi_l, p->ws + p->off.psi_l, p->obj_elems() * sizeof(float2), s));
    HIPCHK(launch_copy(d + L.w_cur, p->ws + p->off.w_cur, MM * sizeof(float2), s));
    HIPCHK(launch_copy(d + L.w_gat, p->ws + p->off.w_gat, MM * sizeof(float2), s));
    HIPCHK(launch_copy(d + L.hist, p->ws + p->off.hist, kHistCap * sizeof(float), s));
    StateHeader h{kMagic, p->iter, p->hist_count, p->nx, p->ny, p->m, p->K, p->g,
                  p->gat_stale ? 1 : 0, p->last_probe_updated ? 1 : 0, 0};
    HIPCHK(hipMemcpyAsync(d + L.header, &h, sizeof(h), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return SHARP_OK;
}

extern "C" int sharp_set_state(sharp_plan p, const void* d_state) {
    if (!p || !d_state) return SHARP_ERR_INVALID_ARG;
    p->stage_gather = false;  // the stage buffer is about to be reused or the gather is out of date
    if (!p->has_ws || !p->has_data) return SHARP_ERR_NOT_READY;
    const StateLayout L = state_layout(*p);
    const char* d = (const char*)d_state;
    hipStream_t s = p->stream;
    StateHeader h{};
    HIPCHK(hipMemcpyAsync(&h, d + L.header, sizeof(h), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (h.magic != kMagic || h.nx != p->nx || h.ny != p->ny || h.m != p->m || h.K != p->K)
        return SHARP_ERR_INVALID_ARG;
    // the counters index the eps_a history and g scales the gather: reject a
    // header whose fields no run of this library writes
    if (h.iter < 0 || h.hist_count < 0 || h.hist_count > h.iter || !std::isfinite(h.g) || h.g < 0.f || h.g > 1.f ||
        (h.gat_stale != 0 && h.gat_stale != 1) || (h.last_probe_updated != 0 && h.last_probe_updated != 1))
        return SHARP_ERR_INVALID_ARG;
    const size_t MM = (size_t)p->m * p->m;
    if (p->carry_form()) {
        HIPCHK(space_to_carry(*p, (const float2*)(d + L.u)));
    } else {
        HIPCHK(launch_copy(p->ws + p->off.u, d + L.u, p->frame_elems() * sizeof(float2), s));
    }
    HIPCHK(launch_copy(p->ws + p->off.psi_v, d + L.psi_v, p->obj_elems() * sizeof(float2), s));
    HIPCHK(launch_copy(p->ws + p->off.psi_l, d + L.psi_l, p->obj_elems() * sizeof(float2), s));
    HIPCHK(launch_copy(p->ws + p->off.w_cur, d + L.w_cur, MM * sizeof(float2), s));
    HIPCHK(launch_copy(p->ws + p->off.w_gat, d + L.w_gat, MM * sizeof(float2), s));
    HIPCHK(launch_copy(p->ws + p->off.hist, d + L.hist, kHistCap * sizeof(float), s));
    p->iter = h.iter;
    p->hist_count = h.hist_count;
    p->g = h.g;
    p->gat_stale = h.gat_stale != 0;
    p->last_probe_updated = h.last_probe_updated != 0;
    int st = density(*p);
    if (st) return st;
    p->has_probe = true;
    p->has_object = true;
    return SHARP_OK;
}

// ---------------------------------------------------------------------------
// introspection
// ---------------------------------------------------------------------------
extern "C" int sharp_get_plan_info(sharp_plan p, sharp_plan_info* info) {
    if (!p || !info) return SHARP_ERR_INVALID_ARG;
    info->nx = p->nx;
    info->ny = p->ny;
    info->m = p->m;
    info->K = p->K;
    info->periodic = p->opt.periodic;
    info->tile = p->T;
    info->tiles_x = p->tiles_x;
    info->tiles_y = p->tiles_y;
    info->merge_split = p->split;
    info->grad_groups = p->grad_groups;
    info->frame_launch = p->frame_launch;
    info->fft_block = p->fft_block;
    info->strip_rows = p->strip_form() ? p->SH : 0;
    info->streaming = p->streams() ? 1 : 0;
    info->csr_nnz = (long long)p->tile_frames.size();
    info->iteration = p->iter;
    return SHARP_OK;
}

extern "C" int sharp_get_plan_csr(sharp_plan p, int32_t* h_ptr, int32_t* h_frames) {
    if (!p || !h_ptr || !h_frames) return SHARP_ERR_INVALID_ARG;
    std::memcpy(h_ptr, p->tile_ptr.data(), p->tile_ptr.size() * sizeof(int32_t));
    std::memcpy(h_frames, p->tile_frames.data(), p->tile_frames.size() * sizeof(int32_t));
    return SHARP_OK;
}

// ---------------------------------------------------------------------------
// kernel timing
// ---------------------------------------------------------------------------
extern "C" int sharp_timing_enable(sharp_plan p, int on) {
    if (!p) return SHARP_ERR_INVALID_ARG;
    p->timing = on != 0;
    p->timer.ctx = p;
    p->timer.mark = timer_mark;
    return SHARP_OK;
}

extern "C" int sharp_timing_read(sharp_plan p, double* h_ms, long long* h_launches) {
    if (!p || !h_ms || !h_launches) return SHARP_ERR_INVALID_ARG;
    HIPCHK(hipStreamSynchronize(p->stream));
    for (int c = 0; c < TC_N; ++c) {
        h_ms[c] = 0.0;
        h_launches[c] = 0;
        for (auto& pr : p->ev_pairs[c]) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, pr.first, pr.second));
            h_ms[c] += ms;
            h_launches[c] += 1;
            p->ev_pool.push_back(pr.first);
            p->ev_pool.push_back(pr.second);
        }
        p->ev_pairs[c].clear();
    }
    return SHARP_OK;
}
