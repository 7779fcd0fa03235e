// Batched RAAR over independent scans (plans) of uneven sizes.
//
// One iteration of every scan is one fixed launch sequence: per frame-size
// class a frame kernel over a (scan, item) work list (one item per
// workgroup), one residual reduction with a block per scan, and per
// merge-tile class a merge kernel over (scan, tile, chunk) items.  Kernels
// take the argument blocks of up to kBatchChunk scans by value, so each class
// is launched once per chunk of scans that has items of that class.  n
// iterations are captured once into a hipGraph (keyed by n and beta) and
// replayed on the batch's own stream, which is ordered after the caller's
// stream with events.  Work items run exactly the single-scan arithmetic, so
// each scan's result equals its single-scan run bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <new>
#include <utility>
#include <vector>

#include "../../include/sharp.h"
#include "plan_impl.hpp"
#include "sharp_internal.hpp"

using namespace sharp;

namespace {
constexpr int kM[5] = {16, 32, 64, 128, 256};
constexpr int kT[3] = {16, 32, 64};
int m_class(int m) {
    for (int i = 0; i < 5; ++i)
        if (kM[i] == m) return i;
    return -1;
}
int t_class(int t) {
    for (int i = 0; i < 3; ++i)
        if (kT[i] == t) return i;
    return -1;
}
}  // namespace

struct sharp_batch_s {
    std::vector<sharp_plan_s*> plans;
    std::vector<unsigned long long> ws_gen;  // each plan's workspace generation when the batch took its pointers
    std::vector<int2> frame_items[5];     // per frame-size class (m = 256: frame-space carry form)
    std::vector<int4> merge_items[3];     // per merge-tile class
    std::vector<int2> finish_items[3];
    std::vector<int2> carry_items[3];     // m = 256 Fourier-carry forms: rows, columns (form 2), strips
    std::vector<int2> colg_items;         // m = 256 form 3: column pass with its own row transform
    // first item of each scan in every list (prefix sums, nplans + 1 entries)
    std::vector<int> frame_first[5], merge_first[3], finish_first[3], carry_first[3], fc_first, colg_first;
    std::vector<BatchArgs> arg_chunks;          // argument blocks by value, kBatchChunk scans each
    std::vector<BatchMergeArgs> merge_chunks;
    std::vector<int2> fc_items;           // m = 128 Fourier-carry form: (scan, frame group)
    size_t carry_smem = 0;                // LDS of the strip phase (widest object)
    struct {
        size_t fargs, eps, fitems[5], mitems[3], fin[3], citems[3], fcitems, gitems, total;
    } off{};
    char* ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t user = nullptr;      // caller's stream
    hipStream_t own = nullptr;       // batch stream (graphs are captured and replayed here)
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    std::map<std::pair<int, float>, std::pair<hipGraph_t, hipGraphExec_t>> graphs;

    ~sharp_batch_s() {
        for (auto& kv : graphs) {
            (void)hipGraphExecDestroy(kv.second.second);
            (void)hipGraphDestroy(kv.second.first);
        }
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (ev_out) (void)hipEventDestroy(ev_out);
        if (own) (void)hipStreamDestroy(own);
    }
    template <class T> T* at(size_t o) const { return reinterpret_cast<T*>(ws + o); }
};

extern "C" int sharp_batch_create(sharp_batch* out, int nplans, const sharp_plan* plans) {
    if (!out) return SHARP_ERR_INVALID_ARG;
    *out = nullptr;
    if (!plans || nplans < 1 || nplans > kMaxBatch) return SHARP_ERR_INVALID_ARG;
    for (int i = 0; i < nplans; ++i) {
        sharp_plan_s* p = plans[i];
        if (!p) return SHARP_ERR_INVALID_ARG;
        for (int j = 0; j < i; ++j)
            if (plans[j] == p) return SHARP_ERR_INVALID_ARG;
        if (p->opt.probe_every != 0) return SHARP_ERR_INVALID_ARG;
        if (!p->has_ws || !p->has_data || !p->has_probe || !p->has_object) return SHARP_ERR_NOT_READY;
    }
    sharp_batch_s* b = new (std::nothrow) sharp_batch_s();
    if (!b) return SHARP_ERR_HOST_ALLOC;
    try {
        for (int s = 0; s < nplans; ++s) {
            sharp_plan_s* p = plans[s];
            b->plans.push_back(p);
            if (p->colg_form()) {
                for (int it = 0; it < colg_items(p->K); ++it) b->colg_items.push_back(make_int2(s, it));
                for (int st = 0; st < p->nstrips; ++st) b->carry_items[2].push_back(make_int2(s, st));
                b->carry_smem = std::max(b->carry_smem, strip_smem_bytes(p->SH, p->nx));
                continue;
            }
            if (p->strip_form()) {
                for (int it = 0; it < p->K * 16; ++it) {
                    b->carry_items[0].push_back(make_int2(s, it));
                    b->carry_items[1].push_back(make_int2(s, it));
                }
                for (int st = 0; st < p->nstrips; ++st) b->carry_items[2].push_back(make_int2(s, st));
                b->carry_smem = std::max(b->carry_smem, strip_smem_bytes(p->SH, p->nx));
                continue;  // merged in the strip phase, no tile merge
            }
            const int items = resid_blocks_default(*p);  // frame groups (m <= 128) or row blocks (m = 256)
            if (p->carry_form()) {  // m = 128, Fourier-domain carry: (scan, frame group) items
                for (int it = 0; it < items; ++it) b->fc_items.push_back(make_int2(s, it));
            } else {
                const int mc = m_class(p->m);
                for (int it = 0; it < items; ++it) b->frame_items[mc].push_back(make_int2(s, it));
            }
            const int tc = t_class(p->T);
            for (int t = 0; t < p->ntiles; ++t)
                for (int c = 0; c < p->split; ++c) b->merge_items[tc].push_back(make_int4(s, t, c, 0));
            if (p->split > 1)
                for (int t = 0; t < p->ntiles; ++t) b->finish_items[tc].push_back(make_int2(s, t));
        }
        // strip items: within each chunk of scans (one launch), the strips with
        // the most frame rows first, as in the single-scan launch order
        {
            auto& it2 = b->carry_items[2];
            auto lines = [&](const int2& w) {
                const sharp_plan_s* q = b->plans[w.x];
                return q->strip_ptr[w.y + 1] - q->strip_ptr[w.y];
            };
            for (size_t c0 = 0; c0 < it2.size();) {
                size_t c1 = c0;
                const int chunk = it2[c0].x / kBatchChunk;
                while (c1 < it2.size() && it2[c1].x / kBatchChunk == chunk) ++c1;
                std::stable_sort(it2.begin() + c0, it2.begin() + c1,
                                 [&](const int2& a, const int2& w) { return lines(a) > lines(w); });
                c0 = c1;
            }
        }
        // items are listed chunk by chunk: the items of scans s0 .. s1 - 1 (one
        // chunk) are first[s0] .. first[s1] - 1
        auto prefix = [&](const auto& items, std::vector<int>& first) {
            first.assign(nplans + 1, 0);
            for (const auto& w : items) ++first[w.x + 1];
            for (int s = 0; s < nplans; ++s) first[s + 1] += first[s];
        };
        for (int c = 0; c < 5; ++c) prefix(b->frame_items[c], b->frame_first[c]);
        for (int c = 0; c < 3; ++c) {
            prefix(b->merge_items[c], b->merge_first[c]);
            prefix(b->finish_items[c], b->finish_first[c]);
            prefix(b->carry_items[c], b->carry_first[c]);
        }
        prefix(b->fc_items, b->fc_first);
        prefix(b->colg_items, b->colg_first);
        size_t cur = 0;
        auto take = [&](size_t bytes) {
            size_t at = cur;
            cur = align_up(cur + bytes);
            return at;
        };
        b->off.fargs = take(nplans * sizeof(FrameArgs));
        b->off.eps = take(nplans * sizeof(EpsDesc));
        for (int c = 0; c < 3; ++c) b->off.citems[c] = take(b->carry_items[c].size() * sizeof(int2));
        b->off.fcitems = take(b->fc_items.size() * sizeof(int2));
        b->off.gitems = take(b->colg_items.size() * sizeof(int2));
        for (int c = 0; c < 5; ++c) b->off.fitems[c] = take(b->frame_items[c].size() * sizeof(int2));
        for (int c = 0; c < 3; ++c) {
            b->off.mitems[c] = take(b->merge_items[c].size() * sizeof(int4));
            b->off.fin[c] = take(b->finish_items[c].size() * sizeof(int2));
        }
        b->off.total = cur;
    } catch (...) {
        delete b;
        return SHARP_ERR_HOST_ALLOC;
    }
    *out = b;
    return SHARP_OK;
}

extern "C" void sharp_batch_destroy(sharp_batch b) { delete b; }

extern "C" size_t sharp_batch_workspace_bytes(sharp_batch b) { return b ? b->off.total : 0; }

extern "C" int sharp_batch_set_stream(sharp_batch b, void* stream) {
    if (!b) return SHARP_ERR_INVALID_ARG;
    b->user = (hipStream_t)stream;
    return SHARP_OK;
}

#define HIPCHK(x)                                   \
    do {                                            \
        hipError_t e_ = (x);                        \
        if (e_ != hipSuccess) return SHARP_ERR_HIP; \
    } while (0)

extern "C" int sharp_batch_set_workspace(sharp_batch b, void* d, size_t bytes) {
    if (!b || !d || ((uintptr_t)d % kAlign) != 0) return SHARP_ERR_INVALID_ARG;
    if (bytes < b->off.total) return SHARP_ERR_WORKSPACE_TOO_SMALL;
    b->ws = (char*)d;
    b->ws_bytes = bytes;
    for (auto& kv : b->graphs) {
        (void)hipGraphExecDestroy(kv.second.second);
        (void)hipGraphDestroy(kv.second.first);
    }
    b->graphs.clear();
    if (!b->own) HIPCHK(hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking));
    if (!b->ev_in) HIPCHK(hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming));
    if (!b->ev_out) HIPCHK(hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming));
    const int n = (int)b->plans.size();
    b->ws_gen.assign(n, 0);
    for (int s = 0; s < n; ++s) {
        if (!b->plans[s]->has_ws) return SHARP_ERR_NOT_READY;
        b->ws_gen[s] = b->plans[s]->ws_generation;
    }
    std::vector<FrameArgs> fa(n);
    std::vector<MergeArgs> ma(n);
    std::vector<EpsDesc> ea(n);
    std::vector<StripArgs> sa(n);
    for (int s = 0; s < n; ++s) {
        sharp_plan_s& p = *b->plans[s];
        fa[s] = frame_args(p);
        ma[s] = merge_args(p);
        // form 3: the column pass gathers for itself and leaves octet rows
        sa[s] = StripArgs{p.at<int>(p.off.sptr), p.at<int4>(p.off.sln), p.at<float>(p.off.Dinv),
                          p.at<float2>(p.off.psi_v), p.SH, p.colg_form() ? 0 : 1, 0, p.colg_form() ? 1 : 0, nullptr};
        ea[s] = EpsDesc{p.at<float>(p.off.resid), resid_blocks_default(p), 0, p.at<float>(p.off.scal),
                        p.at<float>(p.off.hist), p.at<int>(p.off.flag)};
    }
    b->arg_chunks.assign((n + kBatchChunk - 1) / kBatchChunk, BatchArgs{});
    b->merge_chunks.assign((n + kBatchChunk - 1) / kBatchChunk, BatchMergeArgs{});
    for (int s = 0; s < n; ++s) {
        BatchArgs& C = b->arg_chunks[s / kBatchChunk];
        BatchMergeArgs& CM = b->merge_chunks[s / kBatchChunk];
        C.base = CM.base = s / kBatchChunk * kBatchChunk;
        C.a[s % kBatchChunk] = fa[s];
        C.s[s % kBatchChunk] = sa[s];
        CM.a[s % kBatchChunk] = ma[s];
    }
    hipStream_t st = b->own;
    HIPCHK(hipMemcpyAsync(b->ws + b->off.fargs, fa.data(), n * sizeof(FrameArgs), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(b->ws + b->off.eps, ea.data(), n * sizeof(EpsDesc), hipMemcpyHostToDevice, st));
    for (int c = 0; c < 3; ++c)
        if (!b->carry_items[c].empty())
            HIPCHK(hipMemcpyAsync(b->ws + b->off.citems[c], b->carry_items[c].data(),
                                  b->carry_items[c].size() * sizeof(int2), hipMemcpyHostToDevice, st));
    if (!b->fc_items.empty())
        HIPCHK(hipMemcpyAsync(b->ws + b->off.fcitems, b->fc_items.data(), b->fc_items.size() * sizeof(int2),
                              hipMemcpyHostToDevice, st));
    if (!b->colg_items.empty())
        HIPCHK(hipMemcpyAsync(b->ws + b->off.gitems, b->colg_items.data(), b->colg_items.size() * sizeof(int2),
                              hipMemcpyHostToDevice, st));
    for (int c = 0; c < 5; ++c)
        if (!b->frame_items[c].empty())
            HIPCHK(hipMemcpyAsync(b->ws + b->off.fitems[c], b->frame_items[c].data(),
                                  b->frame_items[c].size() * sizeof(int2), hipMemcpyHostToDevice, st));
    for (int c = 0; c < 3; ++c) {
        if (!b->merge_items[c].empty())
            HIPCHK(hipMemcpyAsync(b->ws + b->off.mitems[c], b->merge_items[c].data(),
                                  b->merge_items[c].size() * sizeof(int4), hipMemcpyHostToDevice, st));
        if (!b->finish_items[c].empty())
            HIPCHK(hipMemcpyAsync(b->ws + b->off.fin[c], b->finish_items[c].data(),
                                  b->finish_items[c].size() * sizeof(int2), hipMemcpyHostToDevice, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    // LDS limits of the kernels (grids: one item per workgroup)
    int per = 1;
    for (int c = 0; c < 5; ++c)
        for (int ph = 0; ph < (kM[c] == 256 ? 3 : 1); ++ph) HIPCHK(batch_frame_prepare(kM[c], ph, &per));
    for (int ph = 0; ph < 3; ++ph) {
        const size_t smem = ph == 2 ? b->carry_smem : carry_phase_smem();
        if (!b->carry_items[ph].empty()) HIPCHK(batch_carry_prepare(ph, smem, &per));
    }
    if (!b->fc_items.empty()) HIPCHK(batch_fc128_prepare(&per));
    if (!b->colg_items.empty()) HIPCHK(batch_colg_prepare());
    return SHARP_OK;
}

// One launch per chunk of kBatchChunk scans that has items in the list.
template <class F>
static int per_chunk(const sharp_batch_s& b, const std::vector<int>& first, F launch) {
    const int ns = (int)b.plans.size();
    for (int c = 0; c * kBatchChunk < ns; ++c) {
        const int s0 = c * kBatchChunk, s1 = std::min(ns, s0 + kBatchChunk);
        if (first[s1] > first[s0] && launch(c, first[s0], first[s1] - first[s0]) != hipSuccess) return SHARP_ERR_HIP;
    }
    return SHARP_OK;
}

static int enqueue_iterations(sharp_batch_s& b, int n, float beta, hipStream_t s) {
    FrameArgs* D = b.at<FrameArgs>(b.off.fargs);
    EpsDesc* E = b.at<EpsDesc>(b.off.eps);
    const int ns = (int)b.plans.size();
#define CHUNKS(first, launch)                          \
    do {                                               \
        const int st_ = per_chunk(b, first, launch);   \
        if (st_ != SHARP_OK) return st_;               \
    } while (0)
    for (int l = 0; l < n; ++l) {
        for (int c = 0; c < 5; ++c) {
            const int2* items = b.at<int2>(b.off.fitems[c]);
            for (int ph = 0; ph < (kM[c] == 256 ? 3 : 1); ++ph)
                CHUNKS(b.frame_first[c], [&](int k, int i0, int cnt) {
                    return launch_batch_frame(kM[c], ph, b.arg_chunks[k], D, items + i0, cnt, s);
                });
        }
        CHUNKS(b.fc_first, [&](int k, int i0, int cnt) {
            return launch_batch_fc128(b.arg_chunks[k], D, b.at<int2>(b.off.fcitems) + i0, cnt, s);
        });
        for (int ph = l == 0 ? 0 : 1; ph < 2; ++ph)  // later gathers come from the strip phase
            CHUNKS(b.carry_first[ph], [&](int k, int i0, int cnt) {
                return launch_batch_carry(ph, b.arg_chunks[k], D, b.at<int2>(b.off.citems[ph]) + i0, cnt,
                                          carry_phase_smem(), s);
            });
        CHUNKS(b.colg_first, [&](int k, int i0, int cnt) {
            return launch_batch_colg(b.arg_chunks[k], D, b.at<int2>(b.off.gitems) + i0, cnt, s);
        });
        HIPCHK(launch_batch_eps(E, D, ns, beta, s));
        CHUNKS(b.carry_first[2], [&](int k, int i0, int cnt) {
            return launch_batch_carry(2, b.arg_chunks[k], D, b.at<int2>(b.off.citems[2]) + i0, cnt, b.carry_smem, s);
        });
        for (int c = 0; c < 3; ++c) {
            // a chunk's merge items, then its finish items (the chunk partials of the same scans)
            const int st = per_chunk(b, b.merge_first[c], [&](int k, int i0, int cnt) {
                const int s0 = k * kBatchChunk, s1 = std::min(ns, s0 + kBatchChunk);
                const int f0 = b.finish_first[c][s0], f1 = b.finish_first[c][s1];
                return launch_batch_merge(kT[c], b.merge_chunks[k], b.at<int4>(b.off.mitems[c]) + i0, cnt,
                                          b.at<int2>(b.off.fin[c]) + f0, f1 - f0, s);
            });
            if (st != SHARP_OK) return st;
        }
    }
#undef CHUNKS
    return SHARP_OK;
}

extern "C" int sharp_batch_raar_iterate(sharp_batch b, int n, float beta) {
    if (!b || n < 0 || !(beta > 0.f && beta <= 1.f)) return SHARP_ERR_INVALID_ARG;
    if (!b->ws || b->ws_gen.size() != b->plans.size()) return SHARP_ERR_NOT_READY;
    for (size_t i = 0; i < b->plans.size(); ++i) {
        const sharp_plan_s* p = b->plans[i];
        // the launch arguments hold the workspace pointers recorded by
        // sharp_batch_set_workspace: a plan moved to another workspace since
        // would have its old buffers read and written
        if (p->ws_generation != b->ws_gen[i]) return SHARP_ERR_NOT_READY;
        if (!p->has_ws || !p->has_data || !p->has_probe || !p->has_object || p->gat_stale)
            return SHARP_ERR_NOT_READY;
    }
    if (n == 0) return SHARP_OK;
    BatchBegin bb{};
    bb.n = (int)b->plans.size();
    for (int s = 0; s < bb.n; ++s) {
        bb.g[s] = b->plans[s]->g;
        bb.hist[s] = (int)(b->plans[s]->hist_count % kHistCap);
        bb.gather[s] = b->plans[s]->stage_gather ? 0 : 1;
    }
    // order the batch stream after the caller's stream
    HIPCHK(hipEventRecord(b->ev_in, b->user));
    HIPCHK(hipStreamWaitEvent(b->own, b->ev_in, 0));
    HIPCHK(launch_batch_begin(b->at<FrameArgs>(b->off.fargs), b->at<EpsDesc>(b->off.eps), bb, beta, b->own));
    const auto key = std::make_pair(n, beta);
    auto it = b->graphs.find(key);
    if (it == b->graphs.end()) {
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        HIPCHK(hipStreamBeginCapture(b->own, hipStreamCaptureModeThreadLocal));
        int st = enqueue_iterations(*b, n, beta, b->own);
        hipError_t ec = hipStreamEndCapture(b->own, &g);
        if (st != SHARP_OK || ec != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return st != SHARP_OK ? st : SHARP_ERR_HIP;
        }
        if (hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(g);
            return SHARP_ERR_HIP;
        }
        it = b->graphs.emplace(key, std::make_pair(g, ge)).first;
    }
    HIPCHK(hipGraphLaunch(it->second.second, b->own));
    HIPCHK(hipEventRecord(b->ev_out, b->own));
    HIPCHK(hipStreamWaitEvent(b->user, b->ev_out, 0));
    for (sharp_plan_s* p : b->plans) {
        p->iter += n;
        p->hist_count += n;
        p->g = beta;
        p->last_probe_updated = false;
        p->stage_gather = p->strip_form() && !p->colg_form();
    }
    return SHARP_OK;
}
