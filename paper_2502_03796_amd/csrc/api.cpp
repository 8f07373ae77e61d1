// Host side of libmagus: the C ABI declared in magus.h.
//
// Validates arguments, derives the kernel form of each controller config,
// owns per-context scratch memory and the serving slot pool, and enqueues the
// kernels of replay.hip, sweep.hip and serve.hip on the caller's stream.

#include "host_internal.h"
#include "proxy_internal.h"

using namespace magus;

namespace magus {

namespace {
thread_local std::string g_last_error;
constexpr uint32_t kDefaultChunk = 4096;
constexpr uint32_t kProxyChunkMax = 16384;   // longest chunk the fused proxy pass doubles to
}  // namespace

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

const std::string& last_error() { return g_last_error; }

int derive(const magus_config* c, DevCfg* d) {
    if (!c) return fail(MAGUS_EINVAL, "config is NULL");
    if (c->window < 2 || c->window > 32)
        return fail(MAGUS_EINVAL, "window %u outside 2..32", (unsigned)c->window);
    if (c->hold < 1 || c->hold > 32)
        return fail(MAGUS_EINVAL, "hold %u outside 1..32", (unsigned)c->hold);
    if (c->inc_q16 < 0 || c->inc_q16 > (1 << 20))
        return fail(MAGUS_EINVAL, "inc_q16 %d outside 0..2^20", c->inc_q16);
    if (c->dec_q16 > 0 || c->dec_q16 < -(1 << 20))
        return fail(MAGUS_EINVAL, "dec_q16 %d outside -2^20..0", c->dec_q16);
    if (c->hf_den == 0 || c->hf_num > c->hf_den)
        return fail(MAGUS_EINVAL, "high_freq_threshold %u/%u not in [0, 1]",
                    (unsigned)c->hf_num, (unsigned)c->hf_den);
    if (c->level_min >= c->level_max || c->level_max > 31)
        return fail(MAGUS_EINVAL, "levels need min < max <= 31 (got %u, %u)",
                    (unsigned)c->level_min, (unsigned)c->level_max);
    if (c->level_init < c->level_min || c->level_init > c->level_max)
        return fail(MAGUS_EINVAL, "level_init %u outside [min, max]", (unsigned)c->level_init);
    if (c->up_step > 31 || c->down_step > 31)
        return fail(MAGUS_EINVAL, "step sizes must be 0..31 (got %u, %u)",
                    (unsigned)c->up_step, (unsigned)c->down_step);
    if (c->base > 3) return fail(MAGUS_EINVAL, "base %u is not 0..3", (unsigned)c->base);
    if (c->base == 3 && c->base_ref == 0)
        return fail(MAGUS_EINVAL, "base 3 (fixed reference) needs base_ref >= 1");
    d->W = c->window;
    d->H = c->hold;
    d->mu = (uint32_t)c->window * (uint32_t)c->inc_q16;
    d->md = (uint32_t)c->window * (uint32_t)(-c->dec_q16);
    d->ref = c->base == 3 ? c->base_ref : 0u;
    d->pad = 0;
    d->thr = (uint16_t)(((uint32_t)c->hf_num * c->hold + c->hf_den - 1) / c->hf_den);
    d->up = c->up_step;
    d->down = c->down_step;
    d->lmin = c->level_min;
    d->lmax = c->level_max;
    d->linit = c->level_init;
    d->base = c->base;
    return MAGUS_OK;
}

int DevBuf::ensure(size_t bytes) {
    if (bytes <= cap) return MAGUS_OK;
    if (p) {
        hipError_t e = hipFree(p);
        p = nullptr;
        cap = 0;
        if (e != hipSuccess) return fail(MAGUS_EDEVICE, "hipFree: %s", hipGetErrorString(e));
    }
    size_t want = std::max(bytes, (size_t)256);
    if (hipMalloc(&p, want) != hipSuccess) {
        p = nullptr;
        return fail(MAGUS_ENOMEM, "hipMalloc(%zu) failed", want);
    }
    cap = want;
    return MAGUS_OK;
}

void DevBuf::release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
}

thread_local std::vector<hipGraphNode_t>* capture_marks = nullptr;

hipError_t record_timing_event(hipEvent_t ev, hipStream_t stream) {
    if (!ev) return hipSuccess;
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(stream, &st);
    if (e != hipSuccess) return e;
    if (st == hipStreamCaptureStatusNone) return hipEventRecord(ev, stream);
    if (st != hipStreamCaptureStatusActive) return hipErrorStreamCaptureInvalidated;
    unsigned long long id = 0;
    hipGraph_t graph = nullptr;
    const hipGraphNode_t* deps = nullptr;
    size_t n_deps = 0;
    e = hipStreamGetCaptureInfo_v2(stream, &st, &id, &graph, &deps, &n_deps);
    hipGraphNode_t node = nullptr;
    if (e == hipSuccess) e = hipGraphAddEventRecordNode(&node, graph, deps, n_deps, ev);
    if (e == hipSuccess)
        e = hipStreamUpdateCaptureDependencies(stream, &node, 1, hipStreamSetCaptureDependencies);
    if (e == hipSuccess && capture_marks) capture_marks->push_back(node);
    return e;
}

}  // namespace magus

magus_ctx::Timing::Timing(magus_ctx* c, int k) : ctx(c), kernel(k) {
    if (!ctx->prof) return;
    hipEvent_t e[2] = {nullptr, nullptr};
    for (auto& ev : e) {
        if (!ctx->ev_pool.empty()) {
            ev = ctx->ev_pool.back();
            ctx->ev_pool.pop_back();
        } else if (hipEventCreate(&ev) != hipSuccess) {
            ev = nullptr;
        }
    }
    if (!e[0] || !e[1]) {
        for (auto ev : e)
            if (ev) ctx->ev_pool.push_back(ev);
        return;
    }
    first = e[0];
    second = e[1];
}

void magus_ctx::Timing::commit() {
    if (first) ctx->recorded[kernel].push_back({first, second});
    first = second = nullptr;
}

magus_ctx::Timing::~Timing() {
    if (first) {
        ctx->ev_pool.push_back(first);
        ctx->ev_pool.push_back(second);
    }
}

void magus_ctx::harvest(GraphEntry& e, int i) {
    if (!e.pending[i]) return;
    e.pending[i] = false;
    float ms = 0.f;
    hipError_t err = hipEventSynchronize(e.ev[i][1]);
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e.ev[i][0], e.ev[i][1]);
    if (err != hipSuccess) {
        graph_timing_error = err;
        return;
    }
    graph_ms += ms;
    ++graph_launches;
}

void magus_ctx::destroy_graph(GraphEntry& e) {
    for (int i = 0; i < kGraphRing; ++i) {
        harvest(e, i);
        if (e.exec[i]) (void)hipGraphExecDestroy(e.exec[i]);
        for (auto ev : e.ev[i])
            if (ev) (void)hipEventDestroy(ev);
    }
    if (e.graph) (void)hipGraphDestroy(e.graph);
}

void magus_ctx::drop_graphs() {
    for (auto& e : graphs) destroy_graph(e);
    graphs.clear();
}

int magus_server::Stage::ensure(uint32_t n_pairs, uint32_t n_inits, bool with_h_dec) {
    using magus::fail;
    if (cap_pairs < n_pairs) {
        if (h_pairs) (void)hipHostFree(h_pairs);
        if (h_dec) (void)hipHostFree(h_dec);
        h_pairs = nullptr;
        h_dec = nullptr;
        cap_pairs = 0;
        const uint32_t c = std::max<uint32_t>(n_pairs, 1024);
        if (hipHostMalloc((void**)&h_pairs, (size_t)c * 8, hipHostMallocDefault) != hipSuccess)
            return fail(MAGUS_ENOMEM, "hipHostMalloc(%zu) failed", (size_t)c * 8);
        if (with_h_dec &&
            hipHostMalloc((void**)&h_dec, (size_t)c, hipHostMallocDefault) != hipSuccess)
            return fail(MAGUS_ENOMEM, "hipHostMalloc(%zu) failed", (size_t)c);
        int rc;
        if ((rc = d_pairs.ensure((size_t)c * 8)) || (rc = d_dec.ensure(c))) return rc;
        cap_pairs = c;
    }
    if (cap_inits < n_inits) {
        if (h_inits) (void)hipHostFree(h_inits);
        h_inits = nullptr;
        cap_inits = 0;
        const uint32_t c = std::max<uint32_t>(n_inits, 256);
        if (hipHostMalloc((void**)&h_inits, (size_t)c * sizeof(magus::ServeInit),
                          hipHostMallocDefault) != hipSuccess)
            return fail(MAGUS_ENOMEM, "hipHostMalloc failed");
        int rc;
        if ((rc = d_inits.ensure((size_t)c * sizeof(magus::ServeInit)))) return rc;
        cap_inits = c;
    }
    return MAGUS_OK;
}

void magus_server::Stage::release() {
    if (h_pairs) (void)hipHostFree(h_pairs);
    if (h_inits) (void)hipHostFree(h_inits);
    if (h_dec) (void)hipHostFree(h_dec);
    h_pairs = nullptr;
    h_inits = nullptr;
    h_dec = nullptr;
    d_pairs.release();
    d_inits.release();
    d_dec.release();
    for (hipEvent_t* e : {&done, &h2d, &kern})
        if (*e) {
            (void)hipEventDestroy(*e);
            *e = nullptr;
        }
    cap_pairs = cap_inits = 0;
    used = false;
}

extern "C" {

const char* magus_version(void) { return "magus-mi355x 0.1 (gfx950)"; }

const char* magus_last_error(void) { return last_error().c_str(); }

int magus_config_check(const magus_config* h_cfg) {
    DevCfg d;
    return derive(h_cfg, &d);
}

int magus_ctx_create(int device, magus_ctx** out) {
    if (!out) return fail(MAGUS_EINVAL, "out is NULL");
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n)
        return fail(MAGUS_EINVAL, "no HIP device %d (%d visible)", device, n);
    DeviceGuard g(device);
    if (!g.ok) return fail(MAGUS_EDEVICE, "hipSetDevice(%d) failed", device);
    magus_ctx* c = new magus_ctx();
    c->device = device;
    int rc = c->err.ensure(256);
    if (rc == MAGUS_OK && hipMemset(c->err.p, 0, 256) != hipSuccess)
        rc = fail(MAGUS_EDEVICE, "hipMemset failed");
    if (rc != MAGUS_OK) {
        c->err.release();
        delete c;
        return rc;
    }
    *out = c;
    return MAGUS_OK;
}

int magus_ctx_destroy(magus_ctx* ctx) {
    if (!ctx) return MAGUS_OK;
    {
        DeviceGuard g(ctx->device);
        (void)hipDeviceSynchronize();
        for (DevBuf* b : {&ctx->err, &ctx->chunk_base, &ctx->sums, &ctx->fix, &ctx->cfgs,
                          &ctx->keys, &ctx->sweep_tab, &ctx->step_funcs, &ctx->step_enter,
                          &ctx->step_sums, &ctx->step_masks, &ctx->status,
                          &ctx->proxy_model, &ctx->proxy_sums, &ctx->proxy_redo})
            b->release();
        for (auto& r : ctx->recorded)
            for (auto& pr : r) {
                (void)hipEventDestroy(pr.first);
                (void)hipEventDestroy(pr.second);
            }
        for (auto ev : ctx->ev_pool) (void)hipEventDestroy(ev);
        ctx->drop_graphs();
        for (auto ev : ctx->graph_ev)
            if (ev) (void)hipEventDestroy(ev);
        if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    }
    delete ctx;
    return MAGUS_OK;
}

int magus_ctx_set_chunk(magus_ctx* ctx, uint32_t chunk_steps) {
    if (!ctx) return fail(MAGUS_EINVAL, "ctx is NULL");
    if (chunk_steps == 0) chunk_steps = kDefaultChunk;
    if (chunk_steps % 64 || chunk_steps > (1u << 24))
        return fail(MAGUS_EINVAL, "chunk %u is not a multiple of 64 in 64..2^24", chunk_steps);
    ctx->chunk = chunk_steps;
    return MAGUS_OK;
}

uint32_t magus_ctx_get_chunk(const magus_ctx* ctx) { return ctx ? ctx->chunk : 0; }

int magus_ctx_set_profiling(magus_ctx* ctx, int enable) {
    if (!ctx) return fail(MAGUS_EINVAL, "ctx is NULL");
    ctx->prof = enable != 0;
    return MAGUS_OK;
}

int magus_ctx_kernel_time(magus_ctx* ctx, int kernel, double* total_ms, uint64_t* launches) {
    if (!ctx || !total_ms || !launches) return fail(MAGUS_EINVAL, "NULL argument");
    if (kernel < 0 || kernel > 3) return fail(MAGUS_EINVAL, "unknown kernel id %d", kernel);
    DeviceGuard g(ctx->device);
    double sum = 0.0;
    uint64_t n = 0;
    int rc = MAGUS_OK;
    for (auto& pr : ctx->recorded[kernel]) {
        float ms = 0.f;
        if (rc == MAGUS_OK) {
            hipError_t e = hipEventSynchronize(pr.second);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, pr.first, pr.second);
            if (e != hipSuccess)
                rc = fail(MAGUS_EDEVICE, "event timing: %s", hipGetErrorString(e));
        }
        sum += ms;
        ++n;
        ctx->ev_pool.push_back(pr.first);
        ctx->ev_pool.push_back(pr.second);
    }
    ctx->recorded[kernel].clear();
    if (kernel == MAGUS_KERNEL_REPLAY) {
        // the graph launches: their instances' own event pairs
        for (auto& e : ctx->graphs)
            for (int i = 0; i < magus_ctx::kGraphRing; ++i) ctx->harvest(e, i);
        sum += ctx->graph_ms;
        n += ctx->graph_launches;
        ctx->graph_ms = 0.0;
        ctx->graph_launches = 0;
        if (ctx->graph_timing_error != hipSuccess && rc == MAGUS_OK)
            rc = fail(MAGUS_EDEVICE, "graph event timing: %s",
                      hipGetErrorString(ctx->graph_timing_error));
        ctx->graph_timing_error = hipSuccess;
    }
    *total_ms = sum;
    *launches = n;
    return rc;
}

int magus_ctx_check(magus_ctx* ctx, hipStream_t stream) {
    if (!ctx) return fail(MAGUS_EINVAL, "ctx is NULL");
    DeviceGuard g(ctx->device);
    HIP_TRY(hipStreamSynchronize(stream));
    uint32_t e = 0;
    HIP_TRY(hipMemcpy(&e, ctx->err.p, 4, hipMemcpyDeviceToHost));
    if (e) {
        HIP_TRY(hipMemset(ctx->err.p, 0, 4));
        return fail(MAGUS_EDATA, "device data check failed:%s%s%s",
                    (e & kErrOffsets) ? " offsets not monotone or beyond n_samples" : "",
                    (e & kErrTooLong) ? " trace longer than MAGUS_MAX_TRACE_LEN" : "",
                    (e & kErrCfgIndex) ? " cfg_of_trace index out of range" : "");
    }
    return MAGUS_OK;
}

namespace {

// Validates h_cfgs (skipped when they equal the previous call's), makes sure the
// device table holds their kernel form (uploaded on `stream` when changed) and
// reports whether any config is stepped or uses another derivative base.
int stage_configs(magus_ctx* ctx, const magus_config* h_cfgs, uint32_t n_cfgs,
                  hipStream_t stream, bool* stepped, bool* any_base) {
    const bool same = ctx->cfg_raw.size() == n_cfgs &&
                      std::memcmp(ctx->cfg_raw.data(), h_cfgs,
                                  (size_t)n_cfgs * sizeof(magus_config)) == 0;
    std::vector<DevCfg> fresh;
    if (!same) {
        fresh.resize(n_cfgs);
        for (uint32_t i = 0; i < n_cfgs; ++i) {
            int rc = derive(&h_cfgs[i], &fresh[i]);
            if (rc != MAGUS_OK)
                return fail(rc, "config %u: %s", i, std::string(last_error()).c_str());
        }
    }
    const std::vector<DevCfg>& tab = same ? ctx->cfg_host : fresh;
    *stepped = false;
    *any_base = false;
    for (const DevCfg& d : tab) {
        *stepped |= d.up || d.down;
        *any_base |= d.base != 0;
    }
    const void* before = ctx->cfgs.p;
    int rc;
    if ((rc = ctx->cfgs.ensure((size_t)n_cfgs * sizeof(DevCfg)))) return rc;
    if (ctx->cfgs.p != before) ctx->drop_graphs();
    if (!same || ctx->cfgs.p != before) {
        // pageable source: the runtime stages it before returning
        HIP_TRY(hipMemcpyAsync(ctx->cfgs.p, tab.data(), tab.size() * sizeof(DevCfg),
                               hipMemcpyHostToDevice, stream));
        if (!same) {
            ctx->cfg_host = fresh;
            ctx->cfg_raw.assign(h_cfgs, h_cfgs + n_cfgs);
        }
    }
    return MAGUS_OK;
}

}  // namespace

int magus_replay(magus_ctx* ctx, const uint32_t* d_samples, uint64_t n_samples,
                 const uint64_t* d_offsets, uint32_t n_traces, const magus_config* h_cfgs,
                 uint32_t n_cfgs, const uint32_t* d_cfg_of_trace, magus_result* d_results,
                 uint8_t* d_levels, hipStream_t stream) {
    if (!ctx) return fail(MAGUS_EINVAL, "ctx is NULL");
    if (!h_cfgs || n_cfgs == 0) return fail(MAGUS_EINVAL, "need at least one config");
    if (n_traces && (!d_offsets || !d_results))
        return fail(MAGUS_EINVAL, "offsets and results are required");
    if (n_samples && !d_samples) return fail(MAGUS_EINVAL, "samples is NULL");
    if (n_traces > (1u << 30)) return fail(MAGUS_EINVAL, "too many traces");
    if (n_traces == 0) {
        // nothing to run; the configs are still validated
        for (uint32_t i = 0; i < n_cfgs; ++i) {
            DevCfg d;
            int rc = derive(&h_cfgs[i], &d);
            if (rc != MAGUS_OK)
                return fail(rc, "config %u: %s", i, std::string(last_error()).c_str());
        }
        return MAGUS_OK;
    }
    const uint64_t max_chunks64 = n_samples / ctx->chunk + n_traces + 1;
    if (max_chunks64 > 0xFFFFFFF0ull) return fail(MAGUS_EINVAL, "batch too large for one call");
    const uint32_t max_chunks = (uint32_t)max_chunks64;

    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(MAGUS_EDEVICE, "hipSetDevice(%d) failed", ctx->device);
    // configs identical to the previous call's are neither re-validated nor
    // re-uploaded
    bool stepped = false, any_base = false;
    int rc = stage_configs(ctx, h_cfgs, n_cfgs, stream, &stepped, &any_base);
    if (rc != MAGUS_OK) return rc;
    const void* before[7] = {ctx->chunk_base.p, ctx->sums.p, ctx->fix.p, ctx->step_funcs.p,
                             ctx->step_enter.p, ctx->step_sums.p, ctx->step_masks.p};
    if ((rc = ctx->chunk_base.ensure(((size_t)n_traces + 2) * 4))) return rc;
    if (stepped) {
        if ((rc = ctx->step_funcs.ensure((size_t)max_chunks * sizeof(ClampAdd))) ||
            (rc = ctx->step_enter.ensure((size_t)max_chunks * 4)) ||
            (rc = ctx->step_sums.ensure((size_t)max_chunks * sizeof(StepSum))) ||
            (rc = ctx->step_masks.ensure((size_t)stepped_mask_blocks(n_samples, n_traces) *
                                         (3 * sizeof(uint64_t) + sizeof(uint32_t)))))
            return rc;
    } else {
        if ((rc = ctx->sums.ensure((size_t)max_chunks * sizeof(ChunkSum)))) return rc;
        if (d_levels && (rc = ctx->fix.ensure((size_t)max_chunks * sizeof(ChunkFix)))) return rc;
    }
    const void* after[7] = {ctx->chunk_base.p, ctx->sums.p, ctx->fix.p, ctx->step_funcs.p,
                            ctx->step_enter.p, ctx->step_sums.p, ctx->step_masks.p};
    if (std::memcmp(before, after, sizeof before) != 0) ctx->drop_graphs();
    auto launch = [&](hipStream_t q, hipEvent_t e0, hipEvent_t e1) {
        if (stepped)
            return launch_replay_stepped(
                d_samples, n_samples, d_offsets, n_traces, ctx->cfgs.as<DevCfg>(), n_cfgs,
                d_cfg_of_trace, ctx->chunk, ctx->chunk_base.as<uint32_t>(), max_chunks,
                ctx->step_funcs.as<ClampAdd>(), ctx->step_enter.as<uint32_t>(),
                ctx->step_sums.as<StepSum>(), ctx->step_masks.as<uint64_t>(), d_results,
                d_levels, ctx->err.as<uint32_t>(), any_base, q, e0, e1);
        return launch_replay(d_samples, n_samples, d_offsets, n_traces, ctx->cfgs.as<DevCfg>(),
                             n_cfgs, d_cfg_of_trace, ctx->chunk, ctx->chunk_base.as<uint32_t>(),
                             ctx->sums.as<ChunkSum>(), max_chunks,
                             d_levels ? ctx->fix.as<ChunkFix>() : nullptr, d_results, d_levels,
                             ctx->err.as<uint32_t>(), ctx->persistent_blocks, any_base, q, e0,
                             e1);
    };
    if (!ctx->use_graphs) {
        magus_ctx::Timing tp(ctx, MAGUS_KERNEL_REPLAY);
        HIP_TRY(launch(stream, tp.first, tp.second));
        tp.commit();
        return MAGUS_OK;
    }
    // hipGraph path: the kernels of a call with these exact arguments are
    // captured once and relaunched
    const std::vector<uint64_t> key = {
        (uint64_t)d_samples, n_samples, (uint64_t)d_offsets, n_traces, n_cfgs,
        (uint64_t)d_cfg_of_trace, (uint64_t)d_results, (uint64_t)d_levels, ctx->chunk,
        ctx->persistent_blocks, (uint64_t)ctx->cfgs.p, (uint64_t)ctx->chunk_base.p,
        (uint64_t)ctx->sums.p, (uint64_t)ctx->fix.p, (uint64_t)stepped, (uint64_t)any_base,
        (uint64_t)ctx->step_funcs.p, (uint64_t)ctx->step_enter.p, (uint64_t)ctx->step_sums.p,
        (uint64_t)ctx->step_masks.p};
    magus_ctx::GraphEntry* entry = nullptr;
    for (size_t i = 0; i < ctx->graphs.size(); ++i)
        if (ctx->graphs[i].key == key) {
            std::rotate(ctx->graphs.begin() + i, ctx->graphs.begin() + i + 1, ctx->graphs.end());
            entry = &ctx->graphs.back();       // the hit was rotated to the back
            break;
        }
    if (!entry) {
        if (!ctx->cap_stream)
            HIP_TRY(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
        for (auto& ev : ctx->graph_ev)
            if (!ev) HIP_TRY(hipEventCreate(&ev));
        // the chunk kernel is bracketed by two event-record nodes; every
        // instance points them at a pair of events of its own
        std::vector<hipGraphNode_t> marks;
        HIP_TRY(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
        magus::capture_marks = &marks;
        const hipError_t le = launch(ctx->cap_stream, ctx->graph_ev[0], ctx->graph_ev[1]);
        magus::capture_marks = nullptr;
        hipGraph_t graph = nullptr;
        const hipError_t ce = hipStreamEndCapture(ctx->cap_stream, &graph);
        if (le != hipSuccess || ce != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return fail(MAGUS_EDEVICE, "graph capture (%s): %s",
                        le != hipSuccess ? "launch" : "end",
                        hipGetErrorString(le != hipSuccess ? le : ce));
        }
        if (marks.size() != 2) {
            (void)hipGraphDestroy(graph);
            return fail(MAGUS_EDEVICE, "graph capture: %zu timing nodes instead of 2",
                        marks.size());
        }
        magus_ctx::GraphEntry fresh;
        fresh.key = key;
        fresh.graph = graph;
        hipError_t ge = hipSuccess;
        for (int i = 0; i < magus_ctx::kGraphRing && ge == hipSuccess; ++i) {
            ge = hipGraphInstantiate(&fresh.exec[i], graph, nullptr, nullptr, 0);
            for (int k = 0; k < 2 && ge == hipSuccess; ++k) {
                ge = hipEventCreate(&fresh.ev[i][k]);
                if (ge == hipSuccess)
                    ge = hipGraphExecEventRecordNodeSetEvent(fresh.exec[i], marks[k],
                                                             fresh.ev[i][k]);
            }
        }
        if (ge != hipSuccess) {
            ctx->destroy_graph(fresh);
            return fail(MAGUS_EDEVICE, "graph instantiate: %s", hipGetErrorString(ge));
        }
        if (ctx->graphs.size() >= 8) {
            ctx->destroy_graph(ctx->graphs.front());
            ctx->graphs.erase(ctx->graphs.begin());
        }
        ctx->graphs.push_back(fresh);
        entry = &ctx->graphs.back();
    }
    // the next instance; its previous launch's events are read first if that
    // launch was timed (by then it has long finished unless the host is a
    // whole ring of launches ahead)
    const int i = entry->next;
    entry->next = (i + 1) % magus_ctx::kGraphRing;
    ctx->harvest(*entry, i);
    HIP_TRY(hipGraphLaunch(entry->exec[i], stream));
    entry->pending[i] = ctx->prof;
    return MAGUS_OK;
}

int magus_proxy_model_check(const magus_proxy_model* model) {
    if (!model) return fail(MAGUS_EINVAL, "model is NULL");
    const magus_proxy_model& m = *model;
    if (m.n_levels < 1 || m.n_levels > MAGUS_PROXY_LEVELS)
        return fail(MAGUS_EINVAL, "model n_levels %u outside 1..%d", m.n_levels,
                    MAGUS_PROXY_LEVELS);
    if (m.interval_us < 1) return fail(MAGUS_EINVAL, "model interval_us must be >= 1");
    for (uint32_t i = 0; i < m.n_levels; ++i) {
        if (m.cap_mbps[i] < 1) return fail(MAGUS_EINVAL, "model cap_mbps[%u] must be >= 1", i);
        if ((uint64_t)m.core_mw + m.uncore_mw[i] < 1)
            return fail(MAGUS_EINVAL, "model package power at level %u is 0", i);
    }
    return MAGUS_OK;
}

int magus_proxy(magus_ctx* ctx, const uint32_t* d_samples, uint64_t n_samples,
                const uint64_t* d_offsets, uint32_t n_traces, const magus_config* h_cfgs,
                uint32_t n_cfgs, const uint32_t* d_cfg_of_trace,
                const magus_proxy_model* h_model, magus_proxy_stats* d_stats,
                magus_proxy_metrics* d_metrics, hipStream_t stream) {
    if (!ctx) return fail(MAGUS_EINVAL, "ctx is NULL");
    int rc = magus_proxy_model_check(h_model);
    if (rc != MAGUS_OK) return rc;
    const magus_proxy_model& m = *h_model;
    if (!h_cfgs || n_cfgs == 0) return fail(MAGUS_EINVAL, "need at least one config");
    for (uint32_t i = 0; i < n_cfgs; ++i)
        if (h_cfgs[i].level_max >= m.n_levels)
            return fail(MAGUS_EINVAL, "config %u: level_max %u not described by the model "
                        "(%u levels)", i, (unsigned)h_cfgs[i].level_max, m.n_levels);
    if (n_traces && !d_stats) return fail(MAGUS_EINVAL, "stats is NULL");
    if (n_traces == 0) return magus_replay(ctx, d_samples, n_samples, d_offsets, 0, h_cfgs,
                                           n_cfgs, d_cfg_of_trace, nullptr, nullptr, stream);
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(MAGUS_EDEVICE, "hipSetDevice(%d) failed", ctx->device);
    if ((rc = ctx->proxy_model.ensure(sizeof(magus_proxy_model)))) return rc;
    const uint64_t max_chunks64 = n_samples / ctx->chunk + n_traces + 1;
    if (max_chunks64 > 0xFFFFFFF0ull) return fail(MAGUS_EINVAL, "batch too large for one call");
    const uint32_t max_chunks = (uint32_t)max_chunks64;
    if (n_samples && !d_samples) return fail(MAGUS_EINVAL, "samples is NULL");
    if (!d_offsets) return fail(MAGUS_EINVAL, "offsets is NULL");
    if (n_traces > (1u << 30)) return fail(MAGUS_EINVAL, "too many traces");
    bool stepped = false, any_base = false;
    if ((rc = stage_configs(ctx, h_cfgs, n_cfgs, stream, &stepped, &any_base))) return rc;
    if (!ctx->proxy_model_set ||
        std::memcmp(&ctx->proxy_model_host, &m, sizeof m) != 0) {
        ctx->proxy_model_host = m;
        HIP_TRY(hipMemcpyAsync(ctx->proxy_model.p, &ctx->proxy_model_host, sizeof m,
                               hipMemcpyHostToDevice, stream));
        ctx->proxy_model_set = true;
    }
    if (!stepped) {
        // one pass over the samples: plan, fused chunk pass, fold, metrics;
        // a config that starts between the bounds needs the pass's third
        // prefix total
        bool mid_init = false;
        for (const DevCfg& d : ctx->cfg_host) mid_init |= d.linit != d.lmin && d.linit != d.lmax;
        // the fused pass ends each chunk with more per-chunk work than the
        // replay (seven wave sums): it takes chunks of twice the context's
        // length up to 16,384 steps
        const uint32_t pchunk = ctx->chunk <= kProxyChunkMax / 2 ? 2 * ctx->chunk : ctx->chunk;
        const uint32_t pmax_chunks = (uint32_t)(n_samples / pchunk + n_traces + 1);
        const void* before = ctx->chunk_base.p;
        const void* redo_before = ctx->proxy_redo.p;
        if ((rc = ctx->chunk_base.ensure(((size_t)n_traces + 2) * 4)) ||
            (rc = ctx->proxy_sums.ensure((size_t)max_chunks * sizeof(ProxySum))) ||
            (rc = ctx->proxy_redo.ensure(((size_t)max_chunks + 1) * 4)))
            return rc;
        if (ctx->chunk_base.p != before) ctx->drop_graphs();
        // the exact pass's queue starts empty: its count is cleared once
        // when the buffer is new, and after a call that did not reach its
        // fold (every completed call leaves it at 0)
        if (ctx->proxy_redo.p != redo_before || !ctx->proxy_redo_zero) {
            HIP_TRY(launch_proxy_queue_clear(ctx->proxy_redo.as<uint32_t>(), stream));
            ctx->proxy_redo_zero = true;
        }
        HIP_TRY(launch_plan(d_offsets, n_traces, n_samples, d_cfg_of_trace, n_cfgs, pchunk,
                            pmax_chunks, ctx->chunk_base.as<uint32_t>(), ctx->err.as<uint32_t>(),
                            stream));
        ctx->proxy_redo_zero = false;
        HIP_TRY(launch_proxy_fused(d_samples, d_offsets, n_traces, ctx->chunk_base.as<uint32_t>(),
                                   pmax_chunks, ctx->cfgs.as<DevCfg>(), d_cfg_of_trace, pchunk,
                                   ctx->proxy_model.as<magus_proxy_model>(),
                                   ctx->proxy_sums.as<ProxySum>(),
                                   ctx->proxy_redo.as<uint32_t>(), d_stats, d_metrics, any_base,
                                   mid_init, stream));
        ctx->proxy_redo_zero = true;
        return MAGUS_OK;
    }
    // stepped actuation: pass 1 of the stepped replay (plan, step masks, the
    // level entering every chunk), then one pass over samples and masks
    const void* before[5] = {ctx->chunk_base.p, ctx->step_funcs.p, ctx->step_enter.p,
                             ctx->step_sums.p, ctx->step_masks.p};
    if ((rc = ctx->chunk_base.ensure(((size_t)n_traces + 2) * 4)) ||
        (rc = ctx->step_funcs.ensure((size_t)max_chunks * sizeof(ClampAdd))) ||
        (rc = ctx->step_enter.ensure((size_t)max_chunks * 4)) ||
        (rc = ctx->step_sums.ensure((size_t)max_chunks * sizeof(StepSum))) ||
        (rc = ctx->step_masks.ensure((size_t)stepped_mask_blocks(n_samples, n_traces) *
                                     (3 * sizeof(uint64_t) + sizeof(uint32_t)))) ||
        (rc = ctx->proxy_redo.ensure(((size_t)max_chunks + 1) * 4)))
        return rc;
    const void* after[5] = {ctx->chunk_base.p, ctx->step_funcs.p, ctx->step_enter.p,
                            ctx->step_sums.p, ctx->step_masks.p};
    if (std::memcmp(before, after, sizeof before) != 0) ctx->drop_graphs();
    HIP_TRY(launch_stepped_prepare(d_samples, n_samples, d_offsets, n_traces,
                                   ctx->cfgs.as<DevCfg>(), n_cfgs, d_cfg_of_trace, ctx->chunk,
                                   ctx->chunk_base.as<uint32_t>(), max_chunks,
                                   ctx->step_funcs.as<ClampAdd>(), ctx->step_enter.as<uint32_t>(),
                                   ctx->step_sums.as<StepSum>(), ctx->step_masks.as<uint64_t>(),
                                   ctx->err.as<uint32_t>(), any_base, stream));
    // the statistics pass's per-lane excess bins cover the widest level range
    uint32_t bin_levels = 0;
    for (const DevCfg& d : ctx->cfg_host) bin_levels = std::max(bin_levels, d.lmax - d.lmin + 1u);
    // this path clears the wide pass's queue before it runs and leaves it
    // filled (also when a launch fails part-way): a single-pass call clears
    // it first
    ctx->proxy_redo_zero = false;
    HIP_TRY(launch_proxy_stepped(d_samples, n_samples, d_offsets, n_traces,
                                 ctx->chunk_base.as<uint32_t>(), max_chunks,
                                 ctx->cfgs.as<DevCfg>(), d_cfg_of_trace, ctx->chunk,
                                 ctx->step_enter.as<uint32_t>(), ctx->step_masks.as<uint64_t>(),
                                 ctx->proxy_model.as<magus_proxy_model>(), d_stats, d_metrics,
                                 bin_levels, ctx->proxy_redo.as<uint32_t>(), stream));
    return MAGUS_OK;
}

int magus_ctx_set_persistent(magus_ctx* ctx, uint32_t blocks) {
    if (!ctx) return fail(MAGUS_EINVAL, "ctx is NULL");
    if (blocks > (1u << 20)) return fail(MAGUS_EINVAL, "too many persistent workgroups");
    ctx->persistent_blocks = blocks;
    return MAGUS_OK;
}

uint32_t magus_ctx_get_persistent(const magus_ctx* ctx) { return ctx ? ctx->persistent_blocks : 0; }

int magus_ctx_set_graphs(magus_ctx* ctx, int enable) {
    if (!ctx) return fail(MAGUS_EINVAL, "ctx is NULL");
    ctx->use_graphs = enable != 0;
    if (!ctx->use_graphs) {
        DeviceGuard g(ctx->device);
        ctx->drop_graphs();
    }
    return MAGUS_OK;
}

int magus_autotune_replay(magus_ctx* ctx, const uint32_t* d_samples, uint64_t n_samples,
                          const uint64_t* d_offsets, uint32_t n_traces,
                          const magus_config* h_cfgs, uint32_t n_cfgs,
                          const uint32_t* d_cfg_of_trace, magus_result* d_results,
                          uint32_t reps, hipStream_t stream, magus_tune_result* out) {
    if (!ctx || !out) return fail(MAGUS_EINVAL, "ctx/out is NULL");
    if (n_traces == 0) return fail(MAGUS_EINVAL, "nothing to tune on");
    if (reps == 0) reps = 3;
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(MAGUS_EDEVICE, "hipSetDevice(%d) failed", ctx->device);
    int n_cu = 0;
    HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, ctx->device));
    const uint32_t chunks[] = {2048, 4096, 8192, 16384, 32768};
    const uint32_t pers[] = {0, (uint32_t)n_cu * 4, (uint32_t)n_cu * 8};
    const uint32_t keep_chunk = ctx->chunk, keep_pers = ctx->persistent_blocks;
    const bool keep_graphs = ctx->use_graphs;
    ctx->use_graphs = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    std::vector<magus_result> ref(n_traces), got(n_traces);
    magus_tune_result best{};
    best.best_ms = 1e300;
    int rc = MAGUS_OK;
    uint32_t cand = 0;
    for (uint32_t ch : chunks) {
        for (uint32_t pb : pers) {
            ctx->chunk = ch;
            ctx->persistent_blocks = pb;
            // warm-up call, then the results of every candidate must agree
            rc = magus_replay(ctx, d_samples, n_samples, d_offsets, n_traces, h_cfgs, n_cfgs,
                              d_cfg_of_trace, d_results, nullptr, stream);
            if (rc) break;
            if ((rc = magus_ctx_check(ctx, stream))) break;
            if (hipMemcpy(cand ? got.data() : ref.data(), d_results,
                          (size_t)n_traces * sizeof(magus_result),
                          hipMemcpyDeviceToHost) != hipSuccess) {
                rc = fail(MAGUS_EDEVICE, "result copy failed");
                break;
            }
            if (cand && std::memcmp(got.data(), ref.data(),
                                    (size_t)n_traces * sizeof(magus_result)) != 0) {
                rc = fail(MAGUS_EDEVICE, "autotune: candidate chunk %u / persistent %u changed "
                                         "the results", ch, pb);
                break;
            }
            (void)hipEventRecord(e0, stream);
            for (uint32_t r = 0; r < reps && rc == MAGUS_OK; ++r)
                rc = magus_replay(ctx, d_samples, n_samples, d_offsets, n_traces, h_cfgs, n_cfgs,
                                  d_cfg_of_trace, d_results, nullptr, stream);
            if (rc) break;
            (void)hipEventRecord(e1, stream);
            float ms = 0.f;
            if (hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                rc = fail(MAGUS_EDEVICE, "autotune timing failed");
                break;
            }
            const double per = ms / reps;
            if (ch == kDefaultChunk && pb == 0) best.default_ms = per;
            if (per < best.best_ms) {
                best.best_ms = per;
                best.chunk_steps = ch;
                best.persistent_blocks = pb;
            }
            ++cand;
        }
        if (rc) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->use_graphs = keep_graphs;
    if (rc) {
        ctx->chunk = keep_chunk;
        ctx->persistent_blocks = keep_pers;
        return rc;
    }
    best.candidates = cand;
    ctx->chunk = best.chunk_steps;
    ctx->persistent_blocks = best.persistent_blocks;
    *out = best;
    return MAGUS_OK;
}

int magus_sweep(magus_ctx* ctx, const uint32_t* d_samples, uint64_t n_samples,
                const uint64_t* d_offsets, uint32_t n_traces, const magus_config* h_cfgs,
                uint32_t n_cfgs, uint64_t* d_scores, uint32_t* d_argmin, hipStream_t stream) {
    if (!ctx) return fail(MAGUS_EINVAL, "ctx is NULL");
    if (!h_cfgs || n_cfgs == 0) return fail(MAGUS_EINVAL, "need at least one config");
    if (n_cfgs > (1u << 23)) return fail(MAGUS_EINVAL, "at most 2^23 configs per sweep");
    if (n_traces && (!d_offsets || !d_argmin))
        return fail(MAGUS_EINVAL, "offsets and argmin are required");
    if (n_samples && !d_samples) return fail(MAGUS_EINVAL, "samples is NULL");
    // configs identical to the previous sweep's keep their lane tables
    const bool same = ctx->sweep_cfg_host.size() == n_cfgs &&
                      std::memcmp(ctx->sweep_cfg_host.data(), h_cfgs,
                                  (size_t)n_cfgs * sizeof(magus_config)) == 0;
    std::vector<DevCfg> tab;
    if (!same) {
        tab.resize(n_cfgs);
        for (uint32_t i = 0; i < n_cfgs; ++i) {
            int rc = derive(&h_cfgs[i], &tab[i]);
            if (rc != MAGUS_OK)
                return fail(rc, "config %u: %s", i, std::string(last_error()).c_str());
        }
    }
    if (n_traces == 0) return MAGUS_OK;

    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(MAGUS_EDEVICE, "hipSetDevice(%d) failed", ctx->device);
    if (!same) {
        // Group configs by window into blocks of kSweepLanes lanes.
        std::vector<uint32_t> order(n_cfgs);
        for (uint32_t i = 0; i < n_cfgs; ++i) order[i] = i;
        // blocks share the window, the base and (base 3) the reference
        auto wkey = [&](uint32_t i) {
            return (uint64_t)tab[i].ref << 32 | tab[i].W | ((uint32_t)tab[i].base << 8);
        };
        std::stable_sort(order.begin(), order.end(),
                         [&](uint32_t a, uint32_t b) { return wkey(a) < wkey(b); });
        std::vector<uint32_t> bw, bref;
        std::vector<int32_t> inc, dec;
        std::vector<uint32_t> hmask, thr, lv, orig, steps, bstep;
        size_t i = 0;
        while (i < order.size()) {
            const uint64_t W = wkey(order[i]);
            bw.push_back((uint32_t)W);
            bref.push_back((uint32_t)(W >> 32));
            uint32_t any_step = 0;
            for (int l = 0; l < kSweepLanes; ++l) {
                if (i < order.size() && wkey(order[i]) == W) {
                    const DevCfg& d = tab[order[i]];
                    inc.push_back(h_cfgs[order[i]].inc_q16);
                    dec.push_back(h_cfgs[order[i]].dec_q16);
                    hmask.push_back(d.H >= 32 ? 0xFFFFFFFFu : ((1u << d.H) - 1u));
                    thr.push_back(d.thr);
                    lv.push_back(d.lmin | (d.lmax << 8) | (d.linit << 16));
                    orig.push_back(order[i]);
                    steps.push_back(d.up | ((uint32_t)d.down << 8));
                    any_step |= d.up | d.down;
                    ++i;
                } else {   // padding lane: never predicts, never reported
                    inc.push_back(INT32_MAX);
                    dec.push_back(INT32_MIN);
                    hmask.push_back(1u);
                    thr.push_back(1u);
                    lv.push_back(0u | (1u << 8));
                    orig.push_back(0xFFFFFFFFu);
                    steps.push_back(0u);
                }
            }
            bstep.push_back(any_step ? 1u : 0u);
        }
        const uint32_t nb = (uint32_t)bw.size();
        if ((uint64_t)nb * n_traces >= (1ull << 31))
            return fail(MAGUS_EINVAL, "traces x config blocks too large for one call");
        const size_t nl = (size_t)nb * kSweepLanes;
        const size_t bytes = nb * 4 * 3 + nl * 4 * 7 + 10 * 256;
        int rc;
        if ((rc = ctx->sweep_tab.ensure(bytes))) return rc;
        std::vector<uint8_t> host(bytes, 0);
        size_t off = 0;
        auto put = [&](const void* src, size_t n) {
            size_t at = off;
            std::memcpy(host.data() + at, src, n);
            off += (n + 255) & ~(size_t)255;
            return at;
        };
        size_t o_bw = put(bw.data(), nb * 4), o_bref = put(bref.data(), nb * 4), o_inc = put(inc.data(), nl * 4),
               o_dec = put(dec.data(), nl * 4), o_hm = put(hmask.data(), nl * 4),
               o_thr = put(thr.data(), nl * 4), o_lv = put(lv.data(), nl * 4),
               o_orig = put(orig.data(), nl * 4), o_steps = put(steps.data(), nl * 4),
               o_bstep = put(bstep.data(), nb * 4);
        HIP_TRY(hipMemcpyAsync(ctx->sweep_tab.p, host.data(), off, hipMemcpyHostToDevice, stream));
        char* base = ctx->sweep_tab.as<char>();
        ctx->plan.n_blocks = nb;
        ctx->plan.block_w = reinterpret_cast<const uint32_t*>(base + o_bw);
        ctx->plan.block_ref = reinterpret_cast<const uint32_t*>(base + o_bref);
        ctx->plan.lane_inc = reinterpret_cast<const int32_t*>(base + o_inc);
        ctx->plan.lane_dec = reinterpret_cast<const int32_t*>(base + o_dec);
        ctx->plan.lane_hmask = reinterpret_cast<const uint32_t*>(base + o_hm);
        ctx->plan.lane_thr = reinterpret_cast<const uint32_t*>(base + o_thr);
        ctx->plan.lane_lv = reinterpret_cast<const uint32_t*>(base + o_lv);
        ctx->plan.lane_orig = reinterpret_cast<const uint32_t*>(base + o_orig);
        ctx->plan.lane_steps = reinterpret_cast<const uint32_t*>(base + o_steps);
        ctx->plan.block_stepped = reinterpret_cast<const uint32_t*>(base + o_bstep);
        ctx->sweep_cfg_host.assign(h_cfgs, h_cfgs + n_cfgs);
    }
    const uint32_t parts = kSweepLanes / kSweepShapes[ctx->sweep_shape].lanes;
    if ((uint64_t)ctx->plan.n_blocks * n_traces * parts >= (1ull << 31))
        return fail(MAGUS_EINVAL, "traces x config blocks too large for one call");
    int rc;
    if ((rc = ctx->keys.ensure(((size_t)n_traces + 1) * 8))) return rc;
    magus_ctx::Timing tp(ctx, MAGUS_KERNEL_SWEEP);
    HIP_TRY(launch_sweep(d_samples, n_samples, d_offsets, n_traces, ctx->plan, n_cfgs, d_scores,
                         d_argmin, ctx->keys.as<uint64_t>(), ctx->err.as<uint32_t>(),
                         ctx->sweep_shape, stream, tp.first, tp.second));
    tp.commit();
    return MAGUS_OK;
}

int magus_ctx_set_sweep_shape(magus_ctx* ctx, uint32_t shape) {
    if (!ctx) return fail(MAGUS_EINVAL, "ctx is NULL");
    if (shape >= kSweepShapeCount)
        return fail(MAGUS_EINVAL, "sweep shape %u outside 0..%u", shape, kSweepShapeCount - 1);
    ctx->sweep_shape = shape;
    return MAGUS_OK;
}

uint32_t magus_ctx_get_sweep_shape(const magus_ctx* ctx) { return ctx ? ctx->sweep_shape : 0; }

int magus_sweep_shape_info(uint32_t shape, uint32_t* lanes, uint32_t* tile) {
    if (shape >= kSweepShapeCount)
        return fail(MAGUS_EINVAL, "sweep shape %u outside 0..%u", shape, kSweepShapeCount - 1);
    if (lanes) *lanes = kSweepShapes[shape].lanes;
    if (tile) *tile = kSweepShapes[shape].tile;
    return MAGUS_OK;
}

int magus_autotune_sweep(magus_ctx* ctx, const uint32_t* d_samples, uint64_t n_samples,
                         const uint64_t* d_offsets, uint32_t n_traces,
                         const magus_config* h_cfgs, uint32_t n_cfgs, uint32_t* d_argmin,
                         uint32_t reps, hipStream_t stream, magus_sweep_tune_result* h_out) {
    if (!ctx || !h_out) return fail(MAGUS_EINVAL, "ctx and out are required");
    if (n_traces == 0 || reps == 0) return fail(MAGUS_EINVAL, "need traces and reps >= 1");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(MAGUS_EDEVICE, "hipSetDevice(%d) failed", ctx->device);
    const uint32_t saved = ctx->sweep_shape;
    hipEvent_t ev[2] = {nullptr, nullptr};
    std::vector<uint64_t> first(n_traces), keys(n_traces);
    magus_sweep_tune_result r{};
    double best = 0.0;
    int rc = MAGUS_OK;
    for (auto& e : ev)
        if (rc == MAGUS_OK && hipEventCreate(&e) != hipSuccess)
            rc = fail(MAGUS_EDEVICE, "hipEventCreate failed");
    for (uint32_t shape = 0; rc == MAGUS_OK && shape < kSweepShapeCount; ++shape) {
        ctx->sweep_shape = shape;
        // one untimed call (it also builds the lane tables on the first shape)
        if ((rc = magus_sweep(ctx, d_samples, n_samples, d_offsets, n_traces, h_cfgs, n_cfgs,
                              nullptr, d_argmin, stream)))
            break;
        if (hipEventRecord(ev[0], stream) != hipSuccess) {
            rc = fail(MAGUS_EDEVICE, "hipEventRecord failed");
            break;
        }
        for (uint32_t k = 0; rc == MAGUS_OK && k < reps; ++k)
            rc = magus_sweep(ctx, d_samples, n_samples, d_offsets, n_traces, h_cfgs, n_cfgs,
                             nullptr, d_argmin, stream);
        float ms = 0.f;
        uint32_t status = 0;
        if (rc == MAGUS_OK &&
            (hipEventRecord(ev[1], stream) != hipSuccess ||
             hipEventSynchronize(ev[1]) != hipSuccess ||
             hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess ||
             hipMemcpy(keys.data(), ctx->keys.p, (size_t)n_traces * 8,
                       hipMemcpyDeviceToHost) != hipSuccess ||
             hipMemcpy(&status, ctx->keys.as<uint64_t>() + n_traces, 4,
                       hipMemcpyDeviceToHost) != hipSuccess))
            rc = fail(MAGUS_EDEVICE, "timing sweep shape %u failed", shape);
        if (rc != MAGUS_OK) break;
        if (status != 0) {
            rc = fail(MAGUS_EDATA, "the batch failed its data checks");
            break;
        }
        // every shape must find the same minimal score and config per trace
        if (shape == 0) {
            first = keys;
        } else if (keys != first) {
            rc = fail(MAGUS_EDEVICE, "sweep shape %u gives results unlike shape 0", shape);
            break;
        }
        const double per = (double)ms / reps;
        if (shape == 0) r.default_ms = per;
        if (shape == 0 || per < best) {
            best = per;
            r.shape = shape;
        }
        ++r.candidates;
    }
    for (auto e : ev)
        if (e) (void)hipEventDestroy(e);
    if (rc != MAGUS_OK) {
        ctx->sweep_shape = saved;
        return rc;
    }
    ctx->sweep_shape = r.shape;
    r.lanes = kSweepShapes[r.shape].lanes;
    r.tile = kSweepShapes[r.shape].tile;
    r.best_ms = best;
    *h_out = r;
    return MAGUS_OK;
}

int magus_valu_probe(magus_ctx* ctx, uint32_t workgroups, uint32_t steps, uint32_t mode,
                     uint32_t* d_out, uint64_t* h_lane_ops, hipStream_t stream) {
    if (!ctx) return fail(MAGUS_EINVAL, "ctx is NULL");
    if (workgroups == 0 || steps == 0 || steps % 4 || mode > 1 || !d_out)
        return fail(MAGUS_EINVAL,
                    "need workgroups >= 1, steps a positive multiple of 4, mode 0 or 1, out");
    if (h_lane_ops)
        *h_lane_ops = (uint64_t)workgroups * kSweepLanes * steps * valu_probe_ops_per_step(mode);
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(MAGUS_EDEVICE, "hipSetDevice(%d) failed", ctx->device);
    magus_ctx::Timing tp(ctx, MAGUS_KERNEL_PROBE);
    HIP_TRY(launch_valu_probe(workgroups, steps, mode, 0x5A17u, d_out, stream, tp.first,
                              tp.second));
    tp.commit();
    return MAGUS_OK;
}

int magus_read_probe(magus_ctx* ctx, const uint32_t* d_samples, uint64_t n_samples,
                     uint32_t chunk_steps, uint32_t* d_out, hipStream_t stream) {
    if (!ctx) return fail(MAGUS_EINVAL, "ctx is NULL");
    if (chunk_steps == 0 || chunk_steps % 64 || chunk_steps > (1u << 24))
        return fail(MAGUS_EINVAL, "chunk %u is not a multiple of 64 in 64..2^24", chunk_steps);
    if (n_samples && (!d_samples || !d_out)) return fail(MAGUS_EINVAL, "NULL buffer");
    if ((n_samples + chunk_steps - 1) / chunk_steps > 0xFFFFFFF0ull)
        return fail(MAGUS_EINVAL, "too many chunks");
    if (n_samples == 0) return MAGUS_OK;
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(MAGUS_EDEVICE, "hipSetDevice(%d) failed", ctx->device);
    magus_ctx::Timing tp(ctx, MAGUS_KERNEL_PROBE);
    HIP_TRY(launch_read_probe(d_samples, n_samples, chunk_steps, d_out, stream, tp.first,
                              tp.second));
    tp.commit();
    return MAGUS_OK;
}

int magus_counters_to_mbps(magus_ctx* ctx, const uint64_t* d_counts, const uint64_t* d_ts_ns,
                           uint64_t n_readings, const uint64_t* d_offsets, uint32_t n_traces,
                           uint32_t counter_bits, uint32_t bytes_per_count,
                           uint32_t* d_samples, hipStream_t stream) {
    if (!ctx) return fail(MAGUS_EINVAL, "ctx is NULL");
    if (counter_bits < 1 || counter_bits > 64)
        return fail(MAGUS_EINVAL, "counter_bits %u outside 1..64", counter_bits);
    if (n_traces && (!d_offsets || !d_samples || !d_counts || !d_ts_ns))
        return fail(MAGUS_EINVAL, "NULL argument");
    if (n_traces == 0 || n_readings == 0) return MAGUS_OK;
    if (n_readings / 256 >= 0xFFFFFFFFull) return fail(MAGUS_EINVAL, "too many readings");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(MAGUS_EDEVICE, "hipSetDevice(%d) failed", ctx->device);
    if (int rc = ctx->status.ensure(256)) return rc;
    HIP_TRY(launch_counters(d_counts, d_ts_ns, d_offsets, n_traces, n_readings, counter_bits,
                            bytes_per_count, ctx->status.as<uint32_t>(), ctx->err.as<uint32_t>(),
                            d_samples, stream));
    return MAGUS_OK;
}

// ------------------------------------------------------------------ serving

size_t magus_server_slot_bytes(void) {
    return sizeof(SlotState) + sizeof(SlotAcc) + sizeof(DevCfg);
}

int magus_server_create(magus_ctx* ctx, size_t mem_budget_bytes, magus_server** out) {
    if (!ctx || !out) return fail(MAGUS_EINVAL, "ctx/out is NULL");
    *out = nullptr;
    const size_t per = magus_server_slot_bytes();
    const size_t cap64 = mem_budget_bytes / per;
    if (cap64 == 0) return fail(MAGUS_ENOSLOT, "budget %zu B holds no slot (%zu B each)",
                                mem_budget_bytes, per);
    if (cap64 > (1u << 26)) return fail(MAGUS_EINVAL, "at most 2^26 slots");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(MAGUS_EDEVICE, "hipSetDevice(%d) failed", ctx->device);
    magus_server* s = new magus_server();
    s->ctx = ctx;
    s->cap = (uint32_t)cap64;
    int rc;
    if ((rc = s->st.ensure((size_t)s->cap * sizeof(SlotState))) ||
        (rc = s->acc.ensure((size_t)s->cap * sizeof(SlotAcc))) ||
        (rc = s->slot_cfg.ensure((size_t)s->cap * sizeof(DevCfg)))) {
        magus_server_destroy(s);
        return rc;
    }
    for (auto& st : s->stages) {
        if (hipEventCreateWithFlags(&st.done, hipEventDisableTiming) != hipSuccess) {
            magus_server_destroy(s);
            return fail(MAGUS_EDEVICE, "hipEventCreate failed");
        }
    }
    s->open.assign(s->cap, 0);
    s->host_cfg.resize(s->cap);
    s->mark.assign(s->cap, 0);
    s->free_slots.reserve(s->cap);
    for (uint32_t i = s->cap; i-- > 0;) s->free_slots.push_back(i);
    *out = s;
    return MAGUS_OK;
}

int magus_server_destroy(magus_server* s) {
    if (!s) return MAGUS_OK;
    {
        DeviceGuard g(s->ctx->device);
        (void)hipDeviceSynchronize();
        for (auto& st : s->stages) st.release();
        for (auto& st : s->loop_stages) st.release();
        for (hipStream_t* q : {&s->s_h2d, &s->s_comp, &s->s_d2h})
            if (*q) {
                (void)hipStreamDestroy(*q);
                *q = nullptr;
            }
        s->st.release();
        s->acc.release();
        s->slot_cfg.release();
    }
    delete s;
    return MAGUS_OK;
}

uint32_t magus_server_capacity(const magus_server* s) { return s ? s->cap : 0; }

uint32_t magus_server_open_count(const magus_server* s) {
    return s ? s->cap - (uint32_t)s->free_slots.size() : 0;
}

int magus_stream_open(magus_server* s, const magus_config* h_cfg, uint32_t* slot_out) {
    if (!s || !slot_out) return fail(MAGUS_EINVAL, "server/slot_out is NULL");
    DevCfg d;
    int rc = derive(h_cfg, &d);
    if (rc != MAGUS_OK) return rc;
    if (s->free_slots.empty())
        return fail(MAGUS_ENOSLOT, "all %u slots are in use", s->cap);
    const uint32_t slot = s->free_slots.back();
    s->free_slots.pop_back();
    s->open[slot] = 1;
    s->host_cfg[slot] = d;
    s->pending[slot] = d;
    *slot_out = slot;
    return MAGUS_OK;
}

int magus_stream_close(magus_server* s, uint32_t slot) {
    if (!s) return fail(MAGUS_EINVAL, "server is NULL");
    if (slot >= s->cap || !s->open[slot]) return fail(MAGUS_EINVAL, "slot %u is not open", slot);
    s->open[slot] = 0;
    s->pending.erase(slot);
    s->free_slots.push_back(slot);
    return MAGUS_OK;
}

int magus_serve_step(magus_server* s, const uint32_t* h_slots, const uint32_t* h_samples,
                     uint32_t n, uint8_t* h_decisions, hipStream_t stream) {
    if (!s) return fail(MAGUS_EINVAL, "server is NULL");
    if (n && (!h_slots || !h_samples || !h_decisions))
        return fail(MAGUS_EINVAL, "slots/samples/decisions is NULL");
    if (++s->epoch == 0) {
        std::fill(s->mark.begin(), s->mark.end(), 0);
        s->epoch = 1;
    }
    for (uint32_t i = 0; i < n; ++i) {
        const uint32_t slot = h_slots[i];
        if (slot >= s->cap || !s->open[slot])
            return fail(MAGUS_EINVAL, "pair %u: slot %u is not open", i, slot);
        if (s->mark[slot] == s->epoch)
            return fail(MAGUS_EINVAL, "pair %u: slot %u appears twice in one step", i, slot);
        s->mark[slot] = s->epoch;
    }
    const uint32_t n_inits = (uint32_t)s->pending.size();
    if (n == 0 && n_inits == 0) return MAGUS_OK;

    DeviceGuard g(s->ctx->device);
    if (!g.ok) return fail(MAGUS_EDEVICE, "hipSetDevice(%d) failed", s->ctx->device);
    magus_server::Stage& st = s->stages[s->next_stage];
    s->next_stage = (s->next_stage + 1) % magus_server::kStages;
    if (st.used) HIP_TRY(hipEventSynchronize(st.done));   // staging buffers free again
    if (int rc = st.ensure(n, n_inits, false)) return rc;
    uint32_t k = 0;
    for (const auto& kv : s->pending) {
        st.h_inits[k].slot = kv.first;
        st.h_inits[k].pad = 0;
        st.h_inits[k].cfg = kv.second;
        ++k;
    }
    std::memcpy(st.h_pairs, h_slots, (size_t)n * 4);
    std::memcpy(st.h_pairs + n, h_samples, (size_t)n * 4);
    // the kernel reads the pairs and slot inits from the pinned staging
    // buffers directly; the decisions come back with one copy (the caller's
    // buffer may be pageable)
    magus_ctx::Timing tp(s->ctx, MAGUS_KERNEL_SERVE);
    HIP_TRY(launch_serve(s->st.as<SlotState>(), s->acc.as<SlotAcc>(), s->slot_cfg.as<DevCfg>(),
                         st.h_inits, n_inits, st.h_pairs, n, st.d_dec.as<uint8_t>(), stream,
                         tp.first, tp.second));
    tp.commit();
    if (n)
        HIP_TRY(hipMemcpyAsync(h_decisions, st.d_dec.p, n, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipEventRecord(st.done, stream));
    st.used = true;
    s->pending.clear();
    return MAGUS_OK;
}

int magus_stream_result(magus_server* s, uint32_t slot, magus_result* h_out) {
    if (!s || !h_out) return fail(MAGUS_EINVAL, "server/out is NULL");
    if (slot >= s->cap || !s->open[slot]) return fail(MAGUS_EINVAL, "slot %u is not open", slot);
    if (s->pending.count(slot)) {       // opened, no step yet
        std::memset(h_out, 0, sizeof *h_out);
        return MAGUS_OK;
    }
    DeviceGuard g(s->ctx->device);
    HIP_TRY(hipDeviceSynchronize());
    SlotAcc a;
    HIP_TRY(hipMemcpy(&a, s->acc.as<SlotAcc>() + slot, sizeof a, hipMemcpyDeviceToHost));
    h_out->level_sum = a.level_sum;
    h_out->transitions = a.transitions;
    h_out->ticks_high = a.ticks_high;
    h_out->score = a.level_sum + 1000ull * a.transitions;
    return MAGUS_OK;
}

}  // extern "C"
