// Continuous-batching serving loop over a magus_server.
//
// Telemetry events (samples, joins, leaves of simulated nodes) are ingested as
// they arrive; every dispatch forms one batch from the oldest pending sample
// of each live stream in a pinned host buffer of one of up to `depth` stages
// and launches the state-update kernel on a server-owned stream.  The kernel
// reads the batch and writes the decisions through the pinned buffers
// directly, so a batch costs one launch and no copy-engine round trips;
// batches of several stages are in flight at once, and the kernels stay in
// arrival order (a stream's state update of step k+1 needs the one of step
// k).  Joins are admitted while slots (the
// memory budget) allow, otherwise they wait for a leave; a leave closes the
// slot once the stream's pending samples are served.  A join for a node whose
// old slot is still draining is held until that slot closes, then queues like
// any join that waits.

#include <chrono>
#include <deque>

#include "host_internal.h"

using namespace magus;

namespace {

using Clock = std::chrono::steady_clock;

enum StreamState : uint8_t { kIdle = 0, kLive, kWaiting, kLeaving };

struct StreamRec {
    StreamState state = kIdle;
    uint32_t slot = 0;
    uint32_t cfg = 0;
    uint32_t in_flight = 0;          // dispatched samples not yet retired
    std::deque<uint64_t> fifo;       // pending sample events (indices)
    bool ready = false;              // listed in the ready list
    bool rejoin = false;             // a join arrived while leaving (kLeaving)
    uint32_t rejoin_cfg = 0;         // ... with this config
};

struct Batch {
    int stage = -1;
    std::vector<uint64_t> events;    // sample event of each pair
    std::vector<uint32_t> streams;
};

}  // namespace

extern "C" int magus_server_run(magus_server* srv, const magus_event* ev, uint64_t n_events,
                                uint32_t n_streams, const magus_config* h_cfgs,
                                uint32_t n_cfgs, int realtime, uint32_t max_batch,
                                uint32_t depth, uint8_t* h_decisions, uint64_t* h_latency_ns,
                                magus_run_stats* h_stats) {
    if (!srv || (n_events && !ev) || !h_decisions || !h_latency_ns || !h_stats)
        return fail(MAGUS_EINVAL, "NULL argument");
    if (n_cfgs && !h_cfgs) return fail(MAGUS_EINVAL, "configs are NULL");
    if (depth < 1 || depth > (uint32_t)magus_server::kLoopStages)
        return fail(MAGUS_EINVAL, "depth must be 1..%d", magus_server::kLoopStages);
    if (max_batch == 0) max_batch = srv->cap;
    for (uint64_t i = 0; i < n_events; ++i) {
        if (i && ev[i].t_ns < ev[i - 1].t_ns)
            return fail(MAGUS_EINVAL, "events not sorted by time at %llu", (unsigned long long)i);
        if (ev[i].stream >= n_streams)
            return fail(MAGUS_EINVAL, "event %llu: stream id out of range", (unsigned long long)i);
        if (ev[i].kind > MAGUS_EV_LEAVE)
            return fail(MAGUS_EINVAL, "event %llu: unknown kind", (unsigned long long)i);
        if (ev[i].kind == MAGUS_EV_JOIN && ev[i].value >= n_cfgs)
            return fail(MAGUS_EINVAL, "event %llu: config index out of range",
                        (unsigned long long)i);
    }
    for (uint32_t i = 0; i < n_cfgs; ++i) {
        DevCfg d;
        if (int rc = derive(&h_cfgs[i], &d)) return rc;
    }

    DeviceGuard g(srv->ctx->device);
    if (!g.ok) return fail(MAGUS_EDEVICE, "hipSetDevice failed");
    for (hipStream_t* q : {&srv->s_h2d, &srv->s_comp, &srv->s_d2h})
        if (!*q) HIP_TRY(hipStreamCreateWithFlags(q, hipStreamNonBlocking));
    for (uint32_t k = 0; k < depth; ++k) {
        auto& st = srv->loop_stages[k];
        for (hipEvent_t* e : {&st.done, &st.h2d, &st.kern})
            if (!*e) HIP_TRY(hipEventCreateWithFlags(e, hipEventDisableTiming));
        if (int rc = st.ensure(max_batch, 256, true)) return rc;
    }
    // the serving loop shares the pool with magus_serve_step: wait for it
    HIP_TRY(hipDeviceSynchronize());

    std::vector<StreamRec> rec(n_streams);
    std::deque<uint32_t> waiting;            // joins waiting for a slot
    std::vector<uint32_t> ready;             // streams with pending samples
    std::deque<Batch> flight;
    std::vector<int> free_stage;
    for (int k = (int)depth - 1; k >= 0; --k) free_stage.push_back(k);
    magus_run_stats st{};
    for (uint64_t i = 0; i < n_events; ++i) {
        h_decisions[i] = 0xFF;
        h_latency_ns[i] = UINT64_MAX;
    }

    const auto t0 = Clock::now();
    auto now_ns = [&]() {
        return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now() - t0)
            .count();
    };

    auto try_admit = [&](uint32_t sid) -> bool {
        uint32_t slot;
        if (magus_stream_open(srv, &h_cfgs[rec[sid].cfg], &slot) != MAGUS_OK) return false;
        rec[sid].slot = slot;
        rec[sid].state = kLive;
        return true;
    };
    auto close_stream = [&](uint32_t sid) -> int {
        StreamRec& r = rec[sid];
        if (int rc = magus_stream_close(srv, r.slot)) return rc;
        r.state = kIdle;
        if (r.rejoin) {                          // the node joined again meanwhile
            r.rejoin = false;
            r.cfg = r.rejoin_cfg;
            r.state = kWaiting;
            waiting.push_back(sid);
        }
        while (!waiting.empty()) {               // admit waiting joins, oldest first
            const uint32_t w = waiting.front();
            if (rec[w].state != kWaiting) {
                waiting.pop_front();
                continue;
            }
            if (!try_admit(w)) break;
            waiting.pop_front();
            ++st.joins_waited;
        }
        return MAGUS_OK;
    };
    auto maybe_close = [&](uint32_t sid) -> int {
        StreamRec& r = rec[sid];
        if (r.state == kLeaving && r.fifo.empty() && r.in_flight == 0) return close_stream(sid);
        return MAGUS_OK;
    };
    auto ingest = [&](uint64_t i) -> int {
        const magus_event& e = ev[i];
        StreamRec& r = rec[e.stream];
        switch (e.kind) {
        case MAGUS_EV_JOIN:
            if (r.state == kLeaving) {           // its old slot is still draining
                r.rejoin = true;
                r.rejoin_cfg = e.value;
                break;
            }
            if (r.state != kIdle) break;         // already live or waiting
            r.cfg = e.value;
            if (try_admit(e.stream)) {
                ++st.joins_admitted;
            } else {
                r.state = kWaiting;
                waiting.push_back(e.stream);
            }
            break;
        case MAGUS_EV_LEAVE:
            if (r.state == kWaiting) {
                r.state = kIdle;                 // never admitted
                ++st.joins_refused;
            } else if (r.state == kLeaving && r.rejoin) {
                r.rejoin = false;                // the held join is withdrawn
                ++st.joins_refused;
            } else if (r.state == kLive) {
                r.state = kLeaving;
                return maybe_close(e.stream);
            }
            break;
        default:                                 // sample
            if (r.state != kLive) {
                ++st.samples_dropped;
                break;
            }
            r.fifo.push_back(i);
            if (!r.ready) {
                r.ready = true;
                ready.push_back(e.stream);
            }
            break;
        }
        return MAGUS_OK;
    };

    auto dispatch = [&]() -> int {
        const int k = free_stage.back();
        free_stage.pop_back();
        auto& S = srv->loop_stages[k];
        if (int rc = S.ensure(max_batch, (uint32_t)srv->pending.size(), true)) return rc;
        Batch b;
        b.stage = k;
        // one sample per ready stream, oldest first
        std::vector<uint32_t> still;
        still.reserve(ready.size());
        for (uint32_t sid : ready) {
            StreamRec& r = rec[sid];
            if ((uint32_t)b.events.size() >= max_batch) {
                still.push_back(sid);
                continue;
            }
            const uint64_t i = r.fifo.front();
            r.fifo.pop_front();
            S.h_pairs[b.events.size()] = r.slot;
            b.events.push_back(i);
            b.streams.push_back(sid);
            ++r.in_flight;
            if (!r.fifo.empty()) {
                still.push_back(sid);
                ++st.deferred;
            } else {
                r.ready = false;
            }
        }
        ready.swap(still);
        const uint32_t n = (uint32_t)b.events.size();
        for (uint32_t j = 0; j < n; ++j) S.h_pairs[n + j] = ev[b.events[j]].value;
        const uint32_t n_inits = (uint32_t)srv->pending.size();
        uint32_t q = 0;
        for (const auto& kv : srv->pending) {
            S.h_inits[q].slot = kv.first;
            S.h_inits[q].pad = 0;
            S.h_inits[q].cfg = kv.second;
            ++q;
        }
        srv->pending.clear();
        // the kernel reads the batch (slot inits, pairs) from the stage's
        // pinned host buffers and writes the decisions back into pinned host
        // memory: no copy-engine round trips between arrival and decision
        magus_ctx::Timing tp(srv->ctx, MAGUS_KERNEL_SERVE);
        HIP_TRY(launch_serve(srv->st.as<SlotState>(), srv->acc.as<SlotAcc>(),
                             srv->slot_cfg.as<DevCfg>(), S.h_inits, n_inits, S.h_pairs, n,
                             S.h_dec, srv->s_comp, tp.first, tp.second));
        tp.commit();
        HIP_TRY(hipEventRecord(S.done, srv->s_comp));
        ++st.batches;
        st.max_batch = std::max<uint64_t>(st.max_batch, n);
        flight.push_back(std::move(b));
        st.max_in_flight = std::max<uint64_t>(st.max_in_flight, flight.size());
        return MAGUS_OK;
    };

    auto retire = [&](bool block) -> int {
        while (!flight.empty()) {
            Batch& b = flight.front();
            auto& S = srv->loop_stages[b.stage];
            hipError_t q = block ? hipEventSynchronize(S.done) : hipEventQuery(S.done);
            if (q == hipErrorNotReady) return MAGUS_OK;
            if (q != hipSuccess) return fail(MAGUS_EDEVICE, "serving batch: %s", hipGetErrorString(q));
            const uint64_t t = now_ns();
            for (size_t j = 0; j < b.events.size(); ++j) {
                const uint64_t i = b.events[j];
                h_decisions[i] = S.h_dec[j];
                const uint64_t arrive = realtime ? ev[i].t_ns : 0;
                h_latency_ns[i] = t > arrive ? t - arrive : 0;
                ++st.samples_served;
                const uint32_t sid = b.streams[j];
                --rec[sid].in_flight;
                if (int rc = maybe_close(sid)) return rc;
            }
            free_stage.push_back(b.stage);
            flight.pop_front();
            block = false;
        }
        return MAGUS_OK;
    };

    uint64_t pos = 0;
    int rc = MAGUS_OK;
    while (rc == MAGUS_OK && (pos < n_events || !ready.empty() || !flight.empty())) {
        const uint64_t t = realtime ? now_ns() : UINT64_MAX;
        // ingest what has arrived (flat-out: only as much as a batch needs)
        while (rc == MAGUS_OK && pos < n_events && ev[pos].t_ns <= t &&
               (realtime || ready.size() < (size_t)max_batch))
            rc = ingest(pos++);
        if (rc) break;
        rc = retire(false);
        if (rc) break;
        if (!ready.empty() && !free_stage.empty())
            rc = dispatch();
        else if (!flight.empty() && (free_stage.empty() || !realtime))
            rc = retire(true);      // every stage busy, or nothing else to do flat-out
        // real time with nothing to do: spin until the next arrival or completion
    }
    if (rc == MAGUS_OK) rc = retire(true);
    // the run owns the streams it admitted: close those still open
    for (uint32_t sid = 0; sid < n_streams; ++sid) {
        if (rec[sid].state == kWaiting || (rec[sid].state == kLeaving && rec[sid].rejoin))
            ++st.joins_refused;
        if (rec[sid].state == kLive || rec[sid].state == kLeaving) {
            (void)magus_stream_close(srv, rec[sid].slot);
            rec[sid].state = kIdle;
        }
    }
    st.wall_s = (double)now_ns() * 1e-9;
    *h_stats = st;
    if (rc != MAGUS_OK) (void)hipDeviceSynchronize();
    return rc;
}
