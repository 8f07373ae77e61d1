// Host-side internals of libmagus shared by the C ABI (api.cpp) and the
// serving loop (server_loop.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "magus_internal.h"

namespace magus {

// Records `fmt` as this thread's last error message and returns `code`.
int fail(int code, const char* fmt, ...);
const std::string& last_error();

#define HIP_TRY(expr)                                                                 \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            return ::magus::fail(MAGUS_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// Derives the kernel form of a config; MAGUS_OK or MAGUS_EINVAL.
int derive(const magus_config* c, DevCfg* d);

// Grow-only device buffer.
struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    int ensure(size_t bytes);
    void release();
    template <class T> T* as() const { return static_cast<T*>(p); }
};

// Restores the caller's current device on scope exit.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && hipSetDevice(dev) == hipSuccess) ok = true;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace magus

struct magus_ctx {
    int device = 0;
    uint32_t chunk = 4096;
    magus::DevBuf err;          // uint32 sticky error word
    magus::DevBuf chunk_base;   // replay: chunk prefix sum + status
    magus::DevBuf sums;         // replay: ChunkSum per chunk
    magus::DevBuf fix;          // replay: ChunkFix per chunk
    magus::DevBuf cfgs;         // replay: DevCfg table
    magus::DevBuf step_funcs;   // stepped replay: ClampAdd per chunk
    magus::DevBuf step_enter;   // stepped replay: entering level per chunk
    magus::DevBuf step_sums;    // stepped replay: StepSum per chunk
    magus::DevBuf step_masks;   // stepped replay: 28 B of step masks and map per block
    std::vector<magus::DevCfg> cfg_host;        // last uploaded table
    std::vector<magus_config> cfg_raw;          // ... and the configs it came from
    magus::DevBuf keys;         // sweep: arg-min keys + status
    magus::DevBuf status;       // front end: per-call status word
    magus::DevBuf sweep_tab;    // sweep: lane tables
    std::vector<magus_config> sweep_cfg_host;   // configs of the last sweep plan
    magus::SweepPlan plan{};
    uint32_t sweep_shape = 0;   // sweep launch shape (index into kSweepShapes)
    magus::DevBuf proxy_model;    // proxy: the model in device memory
    magus::DevBuf proxy_sums;     // proxy: per-chunk summaries of the fused pass
    magus::DevBuf proxy_redo;     // proxy: queue of the exact pass (count, chunk indices)
    bool proxy_redo_zero = false; // ... its count is known to be 0
    magus_proxy_model proxy_model_host{};   // ... as last uploaded
    bool proxy_model_set = false;
    // launch shape of the replay chunk kernel (0 = one wave per chunk)
    uint32_t persistent_blocks = 0;
    // hipGraph cache of replay calls
    bool use_graphs = false;
    hipStream_t cap_stream = nullptr;
    // A captured call is instantiated kGraphRing times; instance i's two
    // event-record nodes (around the chunk kernel) record into its own pair
    // of events, set once, and launches take the instances in turn, so no
    // node is re-pointed per launch.  A launch made while timing is on leaves
    // its instance `pending` until its pair is read (when the instance is
    // next launched, or by magus_ctx_kernel_time).
    static constexpr int kGraphRing = 8;
    struct GraphEntry {
        std::vector<uint64_t> key;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec[kGraphRing] = {};
        hipEvent_t ev[kGraphRing][2] = {};
        bool pending[kGraphRing] = {};
        int next = 0;
    };
    hipEvent_t graph_ev[2] = {nullptr, nullptr};      // record targets during capture
    std::vector<GraphEntry> graphs;          // most recent last
    double graph_ms = 0.0;                   // timed graph launches read so far
    uint64_t graph_launches = 0;
    hipError_t graph_timing_error = hipSuccess;
    void harvest(GraphEntry& e, int i);      // reads instance i's pair if pending
    void destroy_graph(GraphEntry& e);
    void drop_graphs();
    // kernel timing: event pairs recorded around the dominant kernel of a call
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> recorded[4];

    // A pair of events to record around one launch of `kernel` (nulls when
    // timing is off).  The pair counts for magus_ctx_kernel_time only once
    // commit() says the launch was queued; otherwise it returns to the pool.
    struct Timing {
        magus_ctx* ctx;
        int kernel;
        hipEvent_t first = nullptr, second = nullptr;
        Timing(magus_ctx* c, int k);
        Timing(const Timing&) = delete;
        Timing& operator=(const Timing&) = delete;
        void commit();
        ~Timing();
    };
};

struct magus_server {
    magus_ctx* ctx = nullptr;
    uint32_t cap = 0;
    magus::DevBuf st, acc, slot_cfg;
    std::vector<uint8_t> open;
    std::vector<magus::DevCfg> host_cfg;
    std::vector<uint32_t> free_slots;
    std::map<uint32_t, magus::DevCfg> pending;  // slots to (re)initialise at the next step
    std::vector<uint32_t> mark;                  // duplicate detection per step
    uint32_t epoch = 0;
    struct Stage {
        uint32_t* h_pairs = nullptr;
        magus::ServeInit* h_inits = nullptr;
        uint8_t* h_dec = nullptr;                // serving loop only
        uint32_t cap_pairs = 0, cap_inits = 0;
        magus::DevBuf d_pairs, d_inits, d_dec;
        hipEvent_t done = nullptr;
        hipEvent_t h2d = nullptr, kern = nullptr; // serving loop only
        bool used = false;
        int ensure(uint32_t n_pairs, uint32_t n_inits, bool with_h_dec);
        void release();
    };
    static constexpr int kStages = 3;
    Stage stages[kStages];
    uint32_t next_stage = 0;
    // serving loop
    static constexpr int kLoopStages = 4;
    Stage loop_stages[kLoopStages];
    hipStream_t s_h2d = nullptr, s_comp = nullptr, s_d2h = nullptr;
};
