// Memory-throughput monitor front end on gfx950.
//
// MAGUS reads memory throughput through a counter API periodically (Sec. 3,
// Sec. 4): what the hardware exposes is a cumulative, wrapping traffic
// counter.  This kernel turns counter readings into the uint32 MB/s samples the
// controller consumes:
//   mbps = floor(((c[i+1] - c[i]) mod 2^bits) * bytes_per_count * 1000
//                / (ts[i+1] - ts[i]))          (bytes per microsecond = MB/s)
// saturated at 2^32-1, and 0 for a zero interval.  The product is formed in
// 128 bits, so the result is exact for every input.

#include "magus_internal.h"

namespace magus {
namespace {

__device__ __forceinline__ uint32_t rate_mbps(uint64_t dc, uint64_t dt, uint32_t bpc) {
    if (dt == 0) return 0;
    const uint64_t k = (uint64_t)bpc * 1000u;                 // < 2^42
    const uint64_t lo = dc * k, hi = __umul64hi(dc, k);       // p = hi:lo = dc * k
    if (hi == 0) {
        const uint64_t q = lo / dt;
        return q > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)q;
    }
    // p >= 2^64: saturate unless p < dt * 2^32
    const uint64_t th = dt >> 32, tl = dt << 32;
    if (hi > th || (hi == th && lo >= tl)) return 0xFFFFFFFFu;
    // quotient < 2^32: restoring division, one bit at a time
    uint64_t rh = hi, rl = lo;
    uint32_t q = 0;
    for (int b = 31; b >= 0; --b) {
        const uint64_t sh = b ? (dt >> (64 - b)) : 0, sl = dt << b;   // dt << b, 128-bit
        if (rh > sh || (rh == sh && rl >= sl)) {
            const uint64_t nl = rl - sl;
            rh = rh - sh - (rl < sl ? 1 : 0);
            rl = nl;
            q |= 1u << b;
        }
    }
    return q;
}

// One thread per reading; reading i of trace t (not its last) writes sample
// i - t, so trace t's samples start at offsets[t] - t.
__global__ __launch_bounds__(256) void counters_kernel(
    const uint64_t* __restrict__ counts, const uint64_t* __restrict__ ts,
    const uint64_t* __restrict__ offsets, uint32_t n_traces, uint64_t n_readings,
    uint32_t bits, uint32_t bpc, const uint32_t* __restrict__ status,
    uint32_t* __restrict__ out)
{
    __shared__ uint32_t s_t0, s_t1;
    if (status[0] != 0) return;
    const uint64_t first = (uint64_t)blockIdx.x * blockDim.x;
    const uint64_t last = min(first + blockDim.x, n_readings) - 1;
    if (first >= n_readings) return;
    if (threadIdx.x == 0) {
        // traces holding the first and the last reading of this block
        auto find = [&](uint64_t i) {
            uint32_t lo = 0, hi = n_traces;            // offsets[lo] <= i < offsets[hi]
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (offsets[mid] <= i) lo = mid; else hi = mid;
            }
            return lo;
        };
        s_t0 = find(first);
        s_t1 = find(last);
    }
    __syncthreads();
    const uint64_t i = first + threadIdx.x;
    if (i >= n_readings || i < offsets[0] || i >= offsets[n_traces]) return;
    uint32_t lo = s_t0, hi = s_t1 + 1;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (offsets[mid] <= i) lo = mid; else hi = mid;
    }
    const uint32_t t = lo;
    if (i + 1 >= offsets[t + 1]) return;               // last reading of the trace
    uint64_t dc = counts[i + 1] - counts[i];
    if (bits < 64) dc &= (1ull << bits) - 1ull;
    out[i - t] = rate_mbps(dc, ts[i + 1] - ts[i], bpc);
}

__global__ __launch_bounds__(1024) void counters_check_kernel(
    const uint64_t* __restrict__ offsets, uint32_t n_traces, uint64_t n_readings,
    uint32_t* __restrict__ status, uint32_t* __restrict__ err)
{
    __shared__ uint32_t s_err;
    if (threadIdx.x == 0) s_err = 0;
    __syncthreads();
    uint32_t e = 0;
    for (uint32_t t = threadIdx.x; t < n_traces; t += blockDim.x)
        if (offsets[t + 1] <= offsets[t] || offsets[t + 1] > n_readings) e |= kErrOffsets;
    if (e) atomicOr(&s_err, e);
    __syncthreads();
    if (threadIdx.x == 0) {
        status[0] = s_err;
        if (s_err) atomicOr(err, s_err);
    }
}

}  // namespace

hipError_t launch_counters(const uint64_t* counts, const uint64_t* ts, const uint64_t* offsets,
                           uint32_t n_traces, uint64_t n_readings, uint32_t bits, uint32_t bpc,
                           uint32_t* status, uint32_t* err, uint32_t* out, hipStream_t stream)
{
    if (n_traces == 0 || n_readings == 0) return hipSuccess;
    counters_check_kernel<<<1, 1024, 0, stream>>>(offsets, n_traces, n_readings, status, err);
    const uint64_t blocks = (n_readings + 255) / 256;
    counters_kernel<<<(uint32_t)blocks, 256, 0, stream>>>(counts, ts, offsets, n_traces,
                                                          n_readings, bits, bpc, status, out);
    return hipGetLastError();
}

}  // namespace magus
