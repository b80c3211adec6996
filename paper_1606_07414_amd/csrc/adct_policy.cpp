// Host policy of the library, free of HIP and of the GPU: status strings,
// the uneven batch's work-queue construction, and the server's pool
// allocator, admission rule and latency percentile (through the simulation
// entry points, which run the very code the server runs).  It is built into
// libadct.so and, alone, into a sanitizer-instrumented CPU library for
// testing.
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "adct.h"
#include "adct_serve_logic.hpp"

using namespace adct;

extern "C" {

const char* adct_strerror(int code) {
    switch (code) {
        case ADCT_OK: return "ok";
        case ADCT_PENDING: return "pending";
        case ADCT_E_ARG: return "invalid argument";
        case ADCT_E_SHAPE: return "plane sides must be positive multiples of 16 with a valid pitch";
        case ADCT_E_DTYPE: return "unsupported sample type";
        case ADCT_E_HIP: return "HIP runtime error";
        case ADCT_E_NOMEM: return "out of memory";
        case ADCT_E_TOO_LARGE: return "request larger than the available capacity";
        case ADCT_E_STOPPED: return "stopped";
        case ADCT_E_TIMEOUT: return "timed out";
        case ADCT_E_NOTFOUND: return "not found";
        case ADCT_E_ALIGN: return "pointer or pitch not 16-byte aligned";
        default: return "unknown status";
    }
}

int adct_work_queue(const int64_t* tiles_per_job, int32_t njobs, int32_t tiles_per_group, int32_t groups_per_item,
                    uint32_t* items, int64_t capacity, int64_t* n_items) {
    if (!tiles_per_job || njobs < 0 || !n_items || capacity < 0) return ADCT_E_ARG;
    if (tiles_per_group <= 0 || groups_per_item <= 0) return ADCT_E_ARG;
    const int64_t span = (int64_t)tiles_per_group * groups_per_item;
    int64_t n = 0;
    for (int32_t j = 0; j < njobs; ++j) {
        const int64_t t = tiles_per_job[j];
        if (t < 0 || t > (int64_t)INT32_MAX) return ADCT_E_ARG;
        for (int64_t first = 0; first < t; first += span) {
            if (items && n < capacity) {
                items[3 * n + 0] = (uint32_t)j;
                items[3 * n + 1] = (uint32_t)first;
                items[3 * n + 2] = (uint32_t)(t - first < span ? t - first : span);
            }
            ++n;
        }
    }
    *n_items = n;
    if (n > (int64_t)UINT32_MAX) return ADCT_E_TOO_LARGE;
    return (items && n > capacity) ? ADCT_E_TOO_LARGE : ADCT_OK;
}

int adct_pool_simulate(int64_t capacity, const int64_t* ops, int32_t nops, int64_t* out, int64_t* high_water) {
    if (!ops || !out || nops < 0 || capacity < 0) return ADCT_E_ARG;
    Pool pool(capacity);
    std::vector<int64_t> sizes((size_t)nops, 0);
    for (int32_t i = 0; i < nops; ++i) {
        if (ops[i] > 0) {
            out[i] = pool.alloc(ops[i]);
            if (out[i] >= 0) sizes[(size_t)i] = ops[i];
        } else {
            const int64_t j = -ops[i];
            if (j >= i || sizes[(size_t)j] == 0) return ADCT_E_ARG;
            pool.release(out[j], sizes[(size_t)j]);
            sizes[(size_t)j] = 0;
            out[i] = 0;
        }
    }
    if (high_water) *high_water = pool.high_water();
    return ADCT_OK;
}

int adct_admission_simulate(int64_t capacity, int32_t max_inflight, const int64_t* arrival, const int64_t* bytes,
                            const int64_t* hold, int32_t n, int64_t* admit) {
    if (!arrival || !bytes || !hold || !admit || n < 0 || max_inflight < 1) return ADCT_E_ARG;
    Pool pool(capacity);
    for (int32_t i = 0; i < n; ++i)
        if (!pool.fits_ever(bytes[i]) || hold[i] < 0) return ADCT_E_TOO_LARGE;
    std::vector<int64_t> off((size_t)n, -1), end((size_t)n, -1);
    int64_t head = 0, inflight = 0, now = n ? arrival[0] : 0;
    while (head < n) {
        head = admit_in_order(
            head, n, now, inflight, max_inflight, pool, [&](int64_t i) { return arrival[i]; },
            [&](int64_t i) { return bytes[i]; }, [](int64_t) { return false; },
            [&](int64_t i, int64_t o) {
                admit[i] = now;
                off[(size_t)i] = o;
                end[(size_t)i] = now + hold[i];
            });
        if (head >= n) break;
        // next event: the head's arrival or the earliest release
        int64_t next = arrival[head] > now ? arrival[head] : INT64_MAX;
        for (int64_t i = 0; i < head; ++i)
            if (off[(size_t)i] >= 0 && end[(size_t)i] > now) next = std::min(next, end[(size_t)i]);
        if (next == INT64_MAX) {
            // all admitted requests are due: release those ending now
            next = now;
        }
        now = next;
        for (int64_t i = 0; i < head; ++i) {
            if (off[(size_t)i] >= 0 && end[(size_t)i] <= now) {
                pool.release(off[(size_t)i], bytes[i]);
                off[(size_t)i] = -1;
                --inflight;
            }
        }
    }
    return ADCT_OK;
}

int adct_percentile(const double* v, int64_t n, double p, double* out) {
    if (!v || !out || n < 0 || !(p >= 0.0 && p <= 100.0)) return ADCT_E_ARG;
    *out = percentile(std::vector<double>(v, v + n), p);
    return ADCT_OK;
}

}  // extern "C"
