// Uneven batches: one persistent launch over a device work queue, captured
// into a hipGraph, with an autotuner for the launch shape.
//
// The host cuts every image into items (runs of whole tile groups of one
// image, see adct_work_queue) and splits the item list into kQueues
// contiguous sub-queues, one per XCD: workgroups are dispatched to the XCDs
// round-robin, so workgroup w serves sub-queue w % kQueues first and keeps
// the atomics on each head (one 128-byte line per head) within one XCD's
// share of the traffic.  A workgroup claims items with one atomic per claim;
// when its sub-queue is empty it moves on to the others, and it exits after
// the last one is drained, so every workgroup terminates.  The per-image SSE
// of an item is reduced in registers and added with one atomic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "adct_core.hpp"
#include "adct_internal.hpp"

namespace adct {

struct ItemDev {
    uint32_t job, first, count;
};

constexpr uint32_t kQueues = 8;        // one sub-queue per XCD
constexpr uint32_t kHeadStride = 32;   // uint32 words between heads (128 bytes)

struct BatchArgs {
    const GroupArgs* jobs;         // per image: planes, outputs, scale factors
    const ItemDev* items;
    uint32_t qbeg[kQueues + 1];    // sub-queue q holds items [qbeg[q], qbeg[q+1])
    uint32_t* heads;               // next unclaimed item of each sub-queue
};

// Claims an item for this workgroup from sub-queue q, moving on through the
// following sub-queues while they are drained.  Returns false once every
// sub-queue is.  Called with uniform control flow.
__device__ __forceinline__ bool claim_item(const BatchArgs& b, uint32_t home, uint32_t& qi, uint32_t& q,
                                           uint32_t& c, uint32_t* sh_claim) {
    for (;;) {
        __syncthreads();  // every thread has read the previous claim
        if (threadIdx.x == 0) *sh_claim = atomicAdd(b.heads + q * kHeadStride, 1u);
        __syncthreads();
        c = __builtin_amdgcn_readfirstlane(*sh_claim);
        if (c < b.qbeg[q + 1] - b.qbeg[q]) return true;
        if (++qi >= kQueues) return false;
        q = (home + qi) % kQueues;
    }
}

// Items are software-pipelined: the claim of the next item is issued when an
// item starts, resolved before its last group, and that group's prefetch
// requests the first rows of the next item (possibly another image), so a
// workgroup's memory stream does not stall between items.
// `jobs` and `items` are read-only for the whole launch (restrict: their
// loads are scalar and are not repeated after the kernel's own stores).
template <int TPW, typename S, typename M>
__global__ __launch_bounds__(TPW * 8) void k_batch(BatchArgs b, const GroupArgs* __restrict__ jobs,
                                                   const ItemDev* __restrict__ items) {
    // the loop below loads each next group's sample rows itself; the zone
    // words of a zonal reconstruction are set up by group_chunk only
    static_assert(M::IN == kInSamples, "the batch codes samples");
    __shared__ uint32_t lds[lds_words(TPW)];
    __shared__ long long red[TPW * 8 / 64];
    __shared__ uint32_t sh_claim;
    const int tid = threadIdx.x;
    const uint32_t home = blockIdx.x % kQueues;
    uint32_t qi = 0, q = home, c = 0;
    if (!claim_item(b, home, qi, q, c, &sh_claim)) return;
    ItemDev item = items[b.qbeg[q] + c];
    RowWords rows;
    load_group_rows<TPW, S>(global_args(jobs[item.job]), item.first, min((uint32_t)TPW, item.count), rows);
    for (;;) {
        // claim the next item of this sub-queue now; the atomic's latency
        // overlaps this item's groups
        uint32_t next = 0;
        if (tid == 0) next = atomicAdd(b.heads + q * kHeadStride, 1u);
        const GroupArgs a = global_args(jobs[item.job]);
        const uint32_t gend = item.first + item.count;
        SseAcc acc{0, kNoImage};
        bool have_next = false;
        ItemDev nitem = item;
        for (uint32_t g0 = item.first; g0 < gend; g0 += (uint32_t)TPW) {
            // the previous group's LDS reads are done, also across items: the
            // last group of the previous item ends in LDS reads (its inverse
            // row pass) and the SSE flush between items, which would
            // otherwise order them, is skipped for jobs without an SSE output
            __syncthreads();
            uint32_t g0n = g0 + (uint32_t)TPW;
            uint32_t ntn = g0n < gend ? min((uint32_t)TPW, gend - g0n) : 0u;
            if (g0n >= gend) {
                // last group of the item: resolve the next claim, prefetch from it
                __syncthreads();  // every thread has read the previous claim
                if (tid == 0) sh_claim = next;
                __syncthreads();
                const uint32_t cn = __builtin_amdgcn_readfirstlane(sh_claim);
                if (cn < b.qbeg[q + 1] - b.qbeg[q]) {
                    nitem = items[b.qbeg[q] + cn];
                    have_next = true;
                    g0n = nitem.first;
                    ntn = min((uint32_t)TPW, nitem.count);
                }
            }
            // (the scale tables are read from the job array itself: indexed
            // reads of a private copy would go through scratch)
            process_group<TPW, S, M>(a, g0, min((uint32_t)TPW, gend - g0), lds, red, acc, rows,
                                     global_args(jobs[nitem.job]), g0n, ntn, jobs[item.job].qs, jobs[item.job].dqs);
        }
        if (a.sse) sse_flush<TPW * 8>(acc, a.sse, red);
        if (have_next) {
            item = nitem;
            continue;
        }
        // sub-queue q is drained: the following ones, without prefetch
        if (++qi >= kQueues) break;
        q = (home + qi) % kQueues;
        if (!claim_item(b, home, qi, q, c, &sh_claim)) break;
        item = items[b.qbeg[q] + c];
        __syncthreads();  // every thread is finished with LDS (sse_flush, last group)
        load_group_rows<TPW, S>(global_args(jobs[item.job]), item.first, min((uint32_t)TPW, item.count), rows);
    }
}

// Clears the queue head and every job's SSE slot (a kernel, not a memset,
// so that it can live in the captured graph).
__global__ __launch_bounds__(256) void k_batch_reset(uint32_t* heads, const GroupArgs* jobs, uint32_t njobs) {
    const uint32_t t = blockIdx.x * 256u + threadIdx.x;
    if (t < kQueues) heads[t * kHeadStride] = 0u;
    if (t < njobs && jobs[t].sse) *as_global(jobs[t].sse) = 0ull;
}

namespace {

int launched() { return hipGetLastError() == hipSuccess ? ADCT_OK : ADCT_E_HIP; }

template <int TPW, typename S, typename M>
void launch_k(unsigned grid, hipStream_t s, const BatchArgs& b) {
    hipLaunchKernelGGL((k_batch<TPW, S, M>), dim3(grid), dim3(TPW * 8), 0, s, b, b.jobs, b.items);
}

template <int TPW>
int launch_tpw(int dtype, int op, int param, unsigned grid, hipStream_t s, const BatchArgs& b) {
    if (op == ADCT_OP_QUANT) {
        using M = Mode<kInSamples, kStoreQ, kMidQuant, kOutSamples, -1, true>;
        if (dtype == ADCT_U8)
            launch_k<TPW, uint8_t, M>(grid, s, b);
        else
            launch_k<TPW, int16_t, M>(grid, s, b);
        return launched();
    }
    if (op == ADCT_OP_ZIGZAG) {
        using M = Mode<kInSamples, kStoreY, kMidZigzag, kOutSamples, -1, true>;
        if (dtype == ADCT_U8)
            launch_k<TPW, uint8_t, M>(grid, s, b);
        else
            launch_k<TPW, int16_t, M>(grid, s, b);
        return launched();
    }
    if (dtype == ADCT_U8) {
        switch (param) {
            case 2: launch_k<TPW, uint8_t, Mode<kInSamples, kStoreY, kMidZonal, kOutSamples, 2, true>>(grid, s, b); break;
            case 4: launch_k<TPW, uint8_t, Mode<kInSamples, kStoreY, kMidZonal, kOutSamples, 4, true>>(grid, s, b); break;
            case 8: launch_k<TPW, uint8_t, Mode<kInSamples, kStoreY, kMidZonal, kOutSamples, 8, true>>(grid, s, b); break;
            case 12: launch_k<TPW, uint8_t, Mode<kInSamples, kStoreY, kMidZonal, kOutSamples, 12, true>>(grid, s, b); break;
            case 16: launch_k<TPW, uint8_t, Mode<kInSamples, kStoreY, kMidZonal, kOutSamples, 16, true>>(grid, s, b); break;
            default: launch_k<TPW, uint8_t, Mode<kInSamples, kStoreY, kMidZonal, kOutSamples, -1, true>>(grid, s, b);
        }
    } else {
        launch_k<TPW, int16_t, Mode<kInSamples, kStoreY, kMidZonal, kOutSamples, -1, true>>(grid, s, b);
    }
    return launched();
}

int launch_batch(int tpw, int dtype, int op, int param, unsigned grid, hipStream_t s, const BatchArgs& b) {
    switch (tpw) {
        case 8: return launch_tpw<8>(dtype, op, param, grid, s, b);
        case 16: return launch_tpw<16>(dtype, op, param, grid, s, b);
        case 32: return launch_tpw<32>(dtype, op, param, grid, s, b);
        default: return ADCT_E_ARG;
    }
}

bool tune_valid(const adct_tune& t) {
    return (t.tiles_per_group == 8 || t.tiles_per_group == 16 || t.tiles_per_group == 32) &&
           t.groups_per_item >= 1 && t.groups_per_item <= 64 && t.wgs_per_cu >= 1 && t.wgs_per_cu <= 16;
}

PlaneRef plane_ref(const adct_plane* p) {
    PlaneRef r;
    r.data = static_cast<const char*>(p->data);
    r.pitch = p->pitch_bytes;
    r.bw = (uint32_t)(p->width / 16);
    return r;
}

// Validates the jobs and fills the per-image argument blocks.
int make_job_args(const adct_job* jobs, int32_t njobs, int32_t op, int32_t param, std::vector<GroupArgs>& out,
                  std::vector<int64_t>& tiles, int& dtype) {
    if (!jobs || njobs <= 0) return ADCT_E_ARG;
    Scale5Host qs{}, dqs{};
    if (op == ADCT_OP_QUANT) {
        if (!quant_scales(param, &qs, &dqs)) return ADCT_E_ARG;
    } else if (op == ADCT_OP_ZONAL) {
        if (param < 0 || param > 16) return ADCT_E_ARG;
    } else if (op == ADCT_OP_ZIGZAG) {
        if (param < 0 || param > 256) return ADCT_E_ARG;
    } else {
        return ADCT_E_ARG;
    }
    out.assign((size_t)njobs, GroupArgs{});
    tiles.assign((size_t)njobs, 0);
    dtype = jobs[0].src.dtype;
    for (int32_t j = 0; j < njobs; ++j) {
        const adct_job& jb = jobs[j];
        int rc;
        if ((rc = check_plane(&jb.src)) || (rc = check_plane(&jb.dst))) return rc;
        if (!same_shape(&jb.src, &jb.dst)) return ADCT_E_SHAPE;
        if (jb.src.dtype != dtype) return ADCT_E_DTYPE;
        if (jb.coef && !aligned16(jb.coef)) return ADCT_E_ALIGN;
        if ((uintptr_t)jb.sse & 7) return ADCT_E_ALIGN;
        GroupArgs& a = out[(size_t)j];
        a.src = plane_ref(&jb.src);
        a.dst = plane_ref(&jb.dst);
        a.cout = jb.coef;
        a.r = param;
        for (int c = 0; c < 5; ++c) {
            a.qs.f[c] = qs.f[c];
            a.dqs.f[c] = dqs.f[c];
        }
        a.bw = (uint32_t)(jb.src.width / 16);
        a.bwdiv = make_fastdiv(a.bw);
        a.ipbdiv = make_fastdiv((uint32_t)(jb.src.height / 16));  // the whole plane is one image
        a.sse = reinterpret_cast<unsigned long long*>(jb.sse);
        tiles[(size_t)j] = plane_blocks(&jb.src);
    }
    return ADCT_OK;
}

int build_items(const std::vector<int64_t>& tiles, const adct_tune& t, std::vector<uint32_t>& items,
                int64_t& n_items) {
    int rc = adct_work_queue(tiles.data(), (int32_t)tiles.size(), t.tiles_per_group, t.groups_per_item, nullptr, 0,
                             &n_items);
    if (rc) return rc;
    items.assign((size_t)(3 * n_items), 0u);
    return adct_work_queue(tiles.data(), (int32_t)tiles.size(), t.tiles_per_group, t.groups_per_item, items.data(),
                           n_items, &n_items);
}

int cu_count(int* cus, std::string* arch) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return ADCT_E_HIP;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return ADCT_E_HIP;
    *cus = prop.multiProcessorCount;
    if (arch) {
        *arch = prop.gcnArchName;
        const size_t c = arch->find(':');
        if (c != std::string::npos) arch->resize(c);
    }
    return ADCT_OK;
}

template <typename T>
int upload(const std::vector<T>& h, T** d) {
    *d = nullptr;
    if (h.empty()) return ADCT_OK;
    if (hipMalloc(reinterpret_cast<void**>(d), h.size() * sizeof(T)) != hipSuccess) return ADCT_E_NOMEM;
    if (hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) return ADCT_E_HIP;
    return ADCT_OK;
}

// Device memory of adct_batch_run_noalloc: queue heads, job table and work
// queue.  Host code never passes the array's name to a kernel or a copy: in
// host code it is a stand-in, and its device address (one per device) comes
// from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[ADCT_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
int scratch_ptr(unsigned char** out) {
    static std::mutex mu;
    static unsigned char* ptrs[kMaxDevices] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return ADCT_E_HIP;
    if (dev < 0 || dev >= kMaxDevices) return ADCT_E_HIP;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptrs[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return ADCT_E_HIP;
        ptrs[dev] = static_cast<unsigned char*>(p);
    }
    *out = ptrs[dev];
    return ADCT_OK;
}

constexpr size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

}  // namespace
}  // namespace adct

using namespace adct;

struct adct_batch {
    int op = 0, param = 0, dtype = 0;
    adct_tune tune{};
    int64_t tiles = 0, n_items = 0;
    uint32_t njobs = 0;
    unsigned grid = 0;
    GroupArgs* d_jobs = nullptr;
    ItemDev* d_items = nullptr;
    uint32_t* d_heads = nullptr;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
};

static void batch_release(adct_batch* b) {
    if (!b) return;
    // best effort: nothing useful can be done with a failure while tearing down
    if (b->done) {
        (void)hipEventSynchronize(b->done);
        (void)hipEventDestroy(b->done);
    }
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->d_heads) (void)hipFree(b->d_heads);
    if (b->d_items) (void)hipFree(b->d_items);
    if (b->d_jobs) (void)hipFree(b->d_jobs);
    delete b;
}

static int record_launch(adct_batch* b, hipStream_t s) {
    BatchArgs args{};
    args.jobs = b->d_jobs;
    args.items = b->d_items;
    for (uint32_t q = 0; q <= kQueues; ++q) args.qbeg[q] = (uint32_t)((uint64_t)b->n_items * q / kQueues);
    args.heads = b->d_heads;
    const uint32_t nreset = std::max(b->njobs, kQueues);
    hipLaunchKernelGGL(k_batch_reset, dim3((nreset + 255) / 256), dim3(256), 0, s, b->d_heads, b->d_jobs, b->njobs);
    int rc = hipGetLastError() == hipSuccess ? ADCT_OK : ADCT_E_HIP;
    if (rc) return rc;
    return launch_batch(b->tune.tiles_per_group, b->dtype, b->op, b->param, b->grid, s, args);
}

// Builds a batch; with_graph = false leaves it launchable only directly (used
// by the autotuner, which times candidates without capturing them).
static int batch_build(adct_batch** out, const std::vector<GroupArgs>& job_args, const std::vector<int64_t>& tiles,
                       int dtype, int32_t op, int32_t param, const adct_tune& t, bool with_graph) {
    *out = nullptr;
    if (!tune_valid(t)) return ADCT_E_ARG;
    int cus = 0;
    int rc = cu_count(&cus, nullptr);
    if (rc) return rc;
    adct_batch* b = new adct_batch();
    b->op = op;
    b->param = param;
    b->dtype = dtype;
    b->tune = t;
    b->njobs = (uint32_t)job_args.size();
    for (int64_t x : tiles) b->tiles += x;
    std::vector<uint32_t> items;
    if ((rc = build_items(tiles, t, items, b->n_items))) {
        batch_release(b);
        return rc;
    }
    std::vector<ItemDev> it((size_t)b->n_items);
    for (int64_t i = 0; i < b->n_items; ++i) it[(size_t)i] = ItemDev{items[3 * i], items[3 * i + 1], items[3 * i + 2]};
    b->grid = (unsigned)(cus * t.wgs_per_cu);
    if ((rc = upload(job_args, &b->d_jobs)) || (rc = upload(it, &b->d_items))) {
        batch_release(b);
        return rc;
    }
    if (hipMalloc(reinterpret_cast<void**>(&b->d_heads), kQueues * kHeadStride * sizeof(uint32_t)) != hipSuccess) {
        batch_release(b);
        return ADCT_E_NOMEM;
    }
    if (hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess) {
        batch_release(b);
        return ADCT_E_HIP;
    }
    if (with_graph) {
        if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess ||
            hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            batch_release(b);
            return ADCT_E_HIP;
        }
        rc = record_launch(b, b->cap);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(b->cap, &g);
        b->graph = g;
        if (rc || e != hipSuccess || hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) {
            batch_release(b);
            return rc ? rc : ADCT_E_HIP;
        }
    }
    *out = b;
    return ADCT_OK;
}

extern "C" {

int adct_batch_create(adct_batch** out, const adct_job* jobs, int32_t njobs, int32_t op, int32_t param,
                      const adct_tune* tune) {
    if (!out) return ADCT_E_ARG;
    *out = nullptr;
    std::vector<GroupArgs> args;
    std::vector<int64_t> tiles;
    int dtype = 0;
    int rc = make_job_args(jobs, njobs, op, param, args, tiles, dtype);
    if (rc) return rc;
    adct_tune t;
    if (tune)
        t = *tune;
    else
        adct_default_tune(&t);
    return batch_build(out, args, tiles, dtype, op, param, t, true);
}

int adct_batch_submit(adct_batch* b, void* stream) {
    if (!b || !b->exec) return ADCT_E_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hipGraphLaunch(b->exec, s) != hipSuccess) return ADCT_E_HIP;
    if (hipEventRecord(b->done, s) != hipSuccess) return ADCT_E_HIP;
    return ADCT_OK;
}

int adct_batch_run_noalloc(const adct_job* jobs, int32_t njobs, int32_t op, int32_t param, const adct_tune* tune,
                           void* stream) {
    std::vector<GroupArgs> args;
    std::vector<int64_t> tiles;
    int dtype = 0;
    int rc = make_job_args(jobs, njobs, op, param, args, tiles, dtype);
    if (rc) return rc;
    adct_tune t;
    if (tune)
        t = *tune;
    else
        adct_default_tune(&t);
    if (!tune_valid(t)) return ADCT_E_ARG;
    std::vector<uint32_t> items;
    int64_t n_items = 0;
    if ((rc = build_items(tiles, t, items, n_items))) return rc;
    // layout of the array: heads, job table, items (each 256-byte aligned)
    const size_t heads_bytes = align256(kQueues * kHeadStride * sizeof(uint32_t));
    const size_t jobs_bytes = align256(args.size() * sizeof(GroupArgs));
    const size_t items_bytes = (size_t)n_items * sizeof(ItemDev);
    if (heads_bytes + jobs_bytes + items_bytes > (size_t)ADCT_NOALLOC_SCRATCH_BYTES) return ADCT_E_TOO_LARGE;
    int cus = 0;
    if ((rc = cu_count(&cus, nullptr))) return rc;
    unsigned char* base = nullptr;
    if ((rc = scratch_ptr(&base))) return rc;
    std::vector<ItemDev> it((size_t)n_items);
    for (int64_t i = 0; i < n_items; ++i) it[(size_t)i] = ItemDev{items[3 * i], items[3 * i + 1], items[3 * i + 2]};
    hipStream_t s = static_cast<hipStream_t>(stream);
    GroupArgs* d_jobs = reinterpret_cast<GroupArgs*>(base + heads_bytes);
    ItemDev* d_items = reinterpret_cast<ItemDev*>(base + heads_bytes + jobs_bytes);
    if (hipMemcpyAsync(d_jobs, args.data(), args.size() * sizeof(GroupArgs), hipMemcpyHostToDevice, s) !=
        hipSuccess)
        return ADCT_E_HIP;
    if (items_bytes &&
        hipMemcpyAsync(d_items, it.data(), items_bytes, hipMemcpyHostToDevice, s) != hipSuccess)
        return ADCT_E_HIP;
    adct_batch b{};
    b.op = op;
    b.param = param;
    b.dtype = dtype;
    b.tune = t;
    b.n_items = n_items;
    b.njobs = (uint32_t)args.size();
    b.grid = (unsigned)(cus * t.wgs_per_cu);
    b.d_jobs = d_jobs;
    b.d_items = d_items;
    b.d_heads = reinterpret_cast<uint32_t*>(base);
    rc = record_launch(&b, s);
    // the object only carried the launch parameters: nothing of it is owned
    b.d_jobs = nullptr;
    b.d_items = nullptr;
    b.d_heads = nullptr;
    return rc;
}

int adct_batch_info(const adct_batch* b, int64_t* tiles, int64_t* items, adct_tune* tune) {
    if (!b) return ADCT_E_ARG;
    if (tiles) *tiles = b->tiles;
    if (items) *items = b->n_items;
    if (tune) *tune = b->tune;
    return ADCT_OK;
}

int adct_batch_destroy(adct_batch* b) {
    if (!b) return ADCT_E_ARG;
    batch_release(b);
    return ADCT_OK;
}

int adct_autotune(int32_t op, int32_t param, const adct_job* jobs, int32_t njobs, const char* cache_path,
                  int32_t reps, adct_tune* out, double* ms) {
    if (!out || reps < 1) return ADCT_E_ARG;
    std::vector<GroupArgs> args;
    std::vector<int64_t> tiles;
    int dtype = 0;
    int rc = make_job_args(jobs, njobs, op, param, args, tiles, dtype);
    if (rc) return rc;
    int cus = 0;
    std::string arch;
    if ((rc = cu_count(&cus, &arch))) return rc;

    if (cache_path) {
        if (FILE* f = std::fopen(cache_path, "r")) {
            char line[512];
            bool found = false;
            while (std::fgets(line, sizeof line, f)) {
                char a[64] = {0};
                int c_cus, c_op, c_param, c_dtype;
                adct_tune t{};
                double c_ms;
                const int n = std::sscanf(line,
                                          "{\"arch\": \"%63[^\"]\", \"cus\": %d, \"op\": %d, \"param\": %d, "
                                          "\"dtype\": %d, \"tiles_per_group\": %d, \"groups_per_item\": %d, "
                                          "\"wgs_per_cu\": %d, \"ms\": %lf}",
                                          a, &c_cus, &c_op, &c_param, &c_dtype, &t.tiles_per_group,
                                          &t.groups_per_item, &t.wgs_per_cu, &c_ms);
                if (n == 9 && arch == a && c_cus == cus && c_op == op && c_param == param && c_dtype == dtype &&
                    tune_valid(t)) {
                    *out = t;  // the last matching line wins
                    found = true;
                }
            }
            std::fclose(f);
            if (found) {
                if (ms) *ms = -1.0;
                return ADCT_OK;
            }
        }
    }

    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return ADCT_E_HIP;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipStreamDestroy(s);
        return ADCT_E_HIP;
    }
    adct_tune best{};
    double best_ms = 1e30;
    rc = ADCT_OK;
    for (int tpw : {8, 16, 32}) {
        for (int gpi : {1, 2, 4, 8, 16, 32, 64}) {
            for (int wpc : {2, 4, 8, 16}) {
                const adct_tune t{tpw, gpi, wpc, 0};
                adct_batch* b = nullptr;
                if ((rc = batch_build(&b, args, tiles, dtype, op, param, t, false))) break;
                std::vector<float> times;
                rc = record_launch(b, s);  // warm-up
                for (int r = 0; r < reps && !rc; ++r) {
                    if (hipEventRecord(e0, s) != hipSuccess) rc = ADCT_E_HIP;
                    if (!rc) rc = record_launch(b, s);
                    if (!rc && hipEventRecord(e1, s) != hipSuccess) rc = ADCT_E_HIP;
                    if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = ADCT_E_HIP;
                    float v = 0.f;
                    if (!rc && hipEventElapsedTime(&v, e0, e1) != hipSuccess) rc = ADCT_E_HIP;
                    times.push_back(v);
                }
                if (hipStreamSynchronize(s) != hipSuccess && !rc) rc = ADCT_E_HIP;
                batch_release(b);
                if (rc) break;
                std::sort(times.begin(), times.end());
                const double med = times[times.size() / 2];
                if (med < best_ms) {
                    best_ms = med;
                    best = t;
                }
            }
            if (rc) break;
        }
        if (rc) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(s);
    if (rc) return rc;
    *out = best;
    if (ms) *ms = best_ms;
    if (cache_path) {
        if (FILE* f = std::fopen(cache_path, "a")) {
            std::fprintf(f,
                         "{\"arch\": \"%s\", \"cus\": %d, \"op\": %d, \"param\": %d, \"dtype\": %d, "
                         "\"tiles_per_group\": %d, \"groups_per_item\": %d, \"wgs_per_cu\": %d, \"ms\": %.6f}\n",
                         arch.c_str(), cus, op, param, dtype, best.tiles_per_group, best.groups_per_item,
                         best.wgs_per_cu, best_ms);
            std::fclose(f);
        }
    }
    return ADCT_OK;
}

}  // extern "C"
