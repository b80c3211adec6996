// Serving: continuous batching of uneven requests on a device-resident loop.
//
// Requests are identified by their sequence number k (= ticket - 1) and, once
// admitted, by a publication slot j (slots are handed out in admission order;
// neither is ever reused within a server).
//
// Publication.  For each admitted request the host thread writes its
// 128-byte descriptor into slot j of a ring in host-mapped memory and then
// stores j + 1 to a host-mapped slot count (release order).  The loop takes
// the pixels straight from the caller's pinned host memory: every work item
// first copies its own sample rows over the host link into the request's
// pool block, in long contiguous runs, and is then coded from there.  Items
// are staged in slot order, at most kStagers at a time, and the coding of
// one item overlaps the transfer of others.  A request may instead be
// copied into its pool block by the DMA engine on a second stream and
// published, with no host address, once the host sees that copy's event
// (route_dma decides which, from the request's size and what is in
// flight).  Results (levels and reconstruction) go to the
// request's block of the device pool.
//
// Loop kernel (persistent).  Workgroup 0 is the dispatcher: one wave polls
// the host-mapped slot count, copies new descriptors into device memory and
// then advances the device slot count (release).  Every other workgroup is a
// worker: it scans slots from the lowest one that may still have unclaimed
// items; for slot j < count it claims item g = atomicAdd(claim[j], 1) and
// codes it when g < items(j), else marks j exhausted (atomicMax on the low
// mark) and moves on.  Over-claims are harmless since claim counters are
// never reused.  Before reading a newly met slot's descriptor a worker
// takes a system-scope acquire fence, so that no cache line left over from
// an earlier slot is read.  After coding an
// item: release fence, then done[j] += 1; the worker that completes slot j
// posts the SSE and a completion flag (system scope) to the host-mapped
// record of request k.  The dispatcher ends the loop: on the host's stop
// flag, or after `idle_polls` consecutive empty polls, it stores this
// launch's epoch to the quit word; a worker leaves once it sees that word
// and finds nothing left to claim.  The host relaunches the loop (with the
// next epoch) when published work is outstanding and the loop has exited.
#include <hip/hip_runtime.h>
#include <sys/prctl.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

#include "adct_core.hpp"
#include "adct_internal.hpp"
#include "adct_serve_logic.hpp"

namespace adct {

// One 128-byte line per publication slot; the kernel reads it as 16 words
// of 8 bytes.
struct ReqDesc {
    uint64_t src, dst, q;                     // words 0-5: device addresses in the pool
    uint32_t height, width;                   // 6, 7: samples
    uint32_t nitems, tiles_per_item;          // 8, 9
    uint32_t bw, bw_m, bw_s1, bw_s2;          // 10-13: tiles per row and its FastDiv
    uint32_t ipb_m, ipb_s1, ipb_s2, nblk;     // 14-17: FastDiv by height / 16, tiles
    uint32_t req;                             // 18: request sequence number
    uint32_t src_pitch;                       // 19: bytes between rows of src
    uint64_t hsrc;                            // 20, 21: the caller's pinned pixels (device-visible)
    uint32_t hsrc_pitch;                      // 22: bytes between their rows
    uint32_t pad[9];
};
static_assert(sizeof(ReqDesc) == 128, "one descriptor per 128-byte line");

struct Completion {
    int64_t sse;
    uint32_t flag;
    uint32_t pad;
};

struct ServeArgs {
    const ReqDesc* h_desc;       // host-mapped descriptor ring, by slot
    const uint32_t* h_count;     // host-mapped: slots written by the host
    ReqDesc* desc;               // device copy of the ring (dispatcher writes)
    uint32_t* count;             // slots copied to the device so far
    uint32_t* low;               // every slot below this is exhausted
    uint32_t* quit;              // epoch of the launch told to end
    uint32_t* claim;             // per slot: items handed out (may overshoot)
    uint32_t* done;              // per slot: items finished
    uint32_t* staged;            // per slot: items whose samples are in the pool
    uint32_t* stage_low;         // every slot below this has all its samples in the pool
    uint32_t* stage_next;        // staging tickets handed out
    uint32_t* stage_done;        // staging tickets finished
    unsigned long long* sse;     // per slot: SSE accumulator
    Completion* comp;            // per request, host-mapped
    const uint32_t* stop;        // host-mapped
    Scale5 qs, dqs;
    uint32_t idle_polls;
    uint32_t epoch;
};

template <typename T>
__device__ __forceinline__ T load_sys(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ __forceinline__ uint32_t rfl(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// A device address held as an integer, as a pointer the compiler knows to
// be in global memory (so it emits global rather than flat instructions).
__device__ __forceinline__ char* global_ptr(uint64_t v) {
    typedef __attribute__((address_space(1))) char gchar;
    return (char*)(gchar*)v;
}
__device__ __forceinline__ uint64_t rfl64(uint64_t v) {
    return ((uint64_t)rfl((uint32_t)(v >> 32)) << 32) | rfl((uint32_t)v);
}

constexpr int kServeTPW = 16;

#ifndef ADCT_SERVE_STAGERS
#define ADCT_SERVE_STAGERS 64
#endif
// Workgroups that copy samples over the host link at one time.  Enough to
// keep the link busy (each has 8 KB of reads in flight), few enough that its
// queue stays short for the loop's own polls of host memory.
constexpr uint32_t kStagers = ADCT_SERVE_STAGERS;

// Copies the samples of tiles t0 .. t1-1 (raster order over tile rows of
// width bw) of a uint8 image from the caller's pinned host memory to its
// copy in device memory, so that the item is then coded from device memory.
// Per tile row the item covers one run of tiles, so each of its 16 sample
// rows is one contiguous segment; lanes take consecutive 64-byte pieces of
// the segments.  Reads of host memory over the bus reach the link's rate
// only in long contiguous runs like these (the coding's own access, 16 bytes
// of each of 16 tiles per sample row, reaches about three quarters of it).
// The caller's barrier then makes the copy visible to the whole workgroup:
// every address the item reads afterwards is one this workgroup wrote.
__device__ __forceinline__ void stage_item(const char* __restrict__ hsrc, uint32_t hpitch, char* __restrict__ dsrc,
                                           uint32_t dpitch, uint32_t bw, const FastDiv& bwdiv, uint32_t t0,
                                           uint32_t t1) {
    for (uint32_t t = t0; t < t1;) {
        const uint32_t by = fdiv(t, bwdiv), bx0 = t - by * bw;
        const uint32_t bx1 = min(bw, bx0 + (t1 - t));
        const uint32_t len = (bx1 - bx0) * 16u;     // bytes of each sample row
        const uint32_t per_row = (len + 63u) / 64u;  // 64-byte pieces per row
        for (uint32_t c = threadIdx.x; c < 16u * per_row; c += blockDim.x) {
            const uint32_t r = c / per_row, k = c - r * per_row;
            const uint32_t off = bx0 * 16u + k * 64u;
            const uint32_t n = min(4u, (len - k * 64u) / 16u);  // 16-byte words in this piece
            const uint4* hp = reinterpret_cast<const uint4*>(hsrc + (int64_t)(by * 16u + r) * hpitch + off);
            uint4* dp = reinterpret_cast<uint4*>(dsrc + (int64_t)(by * 16u + r) * dpitch + off);
            if (n == 4) {
                const uint4 v0 = hp[0], v1 = hp[1], v2 = hp[2], v3 = hp[3];
                dp[0] = v0;
                dp[1] = v1;
                dp[2] = v2;
                dp[3] = v3;
            } else {
                for (uint32_t i = 0; i < n; ++i) dp[i] = hp[i];
            }
        }
        t += bx1 - bx0;
    }
}
using ServeMode = Mode<kInSamples, kStoreQ, kMidQuant, kOutSamples, -1, true>;

// Group arguments of slot j from its descriptor words (held in LDS).
__device__ __forceinline__ GroupArgs args_from_desc(const uint64_t* sh_desc, const ServeArgs& s, uint32_t j) {
    const uint32_t* w = reinterpret_cast<const uint32_t*>(sh_desc);
    const uint32_t width = rfl(w[7]), bw = rfl(w[10]);
    GroupArgs a{};
    a.src.data = global_ptr(rfl64(sh_desc[0]));
    a.src.pitch = rfl(w[19]);
    a.src.bw = bw;
    a.dst.data = global_ptr(rfl64(sh_desc[1]));
    a.dst.pitch = width;
    a.dst.bw = bw;
    a.cout = global_ptr(rfl64(sh_desc[2]));
    a.bw = bw;
    a.bwdiv = FastDiv{rfl(w[11]), rfl(w[12]), rfl(w[13])};
    a.ipbdiv = FastDiv{rfl(w[14]), rfl(w[15]), rfl(w[16])};
    a.sse = s.sse + j;
    return a;
}

// Workgroup 0, first wave: mirrors host-published descriptors to the device.
__device__ void serve_dispatch(const ServeArgs& s) {
    const uint32_t lane = threadIdx.x;
    uint32_t have = rfl(load_sys(s.count));
    uint32_t idle = 0;
    for (;;) {
        const uint32_t c = rfl(load_sys(s.h_count));
        if (c > have) {
            // four descriptors per pass, 16 lanes x 8 bytes each
            for (uint32_t j = have + lane / 16u; j < c; j += 4u) {
                const uint64_t v = load_sys(reinterpret_cast<const uint64_t*>(s.h_desc + j) + (lane & 15u));
                __hip_atomic_store(reinterpret_cast<uint64_t*>(s.desc + j) + (lane & 15u), v, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_SYSTEM);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");  // the wave's descriptor stores reach memory
            // the count is advanced with an atomic: it is performed where every
            // XCD's system-scope loads see it
            if (lane == 0) atomicMax(s.count, c);
            have = c;
            idle = 0;
            continue;
        }
        if ((idle & 63u) == 0u && rfl(load_sys(s.stop))) break;
        if (++idle > s.idle_polls) break;  // watchdog: the host relaunches on demand
        __builtin_amdgcn_s_sleep(16);
    }
    // after the last count update: a worker that sees the quit word also
    // sees the final count
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
    if (lane == 0) atomicMax(s.quit, s.epoch);
}

__global__ __launch_bounds__(kServeTPW * 8) void k_serve(ServeArgs s) {
    constexpr int TPW = kServeTPW;
    if (blockIdx.x == 0) {
        if (threadIdx.x < 64) serve_dispatch(s);
        return;
    }
    __shared__ uint32_t lds[lds_words(TPW)];
    __shared__ long long red[TPW * 8 / 64];
    __shared__ uint32_t sh_j, sh_g, sh_cursor, sh_quit;
    __shared__ uint64_t sh_desc[16];  // descriptor of slot `cur`
    const int tid = threadIdx.x;
    if (tid == 0) sh_cursor = 0;
    uint32_t cur = 0xffffffffu;
    bool quit_seen = false;
    for (;;) {
        __syncthreads();  // the previous item is finished with LDS and sh_*
        if (tid == 0) {
            uint32_t j = max(sh_cursor, load_sys(s.low));
            // A relaxed poll: an acquire here would invalidate this XCD's L2
            // on every poll of every idle workgroup, which costs the working
            // ones their cached staging.  The scan needs no ordering: each
            // slot's item count is written once, over the zero the ring was
            // cleared to at create (a published request has at least one
            // item), so the count read is either 0 -- not visible yet: stop
            // and poll again, claiming nothing -- or the published one.  The
            // rest of a descriptor is read after an acquire fence (below).
            const uint32_t cnt = load_sys(s.count);
            uint32_t res_j = 0xffffffffu, res_g = 0;
            while (j < cnt) {
                const uint32_t n = load_sys(&s.desc[j].nitems);
                if (n == 0u) break;
                const uint32_t g = atomicAdd(s.claim + j, 1u);
                if (g < n) {
                    res_j = j;
                    res_g = g;
                    break;
                }
                atomicMax(s.low, j + 1);
                ++j;
            }
            sh_cursor = j;
            sh_j = res_j;
            sh_g = res_g;
        }
        __syncthreads();
        const uint32_t j = rfl(sh_j);
        if (j == 0xffffffffu) {
            // nothing to claim: leave once the dispatcher has ended this
            // launch and one more scan (after seeing that) found nothing
            if (quit_seen) break;
            if (tid == 0) sh_quit = load_sys(s.quit) == s.epoch;
            __syncthreads();
            if (rfl(sh_quit)) {
                quit_seen = true;
                continue;
            }
            __builtin_amdgcn_s_sleep(64);
            continue;
        }
        const uint32_t g = rfl(sh_g);
        if (j != cur) {
            // first item of a slot met by this workgroup: acquire, then read
            // its descriptor past the caches
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
            if (tid < 16) sh_desc[tid] = load_sys(reinterpret_cast<const uint64_t*>(s.desc + j) + tid);
            __syncthreads();
            cur = j;
        }
        const uint32_t* dw = reinterpret_cast<const uint32_t*>(sh_desc);
        const uint32_t nitems = rfl(dw[8]), tpi = rfl(dw[9]), nblk = rfl(dw[17]), req = rfl(dw[18]);
        // the claim was checked against the item count read during the scan;
        // the descriptor read after the acquire is the one that counts
        if (g >= nitems) continue;
        const uint32_t t0 = g * tpi;
        const uint32_t gend = min(nblk, t0 + tpi);
        // The host link serves requests in order: an item is staged once
        // every earlier request has all its samples in the pool, so a later
        // request does not take link bandwidth from an earlier one (coding
        // still overlaps the next request's transfer).  Claims go in slot
        // order, so the items of earlier slots are all held by workers that
        // are not waiting here: the lowest such slot always progresses.
        // At most kStagers items are staged at one time (tickets in order).
        // A request whose samples the DMA engine has already copied into the
        // pool (no host address in its descriptor) only counts as staged.
        const uint64_t hsrc = rfl64(sh_desc[10]);
        if (hsrc) {
            if (tid == 0) {
                while (load_sys(s.stage_low) < j) __builtin_amdgcn_s_sleep(2);
                const uint32_t ticket = atomicAdd(s.stage_next, 1u);
                while (load_sys(s.stage_done) + kStagers <= ticket) __builtin_amdgcn_s_sleep(1);
            }
            __syncthreads();
            // the item's samples into the pool first (before the group
            // arguments are formed, which keeps fewer scalar values live
            // across the copy)
            stage_item(global_ptr(hsrc), rfl(dw[22]), global_ptr(rfl64(sh_desc[0])), rfl(dw[19]), rfl(dw[10]),
                       FastDiv{rfl(dw[11]), rfl(dw[12]), rfl(dw[13])}, t0, gend);
            __syncthreads();
        }
        if (tid == 0) {
            if (hsrc) atomicAdd(s.stage_done, 1u);
            if (atomicAdd(s.staged + j, 1u) + 1u == nitems) atomicMax(s.stage_low, j + 1u);
        }
        const GroupArgs a = args_from_desc(sh_desc, s, j);
        SseAcc acc{0, kNoImage};
        RowWords rows;
        uint32_t g0 = t0;
        load_group_rows<TPW, uint8_t>(a, g0, min((uint32_t)TPW, gend - g0), rows);
        for (uint32_t i = 0; g0 < gend; ++i, g0 += (uint32_t)TPW) {
            if (i) __syncthreads();
            const uint32_t g0n = g0 + (uint32_t)TPW;
            const uint32_t ntn = g0n < gend ? min((uint32_t)TPW, gend - g0n) : 0u;
            process_group<TPW, uint8_t, ServeMode>(a, g0, min((uint32_t)TPW, gend - g0), lds, red, acc, rows, a,
                                                  g0n, ntn, s.qs, s.dqs);
        }
        sse_flush<TPW * 8>(acc, a.sse, red);
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // this item's outputs and SSE
        if (tid == 0) {
            const uint32_t old = atomicAdd(s.done + j, 1u);
            if (old + 1u == nitems) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // every other item of j
                const long long v = (long long)load_sys(s.sse + j);
                __hip_atomic_store(&s.comp[req].sse, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                __hip_atomic_store(&s.comp[req].flag, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
    }
}

namespace {

int64_t clock_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

enum ReqState { kWaiting = 0, kRunning = 1, kDone = 2, kReleased = 3, kCancelled = 4 };

struct Req {
    const void* host = nullptr;
    uint64_t dev_src = 0;  // persistent: the host pixels' device-visible address
    int32_t h = 0, w = 0;
    int64_t pitch = 0;
    int64_t bytes = 0, tiles = 0;
    int64_t t_arrival = 0, t_admit = -1, t_done = -1;
    int64_t off = -1;
    int64_t sse = -1;
    int state = kWaiting;
    int ev = -1;  // plain: event slot marking the end of the request;
                  // persistent: event slot marking the end of its DMA copy
    bool big_staged = false;  // persistent: a large request staged by the loop
};

// Pool block of a request: the copied source, the reconstruction and the
// levels (4 bytes per pixel).
struct Block {
    char *src, *dst, *q;
};

// While requests are outstanding, or the next one arrives within this
// window, the host thread polls instead of sleeping.
constexpr int64_t kSpinWindowNs = 200000;

}  // namespace
}  // namespace adct

using namespace adct;

struct adct_server {
    adct_server_cfg cfg{};
    int device = 0, cus = 0;
    Scale5Host qs{}, dqs{};
    char* pool_mem = nullptr;
    Pool* pool = nullptr;

    std::mutex mu;
    std::condition_variable cv;       // wakes the server thread
    std::condition_variable done_cv;  // wakes waiters on completions
    std::thread worker;
    bool quit = false, stopping = false, loop_running = false;

    std::vector<Req> reqs;
    int64_t head = 0, inflight = 0;
    std::vector<int64_t> running;     // admitted, not yet done (plain: in stream order)
    int64_t n_done = 0, n_cancelled = 0, loop_launches = 0, n_published = 0;
    int hip_error = 0;
    uint32_t epoch = 0;

    hipStream_t stream = nullptr;     // the loop's stream, or the plain path's one stream
    // plain mode
    std::vector<hipEvent_t> events;
    std::vector<int> free_events;
    // persistent mode
    hipStream_t copy_stream = nullptr; // DMA copies of large requests
    std::vector<int64_t> dma_pending; // copies issued, not yet published (issue order)
    int64_t big_staging = 0;          // large requests in flight that the loop stages
    int64_t dma_copies = 0;           // requests copied by the DMA engine
    ReqDesc* h_desc = nullptr;        // host-mapped descriptor ring, by slot
    ReqDesc* d_hdesc = nullptr;       // its device address
    uint32_t* h_count = nullptr;      // host-mapped slot count
    uint32_t* d_hcount = nullptr;
    ReqDesc* d_desc = nullptr;        // device copy of the ring
    uint32_t* d_state = nullptr;      // count, low, quit, stage_low, stage_next, stage_done, then claim[n], done[n], staged[n]
    unsigned long long* d_sse = nullptr;
    Completion* h_comp = nullptr;     // host-mapped, by request
    Completion* d_comp = nullptr;     // its device address
    uint32_t* h_stop = nullptr;       // host-mapped
    uint32_t* d_stop = nullptr;
    hipEvent_t loop_done = nullptr;
};

namespace {

uint32_t* st_count(adct_server* S) { return S->d_state; }
uint32_t* st_low(adct_server* S) { return S->d_state + 32; }
uint32_t* st_quit(adct_server* S) { return S->d_state + 64; }
uint32_t* st_stage_low(adct_server* S) { return S->d_state + 96; }
uint32_t* st_stage_next(adct_server* S) { return S->d_state + 128; }
uint32_t* st_stage_done(adct_server* S) { return S->d_state + 160; }
uint32_t* st_claim(adct_server* S) { return S->d_state + 192; }
uint32_t* st_done(adct_server* S) { return S->d_state + 192 + S->cfg.max_requests; }
uint32_t* st_staged(adct_server* S) { return S->d_state + 192 + 2 * S->cfg.max_requests; }

bool hip_ok(adct_server* S, hipError_t e) {
    if (e != hipSuccess && !S->hip_error) S->hip_error = (int)e;
    return e == hipSuccess;
}

void launch_loop(adct_server* S) {
    ServeArgs a{};
    a.h_desc = S->d_hdesc;
    a.h_count = S->d_hcount;
    a.desc = S->d_desc;
    a.count = st_count(S);
    a.low = st_low(S);
    a.quit = st_quit(S);
    a.claim = st_claim(S);
    a.done = st_done(S);
    a.staged = st_staged(S);
    a.stage_low = st_stage_low(S);
    a.stage_next = st_stage_next(S);
    a.stage_done = st_stage_done(S);
    a.sse = S->d_sse;
    a.comp = S->d_comp;
    a.stop = S->d_stop;
    for (int c = 0; c < 5; ++c) {
        a.qs.f[c] = S->qs.f[c];
        a.dqs.f[c] = S->dqs.f[c];
    }
    a.idle_polls = (uint32_t)S->cfg.idle_polls;
    a.epoch = ++S->epoch;  // the quit word holds an older epoch, so this launch runs
    // workgroup 0 dispatches, the rest code
    hipLaunchKernelGGL(k_serve, dim3((unsigned)(S->cus * S->cfg.wgs_per_cu + 1)), dim3(kServeTPW * 8), 0,
                       S->stream, a);
    hip_ok(S, hipGetLastError());
    hip_ok(S, hipEventRecord(S->loop_done, S->stream));
    S->loop_running = true;
    ++S->loop_launches;
}

bool loop_exited(adct_server* S) {
    if (!S->loop_running) return true;
    const hipError_t e = hipEventQuery(S->loop_done);
    if (e == hipSuccess) {
        S->loop_running = false;
        return true;
    }
    if (e != hipErrorNotReady) hip_ok(S, e);
    return false;
}

Block block_of(const adct_server* S, const Req& r) {
    const int64_t plane = Pool::round_up((int64_t)r.h * r.w);
    char* base = S->pool_mem + r.off;
    Block b;
    b.src = base;
    b.dst = base + plane;
    b.q = b.dst + plane;
    return b;
}

// Tiles per work item of a request.  Adaptive (cfg value 0): small requests
// are cut into 16-tile items so that many workgroups share them; larger ones
// into items of up to 128 tiles (at most about 128 items for requests up to
// 16384 tiles), which amortises the per-item claim, fence and counter work.
int64_t item_tiles(int32_t cfg_tiles_per_item, int64_t tiles) {
    if (cfg_tiles_per_item > 0) return cfg_tiles_per_item;
    int64_t t = 16;
    while (t < 128 && t * 128 < tiles) t *= 2;
    return t;
}

int64_t block_bytes(int32_t h, int32_t w) {
    const int64_t plane = (int64_t)h * w;
    return 2 * Pool::round_up(plane) + 2 * plane;
}

// Copies a request's pixels into its pool block on `stream` (rows packed).
void copy_in(adct_server* S, const Req& r, const Block& b, hipStream_t stream) {
    if (r.pitch == r.w)
        hip_ok(S, hipMemcpyAsync(b.src, r.host, (size_t)((int64_t)r.h * r.w), hipMemcpyHostToDevice, stream));
    else
        hip_ok(S, hipMemcpy2DAsync(b.src, (size_t)r.w, r.host, (size_t)r.pitch, (size_t)r.w, (size_t)r.h,
                                   hipMemcpyHostToDevice, stream));
}

bool event_done(adct_server* S, int ev);
void publish(adct_server* S, int64_t k, uint64_t hsrc);

// Persistent mode: whether request r goes to the pool by a DMA copy rather
// than through the loop's own staging (called with mu held).
//   ADCT_SERVE_DMA_BY_SIZE: exactly the requests of at least dma_min_pixels.
//   ADCT_SERVE_DMA_ADAPTIVE: a large request (at least dma_min_pixels) is
//   staged by the loop when nothing else is in flight -- the loop's reads
//   reach the link's rate on one long request and its coding overlaps them,
//   where a DMA copy must end before any coding starts -- and copied by DMA
//   when other requests are in flight, so that it neither waits for their
//   staging nor holds theirs up.  A smaller request is staged by the loop,
//   unless the loop is staging a large one: staging goes in order, and
//   behind that one it would wait for the whole transfer, so it is copied
//   by DMA alongside it instead.
bool route_dma(const adct_server* S, const Req& r) {
    if (S->cfg.dma_min_pixels <= 0) return false;
    const bool big = (int64_t)r.h * r.w >= S->cfg.dma_min_pixels;
    if (S->cfg.dma_policy == ADCT_SERVE_DMA_BY_SIZE) return big;
    return big ? !S->running.empty() : S->big_staging > 0;
}

// Hands an admitted request to the device (called with mu held).  Persistent
// mode: publish its descriptor, or start its DMA copy into the pool
// (published when done); plain mode: copy in, code, copy the SSE back and
// record an event, all on the one stream.
void issue(adct_server* S, int64_t k) {
    Req& r = S->reqs[(size_t)k];
    const Block b = block_of(S, r);
    if (S->cfg.mode == ADCT_SERVE_PLAIN) {
        copy_in(S, r, b, S->stream);
        adct_plane ps{b.src, ADCT_U8, r.h, r.w, 0, r.w};
        adct_plane pd{b.dst, ADCT_U8, r.h, r.w, 0, r.w};
        int rc = adct_fwd2d_quant(&ps, S->cfg.qp, reinterpret_cast<int16_t*>(b.q), S->stream);
        if (!rc)
            rc = adct_dequant_recon(reinterpret_cast<int16_t*>(b.q), S->cfg.qp, &pd, &ps, r.h,
                                    reinterpret_cast<int64_t*>(S->d_sse + k), S->stream);
        if (rc && !S->hip_error) S->hip_error = rc;
        hip_ok(S, hipMemcpyAsync(&S->h_comp[k].sse, S->d_sse + k, sizeof(int64_t), hipMemcpyDeviceToHost,
                                 S->stream));
        r.ev = S->free_events.back();
        S->free_events.pop_back();
        hip_ok(S, hipEventRecord(S->events[(size_t)r.ev], S->stream));
    } else if (route_dma(S, r)) {
        // the DMA engine copies it into the pool; published when done
        copy_in(S, r, b, S->copy_stream);
        ++S->dma_copies;
        r.ev = S->free_events.back();
        S->free_events.pop_back();
        hip_ok(S, hipEventRecord(S->events[(size_t)r.ev], S->copy_stream));
        S->dma_pending.push_back(k);
    } else {
        r.big_staged = S->cfg.dma_min_pixels > 0 && (int64_t)r.h * r.w >= S->cfg.dma_min_pixels;
        if (r.big_staged) ++S->big_staging;
        publish(S, k, r.dev_src);
    }
    r.state = kRunning;
    S->running.push_back(k);
}

// Writes request k's descriptor to the next slot and announces it (called
// with mu held).  hsrc: the caller's pixels for the loop to stage, or 0 when
// they are already in the pool.
void publish(adct_server* S, int64_t k, uint64_t hsrc) {
    Req& r = S->reqs[(size_t)k];
    const Block b = block_of(S, r);
    {
        ReqDesc d;
        memset(&d, 0, sizeof d);
        d.src = (uint64_t)(uintptr_t)b.src;
        d.hsrc = hsrc;
        d.hsrc_pitch = (uint32_t)r.pitch;
        d.dst = (uint64_t)(uintptr_t)b.dst;
        d.q = (uint64_t)(uintptr_t)b.q;
        d.height = (uint32_t)r.h;
        d.width = (uint32_t)r.w;
        d.src_pitch = (uint32_t)r.w;
        d.nblk = (uint32_t)r.tiles;
        const int64_t tpi = item_tiles(S->cfg.tiles_per_item, r.tiles);
        d.tiles_per_item = (uint32_t)tpi;
        d.nitems = (uint32_t)((r.tiles + tpi - 1) / tpi);
        d.bw = (uint32_t)(r.w / 16);
        const FastDiv fb = make_fastdiv(d.bw), fi = make_fastdiv((uint32_t)(r.h / 16));
        d.bw_m = fb.m;
        d.bw_s1 = fb.s1;
        d.bw_s2 = fb.s2;
        d.ipb_m = fi.m;
        d.ipb_s1 = fi.s1;
        d.ipb_s2 = fi.s2;
        d.req = (uint32_t)k;
        const int64_t slot = S->n_published++;
        memcpy(&S->h_desc[slot], &d, sizeof d);
        // the descriptor is written before the count that announces it
        __atomic_store_n(S->h_count, (uint32_t)(slot + 1), __ATOMIC_RELEASE);
        if (!S->stopping && loop_exited(S)) launch_loop(S);
    }
}

// Publishes the requests whose DMA copies are done (called with mu held);
// the copies run on one stream and finish in issue order.  Returns whether
// any was published.
bool publish_copied(adct_server* S) {
    size_t i = 0;
    while (i < S->dma_pending.size() && event_done(S, S->reqs[(size_t)S->dma_pending[i]].ev)) {
        const int64_t k = S->dma_pending[i];
        Req& r = S->reqs[(size_t)k];
        S->free_events.push_back(r.ev);
        r.ev = -1;
        publish(S, k, 0);
        ++i;
    }
    S->dma_pending.erase(S->dma_pending.begin(), S->dma_pending.begin() + (ptrdiff_t)i);
    return i > 0;
}

bool event_done(adct_server* S, int ev) {
    const hipError_t e = hipEventQuery(S->events[(size_t)ev]);
    if (e != hipSuccess && e != hipErrorNotReady) hip_ok(S, e);
    return e == hipSuccess;
}

void release_mem(adct_server* S, Req& r) {
    if (r.off >= 0) {
        S->pool->release(r.off, r.bytes);
        r.off = -1;
        --S->inflight;
    }
}

void finish(adct_server* S, int64_t k, int64_t now) {
    Req& r = S->reqs[(size_t)k];
    r.sse = __atomic_load_n(&S->h_comp[k].sse, __ATOMIC_ACQUIRE);
    r.t_done = now;
    r.state = kDone;
    if (r.big_staged) {
        r.big_staged = false;
        --S->big_staging;
    }
    if (r.ev >= 0) {
        S->free_events.push_back(r.ev);
        r.ev = -1;
    }
    if (S->cfg.auto_release) {
        release_mem(S, r);
        r.state = kReleased;
    }
    ++S->n_done;
}

// Completions (called with mu held); returns whether any request finished.
bool poll_done(adct_server* S) {
    bool any = false;
    if (S->cfg.mode == ADCT_SERVE_PLAIN) {
        // one stream: requests complete in issue order
        size_t i = 0;
        while (i < S->running.size() && event_done(S, S->reqs[(size_t)S->running[i]].ev)) ++i;
        if (i) {
            const int64_t now = clock_ns();
            for (size_t t = 0; t < i; ++t) finish(S, S->running[t], now);
            S->running.erase(S->running.begin(), S->running.begin() + (ptrdiff_t)i);
            any = true;
        }
        return any;
    }
    for (size_t i = 0; i < S->running.size();) {
        const int64_t k = S->running[i];
        if (__atomic_load_n(&S->h_comp[k].flag, __ATOMIC_ACQUIRE) != 0) {
            finish(S, k, clock_ns());
            S->running[i] = S->running.back();
            S->running.pop_back();
            any = true;
        } else {
            ++i;
        }
    }
    return any;
}

void serve_thread(adct_server* S) {
    // precise sleeps: the default timer slack would add tens of microseconds
    (void)prctl(PR_SET_TIMERSLACK, 1UL, 0UL, 0UL, 0UL);
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    while (!S->quit) {
        const int64_t now = clock_ns();
        const int64_t n = (int64_t)S->reqs.size();
        int64_t admitted = 0;
        S->head = admit_in_order(
            S->head, n, now, S->inflight, S->cfg.max_inflight, *S->pool,
            [&](int64_t i) { return S->reqs[(size_t)i].t_arrival; },
            [&](int64_t i) { return S->reqs[(size_t)i].bytes; },
            [&](int64_t i) { return S->reqs[(size_t)i].state == kCancelled; },
            [&](int64_t i, int64_t off) {
                Req& r = S->reqs[(size_t)i];
                r.off = off;
                r.t_admit = now;
                issue(S, i);
                ++admitted;
            });
        const bool copied = S->cfg.mode == ADCT_SERVE_PERSISTENT && publish_copied(S);
        if (S->cfg.mode == ADCT_SERVE_PERSISTENT && !S->running.empty() && !S->stopping && loop_exited(S))
            launch_loop(S);  // the loop went idle and exited before this work was published
        const bool fin = poll_done(S);
        if (fin) S->done_cv.notify_all();
        if (admitted || copied || fin) continue;
        // nothing happened: poll again soon while work is outstanding or about
        // to arrive, otherwise sleep until a submission, a release or the
        // next arrival
        int64_t wait_ns = S->running.empty() ? 50000000 : 0;
        if (S->head < n && S->reqs[(size_t)S->head].state == kWaiting && S->inflight < S->cfg.max_inflight) {
            const int64_t until = S->reqs[(size_t)S->head].t_arrival - now;
            if (until < wait_ns) wait_ns = until > 0 ? until : 0;
        }
        if (wait_ns <= kSpinWindowNs) {
            lk.unlock();
            for (int i = 0; i < 32; ++i) __builtin_ia32_pause();
            lk.lock();
        } else {
            S->cv.wait_for(lk, std::chrono::nanoseconds(wait_ns - kSpinWindowNs / 2));
        }
    }
}

void free_server(adct_server* S) {
    if (S->loop_done) (void)hipEventDestroy(S->loop_done);
    for (hipEvent_t e : S->events)
        if (e) (void)hipEventDestroy(e);
    if (S->stream) (void)hipStreamDestroy(S->stream);
    if (S->copy_stream) (void)hipStreamDestroy(S->copy_stream);
    if (S->pool_mem) (void)hipFree(S->pool_mem);
    if (S->d_desc) (void)hipFree(S->d_desc);
    if (S->d_state) (void)hipFree(S->d_state);
    if (S->d_sse) (void)hipFree(S->d_sse);
    if (S->h_desc) (void)hipHostFree(S->h_desc);
    if (S->h_count) (void)hipHostFree(S->h_count);
    if (S->h_comp) (void)hipHostFree(S->h_comp);
    if (S->h_stop) (void)hipHostFree(S->h_stop);
    delete S->pool;
    delete S;
}

}  // namespace

extern "C" {

int64_t adct_now_ns(void) { return clock_ns(); }

int adct_server_create(adct_server** out, const adct_server_cfg* cfg_in) {
    if (!out || !cfg_in) return ADCT_E_ARG;
    *out = nullptr;
    adct_server_cfg cfg = *cfg_in;
    if (cfg.wgs_per_cu == 0) cfg.wgs_per_cu = 2;
    if (cfg.idle_polls == 0) cfg.idle_polls = 100000;
    if (cfg.dma_min_pixels == 0) cfg.dma_min_pixels = ADCT_SERVE_DMA_MIN_DEFAULT;
    if (cfg.dma_policy != ADCT_SERVE_DMA_ADAPTIVE && cfg.dma_policy != ADCT_SERVE_DMA_BY_SIZE) return ADCT_E_ARG;
    if (cfg.pool_bytes < 1024 || cfg.max_inflight < 1 || cfg.max_requests < 1 || cfg.tiles_per_item < 0 ||
        cfg.tiles_per_item % 16 || cfg.wgs_per_cu < 1 || cfg.wgs_per_cu > 8 || cfg.idle_polls < 1 ||
        cfg.dma_min_pixels < -1 ||
        (cfg.mode != ADCT_SERVE_PERSISTENT && cfg.mode != ADCT_SERVE_PLAIN))
        return ADCT_E_ARG;
    adct_server* S = new adct_server();
    S->cfg = cfg;
    if (!quant_scales(cfg.qp, &S->qs, &S->dqs)) {
        delete S;
        return ADCT_E_ARG;
    }
    hipDeviceProp_t prop;
    if (hipGetDevice(&S->device) != hipSuccess || hipGetDeviceProperties(&prop, S->device) != hipSuccess) {
        delete S;
        return ADCT_E_HIP;
    }
    S->cus = prop.multiProcessorCount;
    S->pool = new Pool(cfg.pool_bytes);
    const size_t n = (size_t)cfg.max_requests;
    const unsigned mapped = hipHostMallocMapped | hipHostMallocCoherent;
    bool ok = hipMalloc(reinterpret_cast<void**>(&S->pool_mem), (size_t)S->pool->capacity()) == hipSuccess &&
              hipMalloc(reinterpret_cast<void**>(&S->d_sse), n * sizeof(unsigned long long)) == hipSuccess &&
              hipMemset(S->d_sse, 0, n * sizeof(unsigned long long)) == hipSuccess &&
              hipHostMalloc(reinterpret_cast<void**>(&S->h_comp), n * sizeof(Completion), mapped) == hipSuccess &&
              hipHostMalloc(reinterpret_cast<void**>(&S->h_stop), 128, mapped) == hipSuccess &&
              hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) == hipSuccess;
    const bool use_dma = cfg.mode == ADCT_SERVE_PERSISTENT && cfg.dma_min_pixels > 0;
    if (ok && use_dma) ok = hipStreamCreateWithFlags(&S->copy_stream, hipStreamNonBlocking) == hipSuccess;
    if (cfg.mode == ADCT_SERVE_PLAIN || use_dma) {
        S->events.resize((size_t)cfg.max_inflight, nullptr);
        for (int i = 0; ok && i < cfg.max_inflight; ++i) {
            ok = hipEventCreateWithFlags(&S->events[(size_t)i], hipEventDisableTiming) == hipSuccess;
            S->free_events.push_back(i);
        }
    }
    if (ok) {
        memset(S->h_comp, 0, n * sizeof(Completion));
        *S->h_stop = 0;
        ok = hipHostGetDevicePointer(reinterpret_cast<void**>(&S->d_comp), S->h_comp, 0) == hipSuccess &&
             hipHostGetDevicePointer(reinterpret_cast<void**>(&S->d_stop), S->h_stop, 0) == hipSuccess;
    }
    if (ok && cfg.mode == ADCT_SERVE_PERSISTENT) {
        const size_t state_words = 192 + 3 * n;
        ok = hipMalloc(reinterpret_cast<void**>(&S->d_desc), n * sizeof(ReqDesc)) == hipSuccess &&
             hipMemset(S->d_desc, 0, n * sizeof(ReqDesc)) == hipSuccess &&
             hipMalloc(reinterpret_cast<void**>(&S->d_state), state_words * sizeof(uint32_t)) == hipSuccess &&
             hipMemset(S->d_state, 0, state_words * sizeof(uint32_t)) == hipSuccess &&
             hipHostMalloc(reinterpret_cast<void**>(&S->h_desc), n * sizeof(ReqDesc), mapped) == hipSuccess &&
             hipHostMalloc(reinterpret_cast<void**>(&S->h_count), 128, mapped) == hipSuccess &&
             hipEventCreateWithFlags(&S->loop_done, hipEventDisableTiming) == hipSuccess;
        if (ok) {
            memset(S->h_desc, 0, n * sizeof(ReqDesc));
            *S->h_count = 0;
            ok = hipHostGetDevicePointer(reinterpret_cast<void**>(&S->d_hdesc), S->h_desc, 0) == hipSuccess &&
                 hipHostGetDevicePointer(reinterpret_cast<void**>(&S->d_hcount), S->h_count, 0) == hipSuccess &&
                 hipDeviceSynchronize() == hipSuccess;
        }
    }
    if (!ok) {
        free_server(S);
        return ADCT_E_NOMEM;
    }
    S->reqs.reserve(n);
    if (cfg.mode == ADCT_SERVE_PERSISTENT) launch_loop(S);
    S->worker = std::thread(serve_thread, S);
    *out = S;
    return ADCT_OK;
}

int adct_server_submit(adct_server* S, const void* host_pixels, int32_t height, int32_t width, int64_t pitch_bytes,
                       int64_t arrival_ns, uint64_t* ticket) {
    if (!S || !host_pixels || !ticket) return ADCT_E_ARG;
    if (height <= 0 || width <= 0 || (height & 15) || (width & 15) || pitch_bytes < width) return ADCT_E_SHAPE;
    Req r;
    r.host = host_pixels;
    r.h = height;
    r.w = width;
    r.pitch = pitch_bytes;
    if (S->cfg.mode == ADCT_SERVE_PERSISTENT) {
        // the loop reads the pixels from the caller's memory: it must be
        // pinned host memory that the device can address, 16-byte aligned rows
        if (((uintptr_t)host_pixels & 15) || (pitch_bytes & 15) || pitch_bytes > 0xffffffffll) return ADCT_E_ALIGN;
        hipPointerAttribute_t attr;
        memset(&attr, 0, sizeof attr);
        const hipError_t e = hipPointerGetAttributes(&attr, host_pixels);
        if (e != hipSuccess) (void)hipGetLastError();  // clear this thread's error state
        if (e != hipSuccess || attr.type != hipMemoryTypeHost || !attr.devicePointer) return ADCT_E_ARG;
        r.dev_src = (uint64_t)(uintptr_t)attr.devicePointer;
    }
    r.bytes = block_bytes(height, width);
    r.tiles = (int64_t)height * width / 256;
    r.t_arrival = arrival_ns < 0 ? clock_ns() : arrival_ns;
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stopping) return ADCT_E_STOPPED;
    if (!S->pool->fits_ever(r.bytes) || (int64_t)S->reqs.size() >= S->cfg.max_requests) return ADCT_E_TOO_LARGE;
    S->reqs.push_back(r);
    *ticket = (uint64_t)S->reqs.size();
    S->cv.notify_one();
    return ADCT_OK;
}

int adct_server_poll(adct_server* S, uint64_t ticket, adct_result* out) {
    if (!S || !out) return ADCT_E_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    if (ticket == 0 || ticket > S->reqs.size()) return ADCT_E_NOTFOUND;
    if (S->hip_error) return ADCT_E_HIP;
    const Req& r = S->reqs[(size_t)(ticket - 1)];
    memset(out, 0, sizeof *out);
    out->height = r.h;
    out->width = r.w;
    out->t_arrival_ns = r.t_arrival;
    out->t_admit_ns = r.t_admit;
    if (r.state == kCancelled) {
        out->status = ADCT_E_STOPPED;
        return ADCT_E_STOPPED;
    }
    if (r.state == kWaiting || r.state == kRunning) {
        out->status = ADCT_PENDING;
        return ADCT_PENDING;
    }
    out->status = ADCT_OK;
    out->sse = r.sse;
    out->t_done_ns = r.t_done;
    if (r.off >= 0) {
        const Block b = block_of(S, r);
        out->dst = b.dst;
        out->q = b.q;
    }
    return ADCT_OK;
}

int adct_server_wait_all(adct_server* S, int64_t timeout_ns) {
    if (!S) return ADCT_E_ARG;
    std::unique_lock<std::mutex> lk(S->mu);
    const auto until = std::chrono::steady_clock::now() + std::chrono::nanoseconds(timeout_ns < 0 ? 0 : timeout_ns);
    while (S->n_done + S->n_cancelled < (int64_t)S->reqs.size()) {
        if (S->hip_error) return ADCT_E_HIP;
        if (S->done_cv.wait_until(lk, until) == std::cv_status::timeout &&
            S->n_done + S->n_cancelled < (int64_t)S->reqs.size())
            return ADCT_E_TIMEOUT;
    }
    return S->hip_error ? ADCT_E_HIP : ADCT_OK;
}

int adct_server_release(adct_server* S, uint64_t ticket) {
    if (!S) return ADCT_E_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    if (ticket == 0 || ticket > S->reqs.size()) return ADCT_E_NOTFOUND;
    Req& r = S->reqs[(size_t)(ticket - 1)];
    if (r.state == kWaiting || r.state == kRunning) return ADCT_PENDING;
    if (r.state == kDone) {
        release_mem(S, r);
        r.state = kReleased;
        S->cv.notify_one();
    }
    return ADCT_OK;
}

int adct_server_stats(adct_server* S, adct_stats* out) {
    if (!S || !out) return ADCT_E_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    memset(out, 0, sizeof *out);
    std::vector<double> lat, queue;
    int64_t t_first = INT64_MAX, t_last = INT64_MIN;
    for (const Req& r : S->reqs) {
        if (r.t_admit >= 0) ++out->admitted;
        if (r.state == kDone || r.state == kReleased) {
            ++out->completed;
            out->tiles_completed += r.tiles;
            lat.push_back((double)(r.t_done - r.t_arrival) * 1e-6);
            queue.push_back((double)(r.t_admit - r.t_arrival) * 1e-6);
            t_first = std::min(t_first, r.t_arrival);
            t_last = std::max(t_last, r.t_done);
        }
    }
    out->submitted = (int64_t)S->reqs.size();
    out->cancelled = S->n_cancelled;
    out->in_flight = (int64_t)S->running.size();
    out->pool_bytes = S->pool->capacity();
    out->pool_high_water = S->pool->high_water();
    out->loop_launches = S->loop_launches;
    out->dma_copies = S->dma_copies;
    if (!lat.empty()) {
        out->wall_s = (double)(t_last - t_first) * 1e-9;
        out->tiles_per_s = out->wall_s > 0 ? (double)out->tiles_completed / out->wall_s : 0.0;
        out->latency_p50_ms = percentile(lat, 50);
        out->latency_p99_ms = percentile(lat, 99);
        out->latency_max_ms = percentile(lat, 100);
        double sum = 0;
        for (double v : lat) sum += v;
        out->latency_mean_ms = sum / (double)lat.size();
        out->queue_p50_ms = percentile(queue, 50);
        out->queue_p99_ms = percentile(queue, 99);
    }
    return S->hip_error ? ADCT_E_HIP : ADCT_OK;
}

int adct_server_stop(adct_server* S, int32_t drain) {
    if (!S) return ADCT_E_ARG;
    std::unique_lock<std::mutex> lk(S->mu);
    if (drain) {
        const int64_t t0 = clock_ns();
        while (S->n_done + S->n_cancelled < (int64_t)S->reqs.size() && !S->hip_error) {
            if (clock_ns() - t0 > 60000000000ll) return ADCT_E_TIMEOUT;
            S->done_cv.wait_for(lk, std::chrono::milliseconds(10));
        }
    } else {
        for (int64_t i = S->head; i < (int64_t)S->reqs.size(); ++i) {
            if (S->reqs[(size_t)i].state == kWaiting) {
                S->reqs[(size_t)i].state = kCancelled;
                ++S->n_cancelled;
            }
        }
        // admitted requests finish on the device (bounded wait)
        const int64_t t0 = clock_ns();
        while (!S->running.empty() && !S->hip_error && clock_ns() - t0 < 20000000000ll)
            S->done_cv.wait_for(lk, std::chrono::milliseconds(10));
    }
    S->stopping = true;
    __atomic_store_n(S->h_stop, 1u, __ATOMIC_RELEASE);
    S->done_cv.notify_all();
    if (S->cfg.mode == ADCT_SERVE_PERSISTENT) {
        // the dispatcher sees the flag within a few polls and ends the launch
        const int64_t t0 = clock_ns();
        while (!loop_exited(S)) {
            if (clock_ns() - t0 > 20000000000ll) return ADCT_E_TIMEOUT;
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(200));
            lk.lock();
        }
    }
    return S->hip_error ? ADCT_E_HIP : ADCT_OK;
}

int adct_server_destroy(adct_server* S) {
    if (!S) return ADCT_E_ARG;
    int rc = adct_server_stop(S, 0);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->quit = true;
        S->cv.notify_all();
    }
    if (S->worker.joinable()) S->worker.join();
    if (rc == ADCT_E_TIMEOUT) return rc;  // the loop did not exit: keep its memory alive
    (void)hipStreamSynchronize(S->stream);
    free_server(S);
    return rc;
}

}  // extern "C"
