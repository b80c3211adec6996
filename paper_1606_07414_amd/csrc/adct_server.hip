// Serving: continuous batching of uneven requests on a device-resident loop.
//
// Device state, all indexed by the request's sequence number k (= ticket - 1,
// never reused within a server): a 128-byte descriptor, a claim counter, a
// done counter and an SSE accumulator in device memory, and a completion
// record in host-mapped memory.
//
// Publication: for each admitted request the host thread enqueues on one
// copy stream (i) the pixels into the request's pool block, (ii) its
// descriptor, (iii) the new count of published requests.  Stream order makes
// the count visible only after the data it announces.
//
// Loop kernel (persistent, a few workgroups per CU): a workgroup scans
// requests from the lowest one that may still have unclaimed items; for
// request k < published it claims item g = atomicAdd(claim[k], 1) and codes
// it when g < items(k), else marks k exhausted (atomicMax on the low mark)
// and moves on.  Only published requests are touched and claim counters are
// never reused, so an over-claim is harmless and no claim is ever left
// pending.  Before reading a newly met request's descriptor and pixels the
// workgroup takes a system-scope acquire fence, so that no cache line left
// over from an earlier user of the same pool memory is read.  After coding
// an item: release fence, then done[k] += 1; the workgroup that completes
// request k posts its SSE and a completion flag (system scope) to host
// memory.  An idle workgroup sleeps between polls and exits on the stop flag
// or after `idle_polls` empty polls; the host relaunches the loop when
// published work is outstanding and the loop has exited.
#include <hip/hip_runtime.h>

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

// One 128-byte line per request; the kernel reads it as 32 words.
struct ReqDesc {
    uint64_t src, dst, q;                     // words 0-5: device addresses in the pool
    uint32_t height, width;                   // 6, 7: samples
    uint32_t nitems, tiles_per_item;          // 8, 9
    uint32_t bw, bw_m, bw_s1, bw_s2;          // 10-13: tiles per row and its FastDiv
    uint32_t ipb_m, ipb_s1, ipb_s2, nblk;     // 14-17: FastDiv by height / 16, tiles
    uint32_t pad[14];
};
static_assert(sizeof(ReqDesc) == 128, "one descriptor per 128-byte line");

struct Completion {
    int64_t sse;
    uint32_t flag;
    uint32_t pad;
};

struct ServeArgs {
    const ReqDesc* desc;
    const uint32_t* published;   // requests published so far (written by DMA)
    uint32_t* low;               // every request below this is exhausted
    uint32_t* claim;             // per request: items handed out (may overshoot)
    uint32_t* done;              // per request: items finished
    unsigned long long* sse;     // per request: SSE accumulator
    Completion* comp;            // per request, host-mapped
    const uint32_t* stop;        // host-mapped
    Scale5 qs, dqs;
    uint32_t idle_polls;
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
using ServeMode = Mode<kInSamples, kStoreQ, kMidQuant, kOutSamples, -1, true>;

// Group arguments of request k from its descriptor words (held in LDS).
__device__ __forceinline__ GroupArgs args_from_desc(const uint64_t* sh_desc, const ServeArgs& s, uint32_t k) {
    const uint32_t* w = reinterpret_cast<const uint32_t*>(sh_desc);
    const uint32_t width = rfl(w[7]), bw = rfl(w[10]);
    GroupArgs a{};
    a.src.data = global_ptr(rfl64(sh_desc[0]));
    a.src.pitch = width;
    a.src.bw = bw;
    a.dst.data = global_ptr(rfl64(sh_desc[1]));
    a.dst.pitch = width;
    a.dst.bw = bw;
    a.cout = global_ptr(rfl64(sh_desc[2]));
    a.bw = bw;
    a.bwdiv = FastDiv{rfl(w[11]), rfl(w[12]), rfl(w[13])};
    a.ipbdiv = FastDiv{rfl(w[14]), rfl(w[15]), rfl(w[16])};
    a.sse = s.sse + k;
    return a;
}

__global__ __launch_bounds__(kServeTPW * 8) void k_serve(ServeArgs s) {
    constexpr int TPW = kServeTPW;
    __shared__ uint32_t lds[lds_words(TPW)];
    __shared__ long long red[TPW * 8 / 64];
    __shared__ uint32_t sh_k, sh_g, sh_cursor, sh_stop;
    __shared__ uint64_t sh_desc[16];  // descriptor of request `cur`
    const int tid = threadIdx.x;
    if (tid == 0) sh_cursor = 0;
    uint32_t cur = 0xffffffffu;
    uint32_t idle = 0;
    for (;;) {
        __syncthreads();  // the previous item is finished with LDS and sh_*
        if (tid == 0) {
            uint32_t k = max(sh_cursor, __hip_atomic_load(s.low, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            const uint32_t pub = load_sys(s.published);
            uint32_t res_k = 0xffffffffu, res_g = 0;
            while (k < pub) {
                const uint32_t n = load_sys(&s.desc[k].nitems);
                const uint32_t g = atomicAdd(s.claim + k, 1u);
                if (g < n) {
                    res_k = k;
                    res_g = g;
                    break;
                }
                atomicMax(s.low, k + 1);
                ++k;
            }
            sh_cursor = k;
            sh_k = res_k;
            sh_g = res_g;
        }
        __syncthreads();
        const uint32_t k = rfl(sh_k);
        if (k == 0xffffffffu) {
            if (tid == 0) sh_stop = (idle % 64u == 0u) ? load_sys(s.stop) : 0u;
            __syncthreads();
            if (rfl(sh_stop)) break;
            if (++idle > s.idle_polls) break;  // watchdog: the host relaunches on demand
            __builtin_amdgcn_s_sleep(127);
            continue;
        }
        idle = 0;
        const uint32_t g = rfl(sh_g);
        if (k != cur) {
            // first item of a request met by this workgroup: acquire, then read
            // its descriptor past the caches
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
            if (tid < 16) sh_desc[tid] = load_sys(reinterpret_cast<const uint64_t*>(s.desc + k) + tid);
            __syncthreads();
            cur = k;
        }
        const GroupArgs a = args_from_desc(sh_desc, s, k);
        const uint32_t* dw = reinterpret_cast<const uint32_t*>(sh_desc);
        const uint32_t nitems = rfl(dw[8]), tpi = rfl(dw[9]), nblk = rfl(dw[17]);
        const uint32_t t0 = g * tpi;
        const uint32_t gend = min(nblk, t0 + tpi);
        SseAcc acc{0, kNoImage};
        RowWords rows;
        uint32_t g0 = t0;
        load_group_rows<TPW, uint8_t>(a, g0, min((uint32_t)TPW, gend - g0), rows);
        for (uint32_t j = 0; g0 < gend; ++j, g0 += (uint32_t)TPW) {
            if (j) __syncthreads();
            const uint32_t g0n = g0 + (uint32_t)TPW;
            const uint32_t ntn = g0n < gend ? min((uint32_t)TPW, gend - g0n) : 0u;
            process_group<TPW, uint8_t, ServeMode>(a, g0, min((uint32_t)TPW, gend - g0), lds, red, acc, rows, g0n,
                                                  ntn, s.qs, s.dqs);
        }
        sse_flush<TPW * 8>(acc, a.sse, red);
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // this item's outputs and SSE
        if (tid == 0) {
            const uint32_t old = atomicAdd(s.done + k, 1u);
            if (old + 1u == nitems) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // every other item of k
                const long long v = (long long)__hip_atomic_load(s.sse + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&s.comp[k].sse, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                __hip_atomic_store(&s.comp[k].flag, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
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
    int32_t h = 0, w = 0;
    int64_t pitch = 0;
    int64_t bytes = 0, tiles = 0;
    int64_t t_arrival = 0, t_admit = -1, t_done = -1;
    int64_t off = -1;
    int64_t sse = -1;
    int state = kWaiting;
    int ev = -1;  // plain mode: event slot
};

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
    std::vector<int64_t> running;     // admitted, not yet done
    int64_t n_done = 0, n_cancelled = 0, loop_launches = 0;
    int hip_error = 0;

    hipStream_t copy_stream = nullptr, loop_stream = nullptr;
    // persistent mode
    ReqDesc* d_desc = nullptr;
    ReqDesc* h_desc = nullptr;        // pinned staging, one per request
    uint32_t* h_pubvals = nullptr;    // pinned: value k + 1 published after request k
    uint32_t* d_state = nullptr;      // published, low, then claim[n], done[n]
    unsigned long long* d_sse = nullptr;
    Completion* h_comp = nullptr;     // host-mapped
    Completion* d_comp = nullptr;     // its device address
    uint32_t* h_stop = nullptr;       // host-mapped
    uint32_t* d_stop = nullptr;
    hipEvent_t loop_done = nullptr;
    // plain mode
    std::vector<hipEvent_t> events;
    std::vector<int> free_events;
};

namespace {

uint32_t* st_published(adct_server* S) { return S->d_state; }
uint32_t* st_low(adct_server* S) { return S->d_state + 32; }
uint32_t* st_claim(adct_server* S) { return S->d_state + 64; }
uint32_t* st_done(adct_server* S) { return S->d_state + 64 + S->cfg.max_requests; }

bool hip_ok(adct_server* S, hipError_t e) {
    if (e != hipSuccess && !S->hip_error) S->hip_error = (int)e;
    return e == hipSuccess;
}

void launch_loop(adct_server* S) {
    ServeArgs a{};
    a.desc = S->d_desc;
    a.published = st_published(S);
    a.low = st_low(S);
    a.claim = st_claim(S);
    a.done = st_done(S);
    a.sse = S->d_sse;
    a.comp = S->d_comp;
    a.stop = S->d_stop;
    for (int c = 0; c < 5; ++c) {
        a.qs.f[c] = S->qs.f[c];
        a.dqs.f[c] = S->dqs.f[c];
    }
    a.idle_polls = (uint32_t)S->cfg.idle_polls;
    hipLaunchKernelGGL(k_serve, dim3((unsigned)(S->cus * S->cfg.wgs_per_cu)), dim3(kServeTPW * 8), 0,
                       S->loop_stream, a);
    hip_ok(S, hipGetLastError());
    hip_ok(S, hipEventRecord(S->loop_done, S->loop_stream));
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

PlaneRef plane_of(const char* p, int32_t w) {
    PlaneRef r;
    r.data = p;
    r.pitch = w;
    r.bw = (uint32_t)(w / 16);
    return r;
}

// Copies the request in and hands it to the device (called with mu held).
void issue(adct_server* S, int64_t k) {
    Req& r = S->reqs[(size_t)k];
    char* base = S->pool_mem + r.off;
    const int64_t plane = (int64_t)r.h * r.w;
    char* src = base;
    char* dst = base + Pool::round_up(plane);
    char* q = dst + Pool::round_up(plane);
    if (r.pitch == r.w)
        hip_ok(S, hipMemcpyAsync(src, r.host, (size_t)plane, hipMemcpyHostToDevice, S->copy_stream));
    else
        hip_ok(S, hipMemcpy2DAsync(src, (size_t)r.w, r.host, (size_t)r.pitch, (size_t)r.w, (size_t)r.h,
                                   hipMemcpyHostToDevice, S->copy_stream));
    if (S->cfg.mode == ADCT_SERVE_PERSISTENT) {
        ReqDesc& d = S->h_desc[k];
        memset(&d, 0, sizeof d);
        d.src = (uint64_t)(uintptr_t)src;
        d.dst = (uint64_t)(uintptr_t)dst;
        d.q = (uint64_t)(uintptr_t)q;
        d.height = (uint32_t)r.h;
        d.width = (uint32_t)r.w;
        d.nblk = (uint32_t)r.tiles;
        d.tiles_per_item = (uint32_t)S->cfg.tiles_per_item;
        d.nitems = (uint32_t)((r.tiles + S->cfg.tiles_per_item - 1) / S->cfg.tiles_per_item);
        d.bw = (uint32_t)(r.w / 16);
        const FastDiv fb = make_fastdiv(d.bw), fi = make_fastdiv((uint32_t)(r.h / 16));
        d.bw_m = fb.m;
        d.bw_s1 = fb.s1;
        d.bw_s2 = fb.s2;
        d.ipb_m = fi.m;
        d.ipb_s1 = fi.s1;
        d.ipb_s2 = fi.s2;
        S->h_pubvals[k] = (uint32_t)(k + 1);
        hip_ok(S, hipMemcpyAsync(S->d_desc + k, &d, sizeof d, hipMemcpyHostToDevice, S->copy_stream));
        hip_ok(S, hipMemcpyAsync(st_published(S), S->h_pubvals + k, sizeof(uint32_t), hipMemcpyHostToDevice,
                                 S->copy_stream));
        if (loop_exited(S) && !S->stopping) launch_loop(S);
    } else {
        adct_plane ps{src, ADCT_U8, r.h, r.w, 0, r.w};
        adct_plane pd{dst, ADCT_U8, r.h, r.w, 0, r.w};
        int rc = adct_fwd2d_quant(&ps, S->cfg.qp, reinterpret_cast<int16_t*>(q), S->copy_stream);
        if (!rc)
            rc = adct_dequant_recon(reinterpret_cast<int16_t*>(q), S->cfg.qp, &pd, &ps, r.h,
                                    reinterpret_cast<int64_t*>(S->d_sse + k), S->copy_stream);
        if (rc && !S->hip_error) S->hip_error = rc;
        hip_ok(S, hipMemcpyAsync(&S->h_comp[k].sse, S->d_sse + k, sizeof(int64_t), hipMemcpyDeviceToHost,
                                 S->copy_stream));
        r.ev = S->free_events.back();
        S->free_events.pop_back();
        hip_ok(S, hipEventRecord(S->events[(size_t)r.ev], S->copy_stream));
    }
}

void release_mem(adct_server* S, Req& r) {
    if (r.off >= 0) {
        S->pool->release(r.off, r.bytes);
        r.off = -1;
        --S->inflight;
    }
}

// Completions (called with mu held); returns whether any request finished.
bool poll_done(adct_server* S, int64_t now) {
    bool any = false;
    for (size_t i = 0; i < S->running.size();) {
        const int64_t k = S->running[i];
        Req& r = S->reqs[(size_t)k];
        bool fin = false;
        if (S->cfg.mode == ADCT_SERVE_PERSISTENT) {
            fin = __atomic_load_n(&S->h_comp[k].flag, __ATOMIC_ACQUIRE) != 0;
        } else {
            const hipError_t e = hipEventQuery(S->events[(size_t)r.ev]);
            fin = e == hipSuccess;
            if (e != hipSuccess && e != hipErrorNotReady) hip_ok(S, e);
        }
        if (fin) {
            r.sse = __atomic_load_n(&S->h_comp[k].sse, __ATOMIC_ACQUIRE);
            r.t_done = now;
            r.state = kDone;
            if (r.ev >= 0) {
                S->free_events.push_back(r.ev);
                r.ev = -1;
            }
            if (S->cfg.auto_release) {
                release_mem(S, r);
                r.state = kReleased;
            }
            ++S->n_done;
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
                r.state = kRunning;
                S->running.push_back(i);
                issue(S, i);
                ++admitted;
            });
        const bool fin = poll_done(S, clock_ns());
        if (S->cfg.mode == ADCT_SERVE_PERSISTENT && !S->running.empty() && !S->stopping && loop_exited(S))
            launch_loop(S);  // the loop went idle and exited before this work was published
        if (fin) S->done_cv.notify_all();
        if (!admitted && !fin) {
            // nothing happened: wait for a submission, a release, or the next poll
            int64_t wait_ns = S->running.empty() ? 200000 : 5000;
            if (S->head < n && S->reqs[(size_t)S->head].state == kWaiting) {
                const int64_t until = S->reqs[(size_t)S->head].t_arrival - now;
                if (until > 0 && until < wait_ns) wait_ns = until;
            }
            S->cv.wait_for(lk, std::chrono::nanoseconds(wait_ns));
        }
    }
}

void free_server(adct_server* S) {
    if (S->loop_done) (void)hipEventDestroy(S->loop_done);
    for (hipEvent_t e : S->events) (void)hipEventDestroy(e);
    if (S->copy_stream) (void)hipStreamDestroy(S->copy_stream);
    if (S->loop_stream) (void)hipStreamDestroy(S->loop_stream);
    if (S->pool_mem) (void)hipFree(S->pool_mem);
    if (S->d_desc) (void)hipFree(S->d_desc);
    if (S->d_state) (void)hipFree(S->d_state);
    if (S->d_sse) (void)hipFree(S->d_sse);
    if (S->h_desc) (void)hipHostFree(S->h_desc);
    if (S->h_pubvals) (void)hipHostFree(S->h_pubvals);
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
    if (cfg.tiles_per_item == 0) cfg.tiles_per_item = 128;
    if (cfg.wgs_per_cu == 0) cfg.wgs_per_cu = 2;
    if (cfg.idle_polls == 0) cfg.idle_polls = 1000000;
    if (cfg.pool_bytes < 1024 || cfg.max_inflight < 1 || cfg.max_requests < 1 || cfg.tiles_per_item < 16 ||
        cfg.tiles_per_item % 16 || cfg.wgs_per_cu < 1 || cfg.wgs_per_cu > 8 || cfg.idle_polls < 1 ||
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
    bool ok = hipMalloc(reinterpret_cast<void**>(&S->pool_mem), (size_t)S->pool->capacity()) == hipSuccess &&
              hipMalloc(reinterpret_cast<void**>(&S->d_sse), n * sizeof(unsigned long long)) == hipSuccess &&
              hipMemset(S->d_sse, 0, n * sizeof(unsigned long long)) == hipSuccess &&
              hipHostMalloc(reinterpret_cast<void**>(&S->h_comp), n * sizeof(Completion),
                            hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess &&
              hipHostMalloc(reinterpret_cast<void**>(&S->h_stop), 128, hipHostMallocMapped | hipHostMallocCoherent) ==
                  hipSuccess &&
              hipStreamCreateWithFlags(&S->copy_stream, hipStreamNonBlocking) == hipSuccess;
    if (ok) {
        memset(S->h_comp, 0, n * sizeof(Completion));
        *S->h_stop = 0;
        ok = hipHostGetDevicePointer(reinterpret_cast<void**>(&S->d_comp), S->h_comp, 0) == hipSuccess &&
             hipHostGetDevicePointer(reinterpret_cast<void**>(&S->d_stop), S->h_stop, 0) == hipSuccess;
    }
    if (ok && cfg.mode == ADCT_SERVE_PERSISTENT) {
        const size_t state_words = 64 + 2 * n;
        ok = hipMalloc(reinterpret_cast<void**>(&S->d_desc), n * sizeof(ReqDesc)) == hipSuccess &&
             hipMalloc(reinterpret_cast<void**>(&S->d_state), state_words * sizeof(uint32_t)) == hipSuccess &&
             hipMemset(S->d_state, 0, state_words * sizeof(uint32_t)) == hipSuccess &&
             hipHostMalloc(reinterpret_cast<void**>(&S->h_desc), n * sizeof(ReqDesc), 0) == hipSuccess &&
             hipHostMalloc(reinterpret_cast<void**>(&S->h_pubvals), n * sizeof(uint32_t), 0) == hipSuccess &&
             hipStreamCreateWithFlags(&S->loop_stream, hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&S->loop_done, hipEventDisableTiming) == hipSuccess &&
             hipDeviceSynchronize() == hipSuccess;
    }
    if (ok && cfg.mode == ADCT_SERVE_PLAIN) {
        S->events.resize((size_t)cfg.max_inflight, nullptr);
        for (int i = 0; ok && i < cfg.max_inflight; ++i) {
            ok = hipEventCreateWithFlags(&S->events[(size_t)i], hipEventDisableTiming) == hipSuccess;
            S->free_events.push_back(i);
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
    const int64_t plane = (int64_t)height * width;
    r.bytes = 2 * Pool::round_up(plane) + 2 * plane;
    r.tiles = plane / 256;
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
        char* base = S->pool_mem + r.off;
        const int64_t plane = (int64_t)r.h * r.w;
        out->dst = base + Pool::round_up(plane);
        out->q = base + 2 * Pool::round_up(plane);
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
        // idle workgroups see the flag within a few polls
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
    (void)hipStreamSynchronize(S->copy_stream);
    free_server(S);
    return rc;
}

// ---- host-policy simulation (no GPU) ------------------------------------------

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
