// api.hip -- the C ABI of libws (declared in include/ws.h): argument
// validation, the context's grow-only device scratch, and the host-side
// orchestration of the watershed (Alg. 1), waterfall (Section 4, Alg. 5 layer
// loop) and gradient kernels on the caller's stream.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "ws.h"
#include "ws_kernels.h"

using wsk::Geom;
using wsk::Launch;

namespace {

constexpr int kCounterSlots = 64;   // Step II per-sweep change counters (ring)
constexpr int kMaxSweepBatch = 32;
constexpr size_t kMaxGraphs = 16;   // instantiated launch graphs kept per context

struct Buf {
    void *p = nullptr;
    size_t n = 0;
};

thread_local std::string g_noctx_error;

}  // namespace

// Fixed device scratch of ws_watershed_noalloc, one copy per device, held
// until the process ends. Host code never uses this name as an address (on
// the host it only stands for the symbol): kernels get the per-device address
// that hipGetSymbolAddress returned (noalloc_scratch_of).
constexpr size_t kNoAllocBytes = (size_t)WS_NOALLOC_SCRATCH_MIB << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[kMaxDevices] = {};
std::string g_noalloc_why;   // why the last set-up failed

// Looks up the address of `scratch` on `device`, which must be current; once
// per device.
int noalloc_setup(int device, std::string &why) {
    if (device < 0 || device >= kMaxDevices) {
        why = "device index above the fixed scratch table";
        return WS_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (g_noalloc_ptr[device]) return WS_OK;
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        why = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
        return WS_EDEVICE;
    }
    g_noalloc_ptr[device] = ptr;
    return WS_OK;
}

void *noalloc_scratch_of(int device) {
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    return device >= 0 && device < kMaxDevices ? g_noalloc_ptr[device] : nullptr;
}

}  // namespace

struct ws_ctx {
    int device = 0;
    size_t budget = 0;                    // device scratch limit in bytes (0 = none)
    size_t held = 0;                      // device scratch bytes held now
    std::string err;
    Buf D, stamp, cnt, rec;               // watershed scratch
    Buf key, par, cimg, rlist, mlab;      // waterfall: region tables (dense by id), per-pixel region ids
    Buf rimg;                             // reconstruction waterfall: the raised image (uint16)
    Buf ragoff, ragbuf;                   // adjacency graph export: edge offsets, sort buffers
    Buf edges, ecnt, wfcnt;               // edge slabs, their counts, region count
    Buf g0, g1, mag, gmax;                // gradient scratch
    Buf chunks, tilecnt;                  // region-id rank tables + scan scratch, per-tile counts
    Buf tab;                              // batch descriptor table + tile maps
    int32_t *host_cnt = nullptr;          // pinned readback of counters (kCounterSlots + 1 words;
                                          // the last one is written by captured watershed graphs)
    hipEvent_t sweep_ev = nullptr;        // recorded by captured watershed graphs after their sweeps
    void *stage = nullptr;                // pinned staging of batch tables
    size_t stage_n = 0;
    hipEvent_t stage_ev = nullptr;        // last upload from `stage`
    bool stage_pending = false;
    int step3 = 0, rr = 6, sweep_batch = 4;
    int tile2 = 2, tile3 = 3;             // watershed tile shape ids of 2D / 3D images
    int schedule = 0, step4 = 0;           // per-pixel schedule, PRW Step IV
    int64_t max_sweeps = 0x7fffffff;
    bool timing = false;
    // launch graphs: a call signature seen once is captured on its next use
    // and replayed from then on, while no scratch buffer has moved (gen)
    bool graph = false;
    bool capturing = false;
    uint64_t gen = 0;
    hipStream_t cap = nullptr;
    struct Graph {
        std::string sig;
        uint64_t gen;
        uint64_t used;
        hipGraphExec_t exec;
        void *owned = nullptr;   // device buffer only this graph's kernels read (batch tables)
        size_t owned_n = 0;
        int32_t sweeps = 0;      // Step II sweeps it launches after the initial pass (0: none)
    };
    std::vector<Graph> graphs;
    std::map<std::string, uint64_t> seen;
    // Step II sweeps (after the initial tile pass) a captured watershed call
    // launches: one more than the sweeps that changed something when the
    // signature last ran directly
    std::map<std::string, int32_t> graph_sweeps;
    int32_t cap_sweeps = 0;               // while capturing a watershed: that count
    uint64_t tick = 0;
    wsk::TimingSink sink;
    int64_t stats[7] = {0, 0, 0, 0, 0, 0, 0};
};

namespace {

int fail(ws_ctx *c, int code, const std::string &msg) {
    if (c) c->err = msg;
    else g_noctx_error = msg;
    return code;
}

int hip_fail(ws_ctx *c, hipError_t e, const char *where) {
    return fail(c, WS_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

int ensure(ws_ctx *c, Buf &b, size_t bytes, const char *what) {
    if (bytes == 0) bytes = 256;
    if (b.n >= bytes) return WS_OK;
    if (c->capturing) return fail(c, WS_EUNSUPPORTED, std::string("allocation during graph capture: ") + what);
    // the context's scratch budget: the exact size when geometric growth would
    // exceed it, WS_ENOMEM when even that does
    const size_t need = bytes;
    if (c->budget && c->held - b.n + need > c->budget)
        return fail(c, WS_ENOMEM, std::string("scratch budget of ") + std::to_string(c->budget) +
                                      " bytes exceeded: " + what + " needs " + std::to_string(need) + " bytes, " +
                                      std::to_string(c->held - b.n) + " held by other buffers");
    ++c->gen;  // cached launch graphs hold the old address
    // grow geometrically: hipFree waits for the whole device, so a context
    // that serves growing batches should reallocate rarely
    if (b.n > 0 && bytes < b.n + b.n / 2) bytes = b.n + b.n / 2;
    if (c->budget && c->held - b.n + bytes > c->budget) bytes = need;
    if (b.p) {
        hipError_t e = hipFree(b.p);
        c->held -= b.n;
        b.p = nullptr;
        b.n = 0;
        if (e != hipSuccess) return hip_fail(c, e, "hipFree");
    }
    hipError_t e = hipMalloc(&b.p, bytes);
    ++c->stats[5];
    if (e != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return fail(c, WS_ENOMEM, std::string("cannot allocate ") + std::to_string(bytes) + " bytes for " + what);
    }
    b.n = bytes;
    c->held += bytes;
    return WS_OK;
}

// Pinned host staging of at least `bytes` for the batch tables. A previous
// batch's copy out of it must have finished before it is rewritten or freed.
int ensure_stage(ws_ctx *c, size_t bytes) {
    if (c->stage_pending) {
        hipError_t e = hipEventSynchronize(c->stage_ev);
        if (e != hipSuccess) return hip_fail(c, e, "hipEventSynchronize");
        c->stage_pending = false;
    }
    if (!c->stage_ev) {
        hipError_t e = hipEventCreateWithFlags(&c->stage_ev, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(c, e, "hipEventCreate");
    }
    if (c->stage_n >= bytes) return WS_OK;
    if (c->stage) (void)hipHostFree(c->stage);
    c->stage = nullptr;
    c->stage_n = 0;
    hipError_t e = hipHostMalloc(&c->stage, bytes, hipHostMallocDefault);
    ++c->stats[5];
    if (e != hipSuccess) return hip_fail(c, e, "hipHostMalloc");
    c->stage_n = bytes;
    return WS_OK;
}

// Sizes: every dim >= 1, N < 2^31, and the tile grid fits the launch limits.
bool valid_dims(int64_t nx, int64_t ny, int64_t nz, std::string &why) {
    if (nx < 1 || ny < 1 || nz < 1) { why = "every dimension must be >= 1"; return false; }
    if (nx >= (1LL << 31) || ny >= (1LL << 31) || nz >= (1LL << 31)) { why = "dimension too large"; return false; }
    if (nx * ny >= (1LL << 31) || nx * ny * nz >= (1LL << 31)) { why = "nx*ny*nz must be < 2^31"; return false; }
    return true;
}

bool valid_conn(int64_t nz, int conn) {
    return nz == 1 ? (conn == 4 || conn == 8) : (conn == 6 || conn == 26);
}

// Sizes and the watershed tiling of tile shape `shape` (an id of TileShape;
// the defaults are 2 for 2D and 3 for 3D images).
Geom make_geom(int64_t nx, int64_t ny, int64_t nz, int shape) {
    Geom g;
    g.nx = (int32_t)nx;
    g.ny = (int32_t)ny;
    g.nz = (int32_t)nz;
    g.n = (int32_t)(nx * ny * nz);
    int TX = 1, TY = 1, TZ = 1;
    if (!wsk::tile_dims(shape, TX, TY, TZ)) wsk::tile_dims(nz > 1 ? 3 : 2, TX, TY, TZ);
    g.ntx = (int32_t)((nx + TX - 1) / TX);
    g.nty = (int32_t)((ny + TY - 1) / TY);
    g.ntz = (int32_t)((nz + TZ - 1) / TZ);
    g.dnx = wsk::FastDiv((uint32_t)nx);
    g.dny = wsk::FastDiv((uint32_t)ny);
    return g;
}

// The watershed tile shape the context uses for images of `ndim` dimensions.
int shape_of(const ws_ctx *c, int ndim) { return ndim == 3 ? c->tile3 : c->tile2; }

int set_device(ws_ctx *c) {
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    return WS_OK;
}

Launch make_launch(ws_ctx *c, void *stream) {
    Launch lc;
    lc.stream = (hipStream_t)stream;
    lc.timing = c->timing ? &c->sink : nullptr;
    return lc;
}

// A graphed call's verdict after a graph launch: the graph's result does not
// hold (its Step II sweep count was too small), run the call directly.
constexpr int kRerun = 1;

void drop_graph(ws_ctx *c, size_t i) {
    ws_ctx::Graph &g = c->graphs[i];
    (void)hipGraphExecDestroy(g.exec);
    if (g.owned) {
        (void)hipFree(g.owned);   // waits for the device: no replay still reads it
        c->held -= std::min(c->held, g.owned_n);
    }
    c->graphs.erase(c->graphs.begin() + (long)i);
}

struct NoPrep {
    int operator()(void **, size_t *) const { return WS_OK; }
};
struct NoCheck {
    int operator()(const ws_ctx::Graph &) const { return WS_OK; }
};

// Enqueues through `enqueue(Launch&)`, or replays its captured graph. Without
// the graph option (or with per-launch timing) it simply enqueues on `stream`.
// A signature's first use runs directly (allocating what it needs); its
// second use is captured on the context's own stream (the caller's may be
// the legacy stream, which cannot be captured), instantiated and launched on
// `stream`; later uses replay. If capture fails the call runs directly.
// `prep(&owned, &bytes)` runs before a capture: it may allocate a device
// buffer the graph alone reads (freed with the graph), or return kRerun to
// run the call directly instead. `check(graph)` runs after every launch of
// the graph; kRerun drops the graph and runs the call directly (the next
// identical call is captured again).
template <class F, class P = NoPrep, class K = NoCheck>
int run_graphed(ws_ctx *c, void *stream, const std::string &sig, F &&enqueue, P &&prep = P(), K &&check = K()) {
    if (!c->graph || c->timing) {
        Launch lc = make_launch(c, stream);
        return enqueue(lc);
    }
    auto launch_checked = [&](size_t gi) -> int {
        ws_ctx::Graph &g = c->graphs[gi];
        g.used = ++c->tick;
        ++c->stats[4];
        // a watershed graph writes its last sweep's count here; -1 until it has
        if (g.sweeps > 0) ((volatile int32_t *)c->host_cnt)[kCounterSlots] = -1;
        hipError_t e = hipGraphLaunch(g.exec, (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(c, e, "hipGraphLaunch");
        int v = check(g);
        if (v != kRerun) return v;
        drop_graph(c, gi);
        Launch lc = make_launch(c, stream);
        return enqueue(lc);
    };
    for (size_t i = 0; i < c->graphs.size(); ++i)
        if (c->graphs[i].sig == sig && c->graphs[i].gen == c->gen) return launch_checked(i);
    auto it = c->seen.find(sig);
    if (it == c->seen.end() || it->second != c->gen) {
        c->seen[sig] = c->gen;
        Launch lc = make_launch(c, stream);
        return enqueue(lc);
    }
    hipError_t e;
    if (!c->cap && (e = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(c, e, "hipStreamCreateWithFlags");
    void *owned = nullptr;
    size_t owned_n = 0;
    int rc = prep(&owned, &owned_n);
    auto release = [&]() {
        if (owned) {
            (void)hipFree(owned);
            c->held -= std::min(c->held, owned_n);
        }
        owned = nullptr;
        c->cap_sweeps = 0;
    };
    if (rc != WS_OK) {
        release();
        if (rc != kRerun) return rc;
        Launch lc = make_launch(c, stream);
        return enqueue(lc);
    }
    if ((e = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
        (void)hipGetLastError();
        release();
        Launch lc = make_launch(c, stream);
        return enqueue(lc);
    }
    c->capturing = true;
    Launch cl = make_launch(c, c->cap);
    cl.timing = nullptr;
    rc = enqueue(cl);
    c->capturing = false;
    const int32_t sweeps = c->cap_sweeps;
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(c->cap, &graph);
    hipGraphExec_t exec = nullptr;
    if (rc == WS_OK && e == hipSuccess && graph) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (rc != WS_OK || e != hipSuccess || !exec) {
        (void)hipGetLastError();
        c->err.clear();
        release();
        Launch lc = make_launch(c, stream);
        return enqueue(lc);
    }
    c->cap_sweeps = 0;
    if (c->graphs.size() >= kMaxGraphs) {
        size_t old = 0;
        for (size_t i = 1; i < c->graphs.size(); ++i)
            if (c->graphs[i].used < c->graphs[old].used) old = i;
        drop_graph(c, old);
    }
    ws_ctx::Graph g;
    g.sig = sig;
    g.gen = c->gen;
    g.used = ++c->tick;
    g.exec = exec;
    g.owned = owned;
    g.owned_n = owned_n;
    g.sweeps = sweeps;
    c->graphs.push_back(g);
    return launch_checked(c->graphs.size() - 1);
}

std::string sig_of(const char *what, std::initializer_list<uint64_t> v) {
    std::string s(what);
    for (uint64_t x : v) s += ":" + std::to_string(x);
    return s;
}

#define WS_TRY(expr)                                                      \
    do {                                                                  \
        int _rc = (expr);                                                 \
        if (_rc != 0) {                                                   \
            if (_rc == -3) return hip_fail(c, lc.last, "kernel launch");  \
            return fail(c, WS_EINVAL, "unsupported configuration");       \
        }                                                                 \
    } while (0)

// One connectivity's share of a call: its images' tiles in the watershed and
// waterfall tilings (a contiguous range of each, starting at ws0 / wf0), with
// sources that map those tiles to images (tile indices relative to the range).
// A single-image call has one part; a batch has one per connectivity present.
template <class Src>
struct Part {
    Src ws, wf;
    int32_t nws = 0, nwf = 0;
    int32_t ws0 = 0, wf0 = 0;
    int conn = 0, ndim = 0;
    int shape = 0;   // watershed tile shape id
};

wsk::TileGrid full_grid(int32_t ntiles) {
    wsk::TileGrid tg;
    tg.ntiles = ntiles;
    tg.grid = ntiles > 0 ? ntiles : 1;
    return tg;
}

template <class Src>
int32_t ws_tiles_of(const std::vector<Part<Src>> &parts) {
    int32_t n = 0;
    for (auto &p : parts) n += p.nws;
    return n;
}

// Border records of every part, one after the other.
template <class Src>
size_t rec_ints(const std::vector<Part<Src>> &parts) {
    size_t n = 0;
    for (auto &p : parts) n += (size_t)p.nws * (size_t)wsk::record_ints(p.shape);
    return n;
}

// Device scratch of one watershed call: distances (one per pixel of the
// arena), four stamp words per watershed tile, kCounterSlots sweep counters
// and the parts' border records.
struct WsScratch {
    int32_t *D = nullptr, *stamp = nullptr, *cnt = nullptr, *rec = nullptr;
};

// The watershed's scratch for `arena` pixels in the context's buffers,
// allocated before anything is launched.
template <class Src>
int prepare_watershed(ws_ctx *c, const std::vector<Part<Src>> &parts, size_t arena, bool records, WsScratch &ws) {
    int rc;
    if ((rc = ensure(c, c->D, arena * 4, "distances")) != WS_OK) return rc;
    // per tile and sweep parity: the last sweep that changed its border, and
    // the faces it changed
    if ((rc = ensure(c, c->stamp, (size_t)ws_tiles_of(parts) * 16, "tile stamps")) != WS_OK) return rc;
    if ((rc = ensure(c, c->cnt, kCounterSlots * 4, "counters")) != WS_OK) return rc;
    if (records && (rc = ensure(c, c->rec, rec_ints(parts) * 4, "border records")) != WS_OK) return rc;
    ws.D = (int32_t *)c->D.p;
    ws.stamp = (int32_t *)c->stamp.p;
    ws.cnt = (int32_t *)c->cnt.p;
    ws.rec = records ? (int32_t *)c->rec.p : nullptr;
    return WS_OK;
}

// Step II to convergence: the initial tile pass, then batches of sweeps with
// one counter read-back per batch. Every part's sweep s reads the count of
// sweep s - 1 over all parts. Leaves D converged in c->D (arena-wide).
template <class Src>
int run_distances(ws_ctx *c, Launch &lc, const std::vector<Part<Src>> &parts, bool u16, const WsScratch &ws) {
    const int32_t nt = ws_tiles_of(parts);
    int32_t *D = ws.D, *stamp = ws.stamp, *cnt = ws.cnt;
    WS_TRY(wsk::launch_fill2_i32(lc, stamp, 4 * nt, -1, cnt, kCounterSlots, 0));
    for (auto &p : parts)
        WS_TRY(wsk::launch_ws_init(lc, p.ws, full_grid(p.nws), p.conn, p.shape, u16, D, stamp + 4 * (size_t)p.ws0, cnt));
    if (c->capturing) {
        // a captured call cannot read counters back: it launches a fixed
        // number of sweeps (a sweep after one that changed nothing returns at
        // once), and the graph's check reads the count of the last one
        const int32_t K = c->cap_sweeps;
        if (K < 1 || K >= kCounterSlots) return fail(c, WS_EUNSUPPORTED, "sweep count of a captured call");
        for (int32_t s = 1; s <= K; ++s)
            for (auto &p : parts)
                WS_TRY(wsk::launch_ws_sweep(lc, p.ws, full_grid(p.nws), p.conn, p.shape, u16, D, stamp + 4 * (size_t)p.ws0,
                                            cnt + s, cnt + (s - 1), s));
        // the last sweep's count to pinned host memory, then an event: the
        // call waits for that much of the graph only, the rest keeps running
        hipError_t e = hipMemcpyAsync(c->host_cnt + kCounterSlots, cnt + K, 4, hipMemcpyDeviceToHost, lc.stream);
        if (e != hipSuccess) return hip_fail(c, e, "hipMemcpyAsync");
        if ((e = hipEventRecord(c->sweep_ev, lc.stream)) != hipSuccess) return hip_fail(c, e, "hipEventRecord");
        c->stats[0] = K + 1;
        c->stats[3] = nt;
        return WS_OK;
    }
    int64_t launched = 1, changing = 0;
    int32_t s = 1;
    bool first = true;
    int batch = std::max(1, std::min(c->sweep_batch, kMaxSweepBatch));
    for (;;) {
        if (!first) {
            // this batch's counters only: each sweep reads the count of the
            // sweep before it (the last of the previous batch included)
            const int a = s % kCounterSlots, m = std::min(batch, kCounterSlots - a);
            WS_TRY(wsk::launch_fill_i32(lc, cnt + a, m, 0));
            if (m < batch) WS_TRY(wsk::launch_fill_i32(lc, cnt, batch - m, 0));
        }
        int32_t s0 = s;
        for (int b = 0; b < batch; ++b, ++s)
            for (auto &p : parts)
                WS_TRY(wsk::launch_ws_sweep(lc, p.ws, full_grid(p.nws), p.conn, p.shape, u16, D, stamp + 4 * (size_t)p.ws0,
                                            cnt + (s % kCounterSlots), cnt + ((s - 1) % kCounterSlots), s));
        launched += batch;
        hipError_t e = hipMemcpyAsync(c->host_cnt, cnt, kCounterSlots * 4, hipMemcpyDeviceToHost, lc.stream);
        if (e != hipSuccess) return hip_fail(c, e, "hipMemcpyAsync");
        e = hipStreamSynchronize(lc.stream);
        if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
        bool done = false;
        if (first) {
            if (c->host_cnt[0] == 0) done = true;
            else changing = 1;
        }
        for (int32_t t = s0; !done && t < s; ++t) {
            if (c->host_cnt[t % kCounterSlots] == 0) done = true;
            else ++changing;
        }
        first = false;
        if (done) break;
        if (changing >= c->max_sweeps) {
            c->stats[0] = launched;
            c->stats[1] = changing;
            return fail(c, WS_ENOCONV, "Step II did not converge within max_sweeps");
        }
    }
    c->stats[0] = launched;
    c->stats[1] = changing;
    c->stats[3] = nt;
    return WS_OK;
}

// Watershed of every image of every part into its lab (layer 0). The scratch
// must have been prepared (prepare_watershed with records).
template <class Src>
int run_watershed(ws_ctx *c, Launch &lc, const std::vector<Part<Src>> &parts, bool u16, const WsScratch &ws) {
    int rc;
    c->stats[2] = 0;
    c->stats[6] = 0;
    if ((rc = run_distances(c, lc, parts, u16, ws)) != WS_OK) return rc;
    int32_t *rec = ws.rec;
    const int32_t *D = ws.D;
    size_t ro = 0;
    for (auto &p : parts) {
        WS_TRY(wsk::launch_ws_label(lc, p.ws, full_grid(p.nws), p.conn, p.shape, u16, D, rec + ro));
        WS_TRY(wsk::launch_ws_merge(lc, p.ws, full_grid(p.nws), p.conn, p.shape, u16, rec + ro));
        ro += (size_t)p.nws * (size_t)wsk::record_ints(p.shape);
    }
    if (c->step3 == 0) {
        for (auto &p : parts) WS_TRY(wsk::launch_ws_find(lc, p.ws, full_grid(p.nws), p.conn, p.shape));
    } else {
        int32_t *cnt = ws.cnt;
        int64_t syncs = 0;
        for (;;) {
            WS_TRY(wsk::launch_fill_i32(lc, cnt, 1, 0));
            for (auto &p : parts) WS_TRY(wsk::launch_ws_jump(lc, p.ws, full_grid(p.nws), p.conn, p.shape, c->rr, cnt));
            hipError_t e = hipMemcpyAsync(c->host_cnt, cnt, 4, hipMemcpyDeviceToHost, lc.stream);
            if (e != hipSuccess) return hip_fail(c, e, "hipMemcpyAsync");
            if ((e = hipStreamSynchronize(lc.stream)) != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
            if (c->host_cnt[0] == 0) break;
            ++syncs;
        }
        c->stats[2] = syncs;
    }
    return WS_OK;
}

// After a direct watershed run of signature `sig`: the sweeps a captured
// replay launches (one more than the initial pass and the sweeps that changed
// something, plus one spare; the counter ring bounds it).
void note_sweeps(ws_ctx *c, const std::string &sig) {
    c->graph_sweeps[sig] = (int32_t)std::min<int64_t>(c->stats[1] + 2, kCounterSlots);
}

// Before capturing a watershed signature: its sweep count, or kRerun when it
// has not run directly yet or needs more sweeps than a graph holds.
int prep_sweeps(ws_ctx *c, const std::string &sig) {
    auto it = c->graph_sweeps.find(sig);
    if (it == c->graph_sweeps.end() || it->second < 1 || it->second >= kCounterSlots) return kRerun;
    if (!c->sweep_ev) {
        hipError_t e = hipEventCreateWithFlags(&c->sweep_ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            c->sweep_ev = nullptr;
            return kRerun;
        }
    }
    c->cap_sweeps = it->second;
    return WS_OK;
}

// After a launch of a watershed graph: waits until the graph's sweeps are
// done (the rest of the graph keeps running) and reads the last sweep's
// count: zero means Step II had converged; otherwise kRerun. If the count has
// not arrived when the event reports completion, the call waits for the whole
// stream; a count still missing then counts as not converged.
int check_sweeps(ws_ctx *c, const ws_ctx::Graph &g, void *stream) {
    if (g.sweeps <= 0) return WS_OK;
    volatile int32_t *flag = (volatile int32_t *)c->host_cnt + kCounterSlots;
    hipError_t e = hipEventSynchronize(c->sweep_ev);
    if (e != hipSuccess) return hip_fail(c, e, "hipEventSynchronize");
    if (*flag < 0 && (e = hipStreamSynchronize((hipStream_t)stream)) != hipSuccess)
        return hip_fail(c, e, "hipStreamSynchronize");
    c->stats[0] = g.sweeps + 1;
    return *flag == 0 ? WS_OK : kRerun;
}

// Launches launch(i, counter) for i = 1, 2, ... in batches of sweep_batch,
// each with a change counter of its own, and reads the batch's counters back
// once; stops after the first launch that changed nothing. `changing` counts
// the launches that changed something; reaching `cap` of them is WS_ENOCONV.
template <class F>
int repeat_until_stable(ws_ctx *c, Launch &lc, int64_t cap, const char *what, int64_t &launched, int64_t &changing,
                        F launch) {
    int rc;
    if ((rc = ensure(c, c->cnt, kCounterSlots * 4, "counters")) != WS_OK) return rc;
    int32_t *cnt = (int32_t *)c->cnt.p;
    const int batch = std::max(1, std::min(c->sweep_batch, kMaxSweepBatch));
    launched = changing = 0;
    for (;;) {
        WS_TRY(wsk::launch_fill_i32(lc, cnt, batch, 0));
        for (int b = 0; b < batch; ++b) WS_TRY(launch((int32_t)(launched + b + 1), cnt + b));
        launched += batch;
        hipError_t e = hipMemcpyAsync(c->host_cnt, cnt, (size_t)batch * 4, hipMemcpyDeviceToHost, lc.stream);
        if (e != hipSuccess) return hip_fail(c, e, "hipMemcpyAsync");
        if ((e = hipStreamSynchronize(lc.stream)) != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
        for (int b = 0; b < batch; ++b) {
            if (c->host_cnt[b] == 0) return WS_OK;
            ++changing;
        }
        if (changing >= cap) return fail(c, WS_ENOCONV, std::string(what) + " did not converge within max_sweeps");
    }
}

// The per-pixel synchronous schedule of one image (option "schedule" = 1):
// Step I, Step II sweeps until one resolves nothing, Step III by Find (APRUF)
// or RR jumps per launch (PRUF), Step IV by union-find or by the PRW
// exchange passes, then canonical labels, all in L. With `bal`, stops after
// Step II and writes the balanced states to bal (L then holds the arrows).
int run_watershed_px(ws_ctx *c, Launch &lc, const wsk::Geom &g, const void *grad, int conn, bool u16, int32_t *L,
                     int32_t *bal) {
    int rc;
    for (int i = 0; i < 4; ++i) c->stats[i] = 0;
    c->stats[6] = 0;
    if ((rc = ensure(c, c->D, (size_t)g.n * 4, "distances")) != WS_OK) return rc;
    int32_t *S = (int32_t *)c->D.p;
    WS_TRY(wsk::launch_px_step1(lc, g, conn, u16, grad, L, S));
    int64_t launched = 0, changing = 0;
    rc = repeat_until_stable(c, lc, c->max_sweeps, "Step II", launched, changing, [&](int32_t s, int32_t *cnt) {
        return wsk::launch_px_sweep(lc, g, conn, u16, grad, L, S, s, cnt);
    });
    c->stats[0] = launched + 1;
    c->stats[1] = changing;
    if (rc != WS_OK) return rc;
    if (bal) {
        WS_TRY(wsk::launch_px_stages(lc, g, S, bal));
        return WS_OK;
    }
    const int64_t no_cap = INT64_MAX;
    if (c->step3 == 0) {
        WS_TRY(wsk::launch_px_find(lc, g, L));
    } else {
        rc = repeat_until_stable(c, lc, no_cap, "Step III", launched, changing, [&](int32_t, int32_t *cnt) {
            return wsk::launch_px_jump(lc, g, L, c->rr, cnt);
        });
        if (rc != WS_OK) return rc;
        c->stats[2] = changing;
    }
    if (c->step4 == 0) {
        WS_TRY(wsk::launch_px_union(lc, g, conn, S, L));
        WS_TRY(wsk::launch_px_find(lc, g, L));
    } else {
        rc = repeat_until_stable(c, lc, no_cap, "Step IV", launched, changing, [&](int32_t, int32_t *cnt) {
            return wsk::launch_px_prw(lc, g, conn, S, L, cnt);
        });
        if (rc != WS_OK) return rc;
        c->stats[6] = changing;
    }
    WS_TRY(wsk::launch_fill_i32(lc, S, g.n, 0x7fffffff));
    WS_TRY(wsk::launch_px_canon(lc, g, L, S));
    return WS_OK;
}

// The waterfall's device buffers for `arena` pixels: region-id tables and
// per-chunk counts always; with `tables`, the region tables, the per-pixel ids,
// NL - 1 layer tables and the edge slabs.
struct WfBufs {
    wsk::WfIds ids;
    int32_t *scan_tmp, *nreg0, *cnt;
    uint64_t *key;
    int32_t *par, *cimg, *rlist, *mlab;
    wsk::EdgeSlabs es;
};

// Layer tables: for NL == 2 layer 1 by region id (arena ints: region counts
// are only known on the device). For NL >= 3 one record per region id
// {layer-1 label, rank of its layer-1 root}, the list of layer-1 roots
// (rank_ints), one record per rank of layers 2 .. NL-1 (layer_ints(NL) each)
// and the root scan's scratch.
// Every layer at least halves the regions of an image with two or more
// (each region joins the neighbour across its lowest pass), so an arena of
// nimg images has at most arena / 2 + nimg layer-1 roots.
size_t rank_ints(size_t arena, int nimg) { return arena / 2 + (size_t)nimg + 1; }
// Ints per rank record of layers 2 .. NL-1 (whole 16-byte groups).
size_t layer_ints(int NL) { return NL < 3 ? 0 : (size_t)(NL - 2 + 3) / 4 * 4; }
size_t mlab_ints(size_t arena, int NL, int nimg) {
    if (NL < 3) return arena;
    // [region records {layer 1, rank}: 2 arena][root list: H][rank records: layer_ints(NL) H][scan scratch]
    const size_t H = rank_ints(arena, nimg);
    return 2 * arena + H + layer_ints(NL) * H + (size_t)wsk::root_list_tmp_len((int32_t)arena);
}

// `cap`: edge slab entries per waterfall tile (the largest any part needs).
int wf_buffers(ws_ctx *c, size_t arena, int nimg, int32_t ntiles, int32_t nchunks, int32_t cap, int NL, bool tables,
               WfBufs &b) {
    int rc;
    if ((rc = ensure(c, c->wfcnt, 8, "region counts")) != WS_OK) return rc;
    if ((rc = ensure(c, c->tilecnt, (size_t)NL * nchunks * 4, "chunk counts")) != WS_OK) return rc;
    // region-id tables: [chunk offsets | scan scratch | 64 rank words per chunk]
    size_t off_words = (((size_t)nchunks + wsk::scan_tmp_len(nchunks)) * 4 + 15) & ~(size_t)15;
    if ((rc = ensure(c, c->chunks, off_words + (size_t)nchunks * 64 * sizeof(wsk::RankWord), "region-id tables")) !=
        WS_OK)
        return rc;
    char *tb = (char *)c->chunks.p;
    b.ids = wsk::WfIds{(wsk::RankWord *)(tb + off_words), (int32_t *)tb};
    b.scan_tmp = (int32_t *)tb + nchunks;
    b.nreg0 = (int32_t *)c->wfcnt.p;
    b.cnt = (int32_t *)c->tilecnt.p;
    b.key = nullptr;
    b.par = b.cimg = b.rlist = b.mlab = nullptr;
    b.es = wsk::EdgeSlabs{};
    if (!tables) return WS_OK;
    const size_t E = (size_t)ntiles * (size_t)cap;
    if ((rc = ensure(c, c->key, arena * 8, "region keys")) != WS_OK) return rc;
    if ((rc = ensure(c, c->par, arena * 4, "region parents")) != WS_OK) return rc;
    if ((rc = ensure(c, c->cimg, arena * 4, "pixel region ids")) != WS_OK) return rc;
    if ((rc = ensure(c, c->rlist, arena * 4, "region labels")) != WS_OK) return rc;
    if (NL >= 2 && (rc = ensure(c, c->mlab, mlab_ints(arena, NL, nimg) * 4, "layer labels")) != WS_OK) return rc;
    if ((rc = ensure(c, c->edges, E * wsk::EdgeSlabs::kEntryBytes, "edge slabs")) != WS_OK) return rc;
    if ((rc = ensure(c, c->ecnt, (size_t)ntiles * 4, "edge counts")) != WS_OK) return rc;
    b.key = (uint64_t *)c->key.p;
    b.par = (int32_t *)c->par.p;
    b.cimg = (int32_t *)c->cimg.p;
    b.rlist = (int32_t *)c->rlist.p;
    b.mlab = (int32_t *)c->mlab.p;
    b.es.p = (uint64_t *)c->edges.p;
    b.es.w = (uint16_t *)(b.es.p + E);
    b.es.cnt = (int32_t *)c->ecnt.p;
    b.es.cap = cap;
    return WS_OK;
}

template <class Src>
int32_t wf_tiles_of(const std::vector<Part<Src>> &parts) {
    int32_t n = 0;
    for (auto &p : parts) n += p.nwf;
    return n;
}

template <class Src>
int32_t slab_cap_of(const std::vector<Part<Src>> &parts) {
    int32_t cap = 0;
    for (auto &p : parts) cap = std::max(cap, (int32_t)wsk::wf_slab_cap(p.conn));
    return cap;
}

// NL waterfall layers of every image of every part (layer 0 already in lab):
// region ids over all chunks, the layer-0 pixel pass per part, then per layer
// union + compression and (from layer 2) an edge pass over tile groups growing
// fourfold, and one pass writing every layer. Region counts go to outs[b]
// (batch, device array of device pointers) or one_out (single image). The
// buffers `b` come from wf_buffers.
template <class Src>
int run_waterfall(ws_ctx *c, Launch &lc, const std::vector<Part<Src>> &parts, const Src &src_ch, int32_t nchunks,
                  bool u16, int NL, size_t arena, const WfBufs &b, const wsk::Img *tab_dev, const wsk::Img &one,
                  int nimg, int64_t *const *outs_dev, int64_t *one_out) {
    int32_t bound = (int32_t)arena;
    const int32_t wft = wf_tiles_of(parts);
    if (NL == 1) {
        WS_TRY(wsk::launch_wf_ids(lc, src_ch, nchunks, bound, b.ids, b.scan_tmp, b.nreg0, nullptr, nullptr));
    } else {
        WS_TRY(wsk::launch_wf_ids(lc, src_ch, nchunks, bound, b.ids, b.scan_tmp, b.nreg0, b.key, b.par));
        for (auto &p : parts)
            WS_TRY(wsk::launch_wf_pix(lc, p.wf, full_grid(p.nwf), p.conn, u16, b.ids, b.nreg0, b.cimg, b.rlist, b.key,
                                      b.es.at(p.wf0)));
        WS_TRY(wsk::launch_wf_union(lc, bound, b.nreg0, b.key, b.par));
        if (NL == 2) {
            WS_TRY(wsk::launch_wf_compress(lc, bound, b.nreg0, b.par, b.rlist, b.mlab));
        } else {
            // later layers only concern the roots of layer 1: list them
            const size_t H = rank_ints(arena, nimg), LS = layer_ints(NL);
            int32_t *id1 = b.mlab + 1, *R1 = b.mlab + 2 * arena, *n1 = b.nreg0 + 1;
            int32_t *lay = R1 + H, *scr = lay + LS * H;
            WS_TRY(wsk::launch_root_list(lc, bound, b.nreg0, b.par, R1, id1, 2, (int32_t)H, scr, n1));
            WS_TRY(wsk::launch_wf_compress1(lc, bound, b.nreg0, b.par, b.rlist, b.mlab, id1, 2));
            int32_t gin = 1;
            for (int k = 2; k < NL; ++k) {
                // groups grow fourfold per layer: regions spanning several tiles
                // then share one group (fewer key atomics) while a group's
                // distinct edges still fit its LDS hash
                int32_t f = gin >= wft ? 1 : 4;
                WS_TRY(wsk::launch_wf_level(lc, wft, gin, f, b.par, b.key, b.es));
                gin *= f;
                WS_TRY(wsk::launch_wf_union_l(lc, bound, n1, (int32_t)H, R1, b.key, b.par));
                WS_TRY(wsk::launch_wf_compress_l(lc, bound, n1, (int32_t)H, R1, b.par, b.rlist, lay + (k - 2),
                                                 (int32_t)LS));
            }
        }
    }
    WS_TRY(wsk::launch_wf_out(lc, src_ch, nchunks, NL, b.cimg, b.nreg0, b.ids.coff, b.mlab, (int64_t)arena,
                              (int64_t)rank_ints(arena, nimg), b.cnt));
    if (outs_dev || one_out)
        WS_TRY(wsk::launch_img_counts(lc, tab_dev, one, nimg, NL, nchunks, b.cnt, outs_dev, one_out));
    return WS_OK;
}

// Pre-allocates the scratch of calls covering up to n pixels (any mix of 2D
// and 3D images, NL <= 8, batches of up to kReserveItems images), so that later
// calls allocate nothing.
constexpr int64_t kReserveItems = 1024;
int reserve(ws_ctx *c, int64_t n) {
    // a batch starts every image on a 64-pixel boundary: room for that padding
    size_t N = (size_t)n + 64 * (size_t)kReserveItems;
    size_t tiles = N / 256 + 1024;         // partial tiles of many small images
    size_t wft = N / 1024 + N / 4096 + 1024;  // waterfall tiles of such a mix
    constexpr int kLayers = 8;             // layer tables for NL <= 8
    int rc;
    Buf *four[] = {&c->D, &c->par, &c->cimg, &c->rlist};
    for (Buf *b : four)
        if ((rc = ensure(c, *b, N * 4, "reserved scratch")) != WS_OK) return rc;
    if ((rc = ensure(c, c->key, N * 8, "reserved keys")) != WS_OK) return rc;
    if ((rc = ensure(c, c->mlab, mlab_ints(N, kLayers, kReserveItems) * 4, "reserved layer labels")) != WS_OK)
        return rc;
    if ((rc = ensure(c, c->edges, wft * (size_t)wsk::wf_slab_cap(8) * wsk::EdgeSlabs::kEntryBytes, "reserved edge slabs")) != WS_OK) return rc;
    if ((rc = ensure(c, c->ecnt, wft * 4, "reserved edge counts")) != WS_OK) return rc;
    if ((rc = ensure(c, c->stamp, tiles * 16, "reserved stamps")) != WS_OK) return rc;
    if ((rc = ensure(c, c->rec, tiles * (size_t)wsk::record_ints(3) * 4, "reserved records")) != WS_OK) return rc;
    if ((rc = ensure(c, c->tilecnt, tiles * 16 * 4, "reserved tile counts")) != WS_OK) return rc;
    int32_t nch = (int32_t)std::min<int64_t>((int64_t)N / 4096 + 2 * kReserveItems, 0x7fffffff / 2);
    size_t tbl = (((size_t)nch + wsk::scan_tmp_len(nch)) * 4 + 15) / 16 * 16 + (size_t)nch * 64 * sizeof(wsk::RankWord);
    if ((rc = ensure(c, c->chunks, tbl, "reserved region-id tables")) != WS_OK) return rc;
    // batch tables (device and pinned staging), laid out as ws_batch does
    size_t bt = sizeof(wsk::Img) * (size_t)kReserveItems + 4 * (tiles + wft + (size_t)nch) +
                sizeof(int64_t *) * (size_t)kReserveItems + 4 * 256;
    if ((rc = ensure(c, c->tab, bt, "reserved batch tables")) != WS_OK) return rc;
    if ((rc = ensure_stage(c, bt)) != WS_OK) return rc;
    if ((rc = ensure(c, c->wfcnt, 16 * 4, "reserved counts")) != WS_OK) return rc;
    if ((rc = ensure(c, c->cnt, kCounterSlots * 4, "counters")) != WS_OK) return rc;
    return WS_OK;
}

// The one part of a single-image call.
// `src` must have been made by single_img with the same shape.
std::vector<Part<wsk::OneImg>> one_part(const wsk::OneImg &src, int conn, int shape) {
    Part<wsk::OneImg> p;
    p.ws = p.wf = src;
    p.shape = shape;
    p.ndim = src.im.g.nz > 1 ? 3 : 2;
    p.nws = src.im.g.ntx * src.im.g.nty * src.im.g.ntz;
    p.nwf = wsk::wf_tiles(src.im.g, p.ndim);
    p.conn = conn;
    return {p};
}

wsk::Img single_img(int64_t nx, int64_t ny, int64_t nz, const void *grad, int32_t *lab, int shape) {
    wsk::Img im{};
    im.g = make_geom(nx, ny, nz, shape);
    im.pix0 = 0;
    im.tile0[0] = im.tile0[1] = im.tile0[2] = im.tile0[3] = 0;
    im.slot0 = 0;
    im.grey = grad;
    im.lab = lab;
    return im;
}

}  // namespace

extern "C" {

int ws_create(ws_ctx **out, int device, size_t scratch_budget_bytes) {
    if (!out) return fail(nullptr, WS_EINVAL, "ws_create: ctx is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) return fail(nullptr, WS_EDEVICE, std::string("hipGetDeviceCount: ") + hipGetErrorString(e));
    if (device < 0 || device >= n) return fail(nullptr, WS_EINVAL, "ws_create: bad device index");
    ws_ctx *c = new ws_ctx();
    c->device = device;
    c->budget = scratch_budget_bytes;
    if ((e = hipSetDevice(device)) != hipSuccess) {
        delete c;
        return fail(nullptr, WS_EDEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    }
    if ((e = hipHostMalloc((void **)&c->host_cnt, (kCounterSlots + 1) * 4, hipHostMallocDefault)) != hipSuccess) {
        delete c;
        return fail(nullptr, WS_EDEVICE, std::string("hipHostMalloc: ") + hipGetErrorString(e));
    }
    {
        // the address of the fixed scratch of ws_watershed_noalloc on this
        // device; a failure only disables that entry point (it reports why)
        std::string why;
        if (noalloc_setup(device, why) != WS_OK) {
            (void)hipGetLastError();
            std::lock_guard<std::mutex> lock(g_noalloc_mu);
            g_noalloc_why = why;
        }
    }
    *out = c;
    return WS_OK;
}

void ws_destroy(ws_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    Buf *bufs[] = {&c->ragoff, &c->ragbuf, &c->rimg,  &c->D,     &c->stamp, &c->cnt,  &c->rec, &c->key, &c->par,    &c->cimg,    &c->rlist, &c->mlab,
                   &c->edges, &c->ecnt,  &c->wfcnt, &c->g0, &c->g1,  &c->mag,    &c->gmax,    &c->chunks,
                   &c->tilecnt, &c->tab};
    for (Buf *b : bufs)
        if (b->p) (void)hipFree(b->p);
    for (auto &gr : c->graphs) {
        (void)hipGraphExecDestroy(gr.exec);
        if (gr.owned) (void)hipFree(gr.owned);
    }
    if (c->cap) (void)hipStreamDestroy(c->cap);
    for (auto &r : c->sink.recs) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
    for (auto e : c->sink.pool) (void)hipEventDestroy(e);
    if (c->host_cnt) (void)hipHostFree(c->host_cnt);
    if (c->sweep_ev) (void)hipEventDestroy(c->sweep_ev);
    if (c->stage) (void)hipHostFree(c->stage);
    if (c->stage_ev) (void)hipEventDestroy(c->stage_ev);
    delete c;
}

const char *ws_last_error(const ws_ctx *c) { return c ? c->err.c_str() : g_noctx_error.c_str(); }

int ws_sync(ws_ctx *c, void *stream) {
    if (!c) return fail(nullptr, WS_EINVAL, "ws_sync: ctx is NULL");
    int rc = set_device(c);
    if (rc) return rc;
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
    return WS_OK;
}

size_t ws_footprint_bytes(int64_t nx, int64_t ny, int64_t nz, int conn, int dtype, int NL) {
    std::string why;
    if (!valid_dims(nx, ny, nz, why) || !valid_conn(nz, conn) || (dtype != WS_U8 && dtype != WS_U16) || NL < 1)
        return 0;
    int ndim = nz > 1 ? 3 : 2;
    size_t N = (size_t)(nx * ny * nz);
    size_t b = dtype == WS_U8 ? 1 : 2;
    size_t job = N * (b + 4 * (size_t)NL);
    // at the default tile shapes (2 and 3), which have the most border records per pixel
    const Geom gd = make_geom(nx, ny, nz, ndim);
    size_t ws = N * 4 /* D */ + (size_t)gd.ntx * gd.nty * gd.ntz * (16 + 4 * (size_t)wsk::record_ints(ndim));
    size_t wf = 0;
    if (NL >= 2) {
        size_t tiles = (size_t)wsk::wf_tiles(make_geom(nx, ny, nz, ndim), ndim);
        wf = N * (8 /* keys */ + 4 /* parents */ + 4 /* ids */ + 4 /* labels */) + mlab_ints(N, NL, 1) * 4 /* layers */ +
             tiles * (wsk::EdgeSlabs::kEntryBytes * (size_t)wsk::wf_slab_cap(conn) + 4 + 4 * (size_t)NL) +
             ((size_t)wsk::wf_chunks((int32_t)N) + 2) * (64 * 16 + 8) /* region-id rank tables */;
    }
    return job + ws + wf + (1 <<20);
}

int ws_set_option(ws_ctx *c, const char *name, int64_t v) {
    if (!c || !name) return fail(c, WS_EINVAL, "ws_set_option: NULL argument");
    std::string k(name);
    if (k == "step3" && (v == 0 || v == 1)) c->step3 = (int)v;
    else if (k == "schedule" && (v == 0 || v == 1)) c->schedule = (int)v;
    else if (k == "step4" && (v == 0 || v == 1)) c->step4 = (int)v;
    else if (k == "rr" && v >= 1 && v <= 64) c->rr = (int)v;
    else if (k == "sweep_batch" && v >= 1 && v <= kMaxSweepBatch) c->sweep_batch = (int)v;
    else if (k == "max_sweeps" && v >= 1) c->max_sweeps = v;
    else if (k == "timing" && (v == 0 || v == 1)) c->timing = v != 0;
    else if (k == "graph" && (v == 0 || v == 1)) c->graph = v != 0;
    else if (k == "tile2d" && (v == 2 || v == 12 || v == 22 || v == 32)) c->tile2 = (int)v;
    else if (k == "tile3d" && (v == 3 || v == 13 || v == 23 || v == 33)) c->tile3 = (int)v;
    else if (k == "reserve_pixels" && v >= 0 && v < (1LL << 31)) {
        int rc = set_device(c);
        if (rc) return rc;
        return reserve(c, v);
    }
    else return fail(c, WS_EINVAL, "ws_set_option: unknown option or value out of range: " + k);
    return WS_OK;
}

int ws_get_stats(const ws_ctx *c, int64_t *out, int n) {
    if (!c || !out || n < 0) return WS_EINVAL;
    int m = std::min(n, 7);
    for (int i = 0; i < m; ++i) out[i] = c->stats[i];
    return m;
}

int ws_gradient(ws_ctx *c, const float *img, int64_t nx, int64_t ny, int64_t nz, float sigma, int dtype, void *grad,
                float *mag_or_null, void *stream) {
    std::string why;
    if (!c) return fail(c, WS_EINVAL, "ws_gradient: ctx is NULL");
    if (!img || !grad) return fail(c, WS_EINVAL, "ws_gradient: NULL buffer");
    if (!valid_dims(nx, ny, nz, why)) return fail(c, WS_EINVAL, "ws_gradient: " + why);
    if (dtype != WS_U8 && dtype != WS_U16) return fail(c, WS_EINVAL, "ws_gradient: dtype must be WS_U8 or WS_U16");
    if (!(sigma == sigma)) return fail(c, WS_EINVAL, "ws_gradient: sigma is NaN");
    int r = sigma > 0.f ? (int)(4.0 * (double)sigma + 0.5) : 0;
    if (r > 64) return fail(c, WS_EUNSUPPORTED, "ws_gradient: blur radius above 64 (sigma > 15.9)");
    int rc = set_device(c);
    if (rc) return rc;
    int ndim = nz > 1 ? 3 : 2;
    Geom g = make_geom(nx, ny, nz, ndim);  // the default shape of this dimensionality (tiling unused)
    size_t N = (size_t)g.n;
    uint32_t sbits;
    memcpy(&sbits, &sigma, 4);
    std::string sig = sig_of("gr", {(uint64_t)(uintptr_t)img, (uint64_t)nx, (uint64_t)ny, (uint64_t)nz, sbits,
                                    (uint64_t)dtype, (uint64_t)(uintptr_t)grad, (uint64_t)(uintptr_t)mag_or_null});
    return run_graphed(c, stream, sig, [&](Launch &lc) -> int {
        int rc;
        const int32_t nparts = wsk::grad_parts(g, ndim, r);
        if ((rc = ensure(c, c->gmax, ((size_t)nparts + 257) * 4, "partial maxima")) != WS_OK) return rc;
        float *part = (float *)c->gmax.p, *part_tmp = part + nparts, *gmax = part_tmp + 256;
        float *mag = mag_or_null;
        if (!mag) {
            if ((rc = ensure(c, c->mag, N * 4, "magnitude buffer")) != WS_OK) return rc;
            mag = (float *)c->mag.p;
        }
        wsk::BlurTaps taps;
        taps.r = r;
        {
            double w[129], sum = 0.0;
            for (int k = -r; k <= r; ++k) {
                w[k + r] = r > 0 ? exp(-0.5 * (double)k * (double)k / ((double)sigma * (double)sigma)) : 1.0;
                sum += w[k + r];
            }
            for (int k = 0; k <= 2 * r; ++k) taps.w[k] = (float)(w[k] / sum);
        }
        if (ndim == 2 && r <= wsk::FUSED_MAX_R) {
            WS_TRY(wsk::launch_grad_fused2d(lc, g, img, mag, part, taps));
        } else {
            const float *src = img;
            if (r > 0) {
                if ((rc = ensure(c, c->g0, N * 4, "blur buffer")) != WS_OK) return rc;
                if ((rc = ensure(c, c->g1, N * 4, "blur buffer")) != WS_OK) return rc;
                float *bufs[2] = {(float *)c->g0.p, (float *)c->g1.p};
                for (int ax = 0; ax < ndim; ++ax) {
                    float *dst = bufs[ax & 1];
                    WS_TRY(wsk::launch_grad_blur(lc, g, src, dst, ax, taps));
                    src = dst;
                }
            }
            WS_TRY(wsk::launch_grad_sobel(lc, g, ndim, src, mag, part));
        }
        WS_TRY(wsk::launch_grad_max(lc, nparts, part, part_tmp, gmax));
        WS_TRY(wsk::launch_grad_quant(lc, g.n, dtype == WS_U16, mag, grad, gmax));
        return WS_OK;
    });
}

static int ws_validate_ws(ws_ctx *c, const void *grad, int dtype, int64_t nx, int64_t ny, int64_t nz, int conn,
                          const void *out, const char *who) {
    std::string why;
    if (!c) return fail(c, WS_EINVAL, std::string(who) + ": ctx is NULL");
    if (!grad || !out) return fail(c, WS_EINVAL, std::string(who) + ": NULL buffer");
    if (!valid_dims(nx, ny, nz, why)) return fail(c, WS_EINVAL, std::string(who) + ": " + why);
    if (dtype != WS_U8 && dtype != WS_U16) return fail(c, WS_EINVAL, std::string(who) + ": dtype must be WS_U8 or WS_U16");
    if (!valid_conn(nz, conn))
        return fail(c, WS_EINVAL, std::string(who) + ": conn must be 4 or 8 for 2D (nz == 1) and 6 or 26 for 3D");
    return WS_OK;
}

int ws_watershed(ws_ctx *c, const void *grad, int dtype, int64_t nx, int64_t ny, int64_t nz, int conn, int32_t *labels,
                 void *stream) {
    int rc = ws_validate_ws(c, grad, dtype, nx, ny, nz, conn, labels, "ws_watershed");
    if (rc) return rc;
    if ((rc = set_device(c))) return rc;
    int ndim = nz > 1 ? 3 : 2;
    Launch lc = make_launch(c, stream);
    const int shape = shape_of(c, ndim);
    wsk::OneImg src{single_img(nx, ny, nz, grad, labels, shape)};
    const wsk::Geom &g = src.im.g;
    if (c->schedule == 1) return run_watershed_px(c, lc, g, grad, conn, dtype == WS_U16, labels, nullptr);
    if (c->step4 == 1) return fail(c, WS_EUNSUPPORTED, "ws_watershed: step4 = 1 (PRW) needs schedule = 1");
    auto parts = one_part(src, conn, shape);
    auto enqueue = [&](Launch &l) -> int {
        WsScratch ws;
        int rc2 = prepare_watershed(c, parts, (size_t)g.n, true, ws);
        if (rc2 != WS_OK) return rc2;
        return run_watershed(c, l, parts, dtype == WS_U16, ws);
    };
    // PRUF reads a counter back after every synchronisation: never captured
    if (c->step3 != 0) return enqueue(lc);
    std::string sig = sig_of("ws", {(uint64_t)(uintptr_t)grad, (uint64_t)dtype, (uint64_t)nx, (uint64_t)ny,
                                    (uint64_t)nz, (uint64_t)conn, (uint64_t)(uintptr_t)labels, (uint64_t)shape});
    return run_graphed(
        c, stream, sig,
        [&](Launch &l) -> int {
            int rc2 = enqueue(l);
            if (rc2 == WS_OK && !c->capturing) note_sweeps(c, sig);
            return rc2;
        },
        [&](void **, size_t *) { return prep_sweeps(c, sig); },
        [&](const ws_ctx::Graph &gr) { return check_sweeps(c, gr, stream); });
}

int ws_watershed_noalloc(ws_ctx *c, const void *grad, int dtype, int64_t nx, int64_t ny, int64_t nz, int conn,
                         int32_t *labels, void *stream) {
    int rc = ws_validate_ws(c, grad, dtype, nx, ny, nz, conn, labels, "ws_watershed_noalloc");
    if (rc) return rc;
    if (c->schedule != 0)
        return fail(c, WS_EUNSUPPORTED, "ws_watershed_noalloc: only the tile schedule (schedule = 0)");
    if (c->step4 != 0) return fail(c, WS_EUNSUPPORTED, "ws_watershed_noalloc: step4 = 1 (PRW) needs schedule = 1");
    const int shape = shape_of(c, nz > 1 ? 3 : 2);
    wsk::OneImg src{single_img(nx, ny, nz, grad, labels, shape)};
    const wsk::Geom &g = src.im.g;
    auto parts = one_part(src, conn, shape);
    // [distances | stamps | counters | border records], 256-byte aligned parts
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t oD = 0, oS = oD + up((size_t)g.n * 4), oC = oS + up((size_t)ws_tiles_of(parts) * 16),
                 oR = oC + up((size_t)kCounterSlots * 4), need = oR + up(rec_ints(parts) * 4);
    if (need > kNoAllocBytes)
        return fail(c, WS_EINVAL, "ws_watershed_noalloc: this image needs " + std::to_string(need) +
                                      " bytes of scratch, the fixed area holds " + std::to_string(kNoAllocBytes));
    if ((rc = set_device(c))) return rc;
    char *base = (char *)noalloc_scratch_of(c->device);
    if (!base) {
        std::lock_guard<std::mutex> lock(g_noalloc_mu);
        return fail(c, WS_EDEVICE, "ws_watershed_noalloc: no fixed scratch on this device: " + g_noalloc_why);
    }
    WsScratch ws;
    ws.D = (int32_t *)(base + oD);
    ws.stamp = (int32_t *)(base + oS);
    ws.cnt = (int32_t *)(base + oC);
    ws.rec = (int32_t *)(base + oR);
    Launch lc = make_launch(c, stream);
    return run_watershed(c, lc, parts, dtype == WS_U16, ws);
}

int ws_watershed_stages(ws_ctx *c, const void *grad, int dtype, int64_t nx, int64_t ny, int64_t nz, int conn,
                        int32_t *bal, int32_t *arrow, void *stream) {
    int rc = ws_validate_ws(c, grad, dtype, nx, ny, nz, conn, bal, "ws_watershed_stages");
    if (rc) return rc;
    if (!arrow) return fail(c, WS_EINVAL, "ws_watershed_stages: NULL buffer");
    if ((rc = set_device(c))) return rc;
    Launch lc = make_launch(c, stream);
    bool u16 = dtype == WS_U16;
    const int shape = shape_of(c, nz > 1 ? 3 : 2);
    wsk::OneImg src{single_img(nx, ny, nz, grad, nullptr, shape)};
    const wsk::Geom &g = src.im.g;
    if (c->schedule == 1) return run_watershed_px(c, lc, g, grad, conn, u16, arrow, bal);
    auto parts = one_part(src, conn, shape);
    WsScratch ws;
    if ((rc = prepare_watershed(c, parts, (size_t)g.n, false, ws)) != WS_OK) return rc;
    if ((rc = run_distances(c, lc, parts, u16, ws)) != WS_OK) return rc;
    WS_TRY(wsk::launch_ws_stages(lc, g, conn, u16, grad, ws.D, bal, arrow));
    return WS_OK;
}

int ws_waterfall(ws_ctx *c, const int32_t *labels, const void *grad, int dtype, int64_t nx, int64_t ny, int64_t nz,
                 int conn, int NL, int32_t *out, int64_t *nregions, void *stream) {
    int rc = ws_validate_ws(c, grad, dtype, nx, ny, nz, conn, out, "ws_waterfall");
    if (rc) return rc;
    if (!labels) return fail(c, WS_EINVAL, "ws_waterfall: NULL labels");
    if (NL < 1) return fail(c, WS_EINVAL, "ws_waterfall: NL must be >= 1");
    if ((rc = set_device(c))) return rc;
    int ndim = nz > 1 ? 3 : 2;
    const int shape = shape_of(c, ndim);
    wsk::OneImg src{single_img(nx, ny, nz, grad, out, shape)};
    const wsk::Geom &g = src.im.g;
    std::string sig = sig_of("wf", {(uint64_t)(uintptr_t)labels, (uint64_t)(uintptr_t)grad, (uint64_t)dtype,
                                    (uint64_t)nx, (uint64_t)ny, (uint64_t)nz, (uint64_t)conn, (uint64_t)NL,
                                    (uint64_t)(uintptr_t)out, (uint64_t)(uintptr_t)nregions});
    (void)ndim;
    return run_graphed(c, stream, sig, [&](Launch &lc) -> int {
        auto parts = one_part(src, conn, shape);
        const int32_t nchunks = wsk::wf_chunks(g.n);
        WfBufs b;
        int rc2 = wf_buffers(c, (size_t)g.n, 1, wf_tiles_of(parts), nchunks, slab_cap_of(parts), NL, NL >= 2, b);
        if (rc2 != WS_OK) return rc2;
        if (labels != out) {
            hipError_t e = hipMemcpyAsync(out, labels, (size_t)g.n * 4, hipMemcpyDeviceToDevice, lc.stream);
            if (e != hipSuccess) return hip_fail(c, e, "hipMemcpyAsync");
        }
        return run_waterfall(c, lc, parts, src, nchunks, dtype == WS_U16, NL, (size_t)g.n, b, nullptr, src.im, 1,
                             nullptr, nregions);
    });
}

int ws_waterfall_recon(ws_ctx *c, const int32_t *labels, const void *grad, int dtype, int64_t nx, int64_t ny,
                       int64_t nz, int conn, int NL, int32_t *out, int64_t *nregions, void *stream) {
    int rc = ws_validate_ws(c, grad, dtype, nx, ny, nz, conn, out, "ws_waterfall_recon");
    if (rc) return rc;
    if (!labels) return fail(c, WS_EINVAL, "ws_waterfall_recon: NULL labels");
    if (NL < 1) return fail(c, WS_EINVAL, "ws_waterfall_recon: NL must be >= 1");
    if ((rc = set_device(c))) return rc;
    const int ndim = nz > 1 ? 3 : 2;
    Launch lc = make_launch(c, stream);
    const int shape = shape_of(c, ndim);
    const Geom g = make_geom(nx, ny, nz, shape);
    const size_t N = (size_t)g.n;
    const int32_t nchunks = wsk::wf_chunks(g.n), bound = g.n;
    const wsk::TileGrid tgw = full_grid(wsk::wf_tiles(g, ndim));
    WfBufs b;
    if ((rc = wf_buffers(c, N, 1, tgw.ntiles, nchunks, wsk::wf_slab_cap(conn), 1, NL >= 2, b)) != WS_OK) return rc;
    if ((rc = ensure(c, c->rimg, N * 2, "raised image")) != WS_OK) return rc;
    WsScratch ws;
    {
        wsk::OneImg probe{single_img(nx, ny, nz, grad, out, shape)};
        if ((rc = prepare_watershed(c, one_part(probe, conn, shape), N, true, ws)) != WS_OK) return rc;
    }
    uint16_t *I = (uint16_t *)c->rimg.p;
    if (labels != out) {
        hipError_t e = hipMemcpyAsync(out, labels, N * 4, hipMemcpyDeviceToDevice, lc.stream);
        if (e != hipSuccess) return hip_fail(c, e, "hipMemcpyAsync");
    }
    WS_TRY(wsk::launch_grey_u16(lc, grad, dtype == WS_U16, I, g.n));
    for (int k = 0; k < NL; ++k) {
        wsk::OneImg src{single_img(nx, ny, nz, I, out + (size_t)k * N, shape)};
        // region ids and the layer's region count
        WS_TRY(wsk::launch_wf_ids(lc, src, nchunks, bound, b.ids, b.scan_tmp, b.nreg0, k + 1 < NL ? b.key : nullptr,
                                  b.par));
        if (nregions) {
            WS_TRY(wsk::launch_wf_out(lc, src, nchunks, 1, nullptr, b.nreg0, b.ids.coff, nullptr, 0, 0, b.cnt));
            WS_TRY(wsk::launch_img_counts(lc, nullptr, src.im, 1, 1, nchunks, b.cnt, nullptr, nregions + k));
        }
        if (k + 1 == NL) break;
        // Step V (lowest boundary pass of every region, the keys' heights) on
        // the current image, Step VI (raise), then the watershed again
        WS_TRY(wsk::launch_wf_pix(lc, src, tgw, conn, true, b.ids, b.nreg0, b.cimg, b.rlist, b.key, b.es));
        WS_TRY(wsk::launch_recon_raise(lc, I, b.cimg, b.key, b.nreg0, g.n));
        wsk::OneImg next{single_img(nx, ny, nz, I, out + (size_t)(k + 1) * N, shape)};
        if ((rc = run_watershed(c, lc, one_part(next, conn, shape), true, ws)) != WS_OK) return rc;
    }
    return WS_OK;
}

int ws_rag(ws_ctx *c, const int32_t *labels, const void *grad, int dtype, int64_t nx, int64_t ny, int64_t nz, int conn,
           int64_t capacity, int32_t *edge_a, int32_t *edge_b, int32_t *edge_h, int64_t *n_edges, void *stream) {
    int rc = ws_validate_ws(c, grad, dtype, nx, ny, nz, conn, labels, "ws_rag");
    if (rc) return rc;
    if (capacity < 0) return fail(c, WS_EINVAL, "ws_rag: capacity must be >= 0");
    if (capacity > 0 && (!edge_a || !edge_b || !edge_h)) return fail(c, WS_EINVAL, "ws_rag: NULL edge buffer");
    if ((rc = set_device(c))) return rc;
    const int ndim = nz > 1 ? 3 : 2;
    Launch lc = make_launch(c, stream);
    const Geom g = make_geom(nx, ny, nz, shape_of(c, ndim));
    const size_t N = (size_t)g.n;
    const int32_t nchunks = wsk::wf_chunks(g.n), bound = g.n;
    const wsk::TileGrid tg = full_grid(wsk::wf_tiles(g, ndim));
    WfBufs b;
    if ((rc = wf_buffers(c, N, 1, tg.ntiles, nchunks, wsk::wf_slab_cap(conn), 1, true, b)) != WS_OK) return rc;
    // the labels are read, never written (the pixel pass only reads its layer 0)
    wsk::OneImg src{single_img(nx, ny, nz, grad, const_cast<int32_t *>(labels), shape_of(c, ndim))};
    WS_TRY(wsk::launch_wf_ids(lc, src, nchunks, bound, b.ids, b.scan_tmp, b.nreg0, b.key, b.par));
    WS_TRY(wsk::launch_wf_pix(lc, src, tg, conn, dtype == WS_U16, b.ids, b.nreg0, b.cimg, b.rlist, b.key, b.es));
    // offsets of the tiles' edges in one list, and their total (read back once)
    const int32_t nt = tg.ntiles;
    if ((rc = ensure(c, c->ragoff, ((size_t)nt + 1 + wsk::scan_tmp_len(nt)) * 4, "edge offsets")) != WS_OK) return rc;
    int32_t *eoff = (int32_t *)c->ragoff.p, *etot = eoff + nt, *etmp = etot + 1;
    hipError_t e = hipMemcpyAsync(eoff, b.es.cnt, (size_t)nt * 4, hipMemcpyDeviceToDevice, lc.stream);
    if (e != hipSuccess) return hip_fail(c, e, "hipMemcpyAsync");
    WS_TRY(wsk::launch_scan(lc, nt, eoff, etmp, etot));
    if ((e = hipMemcpyAsync(c->host_cnt, etot, 4, hipMemcpyDeviceToHost, lc.stream)) != hipSuccess)
        return hip_fail(c, e, "hipMemcpyAsync");
    if ((e = hipStreamSynchronize(lc.stream)) != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
    const int32_t total = c->host_cnt[0];
    const size_t tmp_bytes = wsk::rag_sort_tmp_bytes(total > 0 ? total : 1);
    const size_t M = (size_t)(total > 0 ? total : 1);
    // [keys | keys2 | ukeys | h | h2 | uh | count | sort scratch]
    size_t o_k2 = M * 8, o_uk = 2 * M * 8, o_h = 3 * M * 8, o_h2 = o_h + M * 4, o_uh = o_h2 + M * 4;
    size_t o_cnt = (o_uh + M * 4 + 255) & ~(size_t)255, o_tmp = o_cnt + 256;
    if ((rc = ensure(c, c->ragbuf, o_tmp + tmp_bytes, "adjacency sort buffers")) != WS_OK) return rc;
    char *rb = (char *)c->ragbuf.p;
    auto *keys = (unsigned long long *)rb, *keys2 = (unsigned long long *)(rb + o_k2),
         *ukeys = (unsigned long long *)(rb + o_uk);
    auto *h = (int32_t *)(rb + o_h), *h2 = (int32_t *)(rb + o_h2), *uh = (int32_t *)(rb + o_uh);
    auto *ucount = (unsigned int *)(rb + o_cnt);
    WS_TRY(wsk::launch_fill_i32(lc, (int32_t *)ucount, 1, 0));
    if (total > 0) {
        WS_TRY(wsk::launch_rag_gather(lc, nt, b.es, eoff, keys, h));
        WS_TRY(wsk::rag_sort_reduce(lc, total, keys, h, keys2, h2, ukeys, uh, ucount, rb + o_tmp, tmp_bytes));
    }
    WS_TRY(wsk::launch_rag_final(lc, ukeys, uh, ucount, b.rlist, capacity, edge_a, edge_b, edge_h, n_edges));
    return WS_OK;
}

int ws_batch(ws_ctx *c, const ws_item *items, int n_items, int dtype, int NL, void *stream) {
    if (!c) return fail(c, WS_EINVAL, "ws_batch: ctx is NULL");
    if (!items || n_items < 1) return fail(c, WS_EINVAL, "ws_batch: no items");
    if (dtype != WS_U8 && dtype != WS_U16) return fail(c, WS_EINVAL, "ws_batch: dtype must be WS_U8 or WS_U16");
    if (NL < 1) return fail(c, WS_EINVAL, "ws_batch: NL must be >= 1");
    // images are grouped by connectivity: one part per connectivity present,
    // each a contiguous range of the call's watershed and waterfall tiles
    static const int kConns[4] = {4, 8, 6, 26};
    int64_t arena = 0, tws[4] = {0, 0, 0, 0}, twf[4] = {0, 0, 0, 0}, tch = 0;
    std::string why;
    for (int i = 0; i < n_items; ++i) {
        const ws_item &it = items[i];
        const std::string who = "ws_batch: item " + std::to_string(i);
        if (!it.grad || !it.out) return fail(c, WS_EINVAL, who + " has a NULL buffer");
        if (!valid_dims(it.nx, it.ny, it.nz, why)) return fail(c, WS_EINVAL, who + ": " + why);
        if (!valid_conn(it.nz, it.conn))
            return fail(c, WS_EINVAL, who + ": conn must be 4 or 8 for 2D (nz == 1) and 6 or 26 for 3D");
        arena += (it.nx * it.ny * it.nz + 63) / 64 * 64;  // image offsets stay 64-pixel aligned
        const int ndim = it.nz > 1 ? 3 : 2;
        const int gi = (int)(std::find(kConns, kConns + 4, it.conn) - kConns);
        wsk::Geom g = make_geom(it.nx, it.ny, it.nz, shape_of(c, ndim));
        tws[gi] += (int64_t)g.ntx * g.nty * g.ntz;
        twf[gi] += wsk::wf_tiles(g, ndim);
        tch += wsk::wf_chunks(g.n);
        if (arena >= (1LL << 31)) return fail(c, WS_EINVAL, "ws_batch: total pixels must be < 2^31");
    }
    int64_t ws_all = tws[0] + tws[1] + tws[2] + tws[3], wf_all = twf[0] + twf[1] + twf[2] + twf[3];
    int rc;
    if ((rc = set_device(c))) return rc;
    // tables: [Img table][ws tile map][wf tile map][chunk map][nregions pointers]
    size_t tab_b = sizeof(wsk::Img) * (size_t)n_items;
    size_t off_ws = (tab_b + 255) & ~(size_t)255;
    size_t off_wf = (off_ws + 4 * (size_t)ws_all + 255) & ~(size_t)255;
    size_t off_ch = (off_wf + 4 * (size_t)wf_all + 255) & ~(size_t)255;
    size_t off_outs = (off_ch + 4 * (size_t)tch + 255) & ~(size_t)255;
    size_t total = off_outs + sizeof(int64_t *) * (size_t)n_items;
    // parts in connectivity order; tile ranges relative to the part's first tile
    struct PartSpec {
        int conn, ndim, gi;
        int32_t ws0, wf0, nws, nwf;
    };
    std::vector<PartSpec> specs;
    int32_t ws0 = 0, wf0 = 0;
    for (int gi = 0; gi < 4; ++gi) {
        if (tws[gi] == 0) continue;
        specs.push_back({kConns[gi], gi < 2 ? 2 : 3, gi, ws0, wf0, (int32_t)tws[gi], (int32_t)twf[gi]});
        ws0 += (int32_t)tws[gi];
        wf0 += (int32_t)twf[gi];
    }
    // the tables on the host (no device pointers of the context in them)
    std::vector<char> host(total, 0);
    {
        char *h = host.data();
        wsk::Img *tab = (wsk::Img *)h;
        int32_t *mws = (int32_t *)(h + off_ws), *mwf = (int32_t *)(h + off_wf), *mch = (int32_t *)(h + off_ch);
        int64_t **outs = (int64_t **)(h + off_outs);
        int32_t next_ws[4] = {0, 0, 0, 0}, next_wf[4] = {0, 0, 0, 0};
        int32_t pix = 0, t2 = 0;
        for (int i = 0; i < n_items; ++i) {
            const ws_item &it = items[i];
            const int ndim = it.nz > 1 ? 3 : 2;
            const int gi = (int)(std::find(kConns, kConns + 4, it.conn) - kConns);
            const PartSpec *pp = nullptr;
            for (auto &p : specs)
                if (p.gi == gi) pp = &p;
            wsk::Img im{};
            im.g = make_geom(it.nx, it.ny, it.nz, shape_of(c, ndim));
            im.pix0 = pix;
            im.tile0[wsk::TK_WS] = next_ws[gi];
            im.tile0[wsk::TK_WF] = next_wf[gi];
            im.tile0[wsk::TK_GR] = 0;
            im.tile0[wsk::TK_CH] = t2;
            im.slot0 = 0;
            im.grey = it.grad;
            im.lab = it.out;
            tab[i] = im;
            int32_t nws = im.g.ntx * im.g.nty * im.g.ntz, nwf = wsk::wf_tiles(im.g, ndim),
                    nch = wsk::wf_chunks(im.g.n);
            for (int32_t k = 0; k < nws; ++k) mws[pp->ws0 + next_ws[gi] + k] = i;
            for (int32_t k = 0; k < nwf; ++k) mwf[pp->wf0 + next_wf[gi] + k] = i;
            for (int32_t k = 0; k < nch; ++k) mch[t2 + k] = i;
            outs[i] = it.nregions;
            pix += (im.g.n + 63) / 64 * 64;
            next_ws[gi] += nws;
            next_wf[gi] += nwf;
            t2 += nch;
        }
    }
    bool any_counts = false;
    for (int i = 0; i < n_items; ++i) any_counts = any_counts || items[i].nregions;
    const int32_t nchunks = (int32_t)tch;
    const bool u16 = dtype == WS_U16;
    void *cap_tab = nullptr;  // the tables a graph being captured reads (its own device copy)
    auto enqueue = [&](Launch &lc) -> int {
        int rc2;
        char *d;
        if (c->capturing) {
            d = (char *)cap_tab;
        } else {
            // every buffer of the call before anything is launched
            if ((rc2 = ensure_stage(c, total)) != WS_OK) return rc2;
            if ((rc2 = ensure(c, c->tab, total, "batch tables")) != WS_OK) return rc2;
            d = (char *)c->tab.p;
        }
        const wsk::Img *tab_dev = (const wsk::Img *)d;
        std::vector<Part<wsk::ImgTable>> parts;
        for (auto &sp : specs) {
            Part<wsk::ImgTable> p;
            p.conn = sp.conn;
            p.ndim = sp.ndim;
            p.shape = shape_of(c, sp.ndim);
            p.ws0 = sp.ws0;
            p.wf0 = sp.wf0;
            p.nws = sp.nws;
            p.nwf = sp.nwf;
            p.ws = wsk::ImgTable{tab_dev, (const int32_t *)(d + off_ws) + sp.ws0};
            p.wf = wsk::ImgTable{tab_dev, (const int32_t *)(d + off_wf) + sp.wf0};
            parts.push_back(p);
        }
        WfBufs wb;
        WsScratch ws;
        if ((rc2 = prepare_watershed(c, parts, (size_t)arena, true, ws)) != WS_OK) return rc2;
        if ((rc2 = wf_buffers(c, (size_t)arena, n_items, (int32_t)wf_all, nchunks, slab_cap_of(parts), NL, NL >= 2,
                              wb)) !=
            WS_OK)
            return rc2;
        if (!c->capturing) {
            memcpy(c->stage, host.data(), total);
            hipError_t e = hipMemcpyAsync(c->tab.p, c->stage, total, hipMemcpyHostToDevice, lc.stream);
            if (e != hipSuccess) return hip_fail(c, e, "hipMemcpyAsync");
            if ((e = hipEventRecord(c->stage_ev, lc.stream)) != hipSuccess) return hip_fail(c, e, "hipEventRecord");
            c->stage_pending = true;
        }
        wsk::ImgTable src_ch{tab_dev, (const int32_t *)(d + off_ch)};
        if ((rc2 = run_watershed(c, lc, parts, u16, ws)) != WS_OK) return rc2;
        wsk::Img none{};
        return run_waterfall(c, lc, parts, src_ch, nchunks, u16, NL, (size_t)arena, wb, tab_dev, none, n_items,
                             any_counts ? (int64_t *const *)(d + off_outs) : nullptr, nullptr);
    };
    Launch lc = make_launch(c, stream);
    if (c->step3 != 0) return enqueue(lc);
    // signature: the items as given, the grey type, NL
    std::string sig = sig_of("bt", {(uint64_t)n_items, (uint64_t)dtype, (uint64_t)NL, (uint64_t)c->tile2,
                                    (uint64_t)c->tile3});
    for (int i = 0; i < n_items; ++i) {
        const ws_item &it = items[i];
        const uint64_t f[7] = {(uint64_t)(uintptr_t)it.grad, (uint64_t)it.nx, (uint64_t)it.ny, (uint64_t)it.nz,
                               (uint64_t)it.conn, (uint64_t)(uintptr_t)it.out, (uint64_t)(uintptr_t)it.nregions};
        sig.append((const char *)f, sizeof(f));
    }
    return run_graphed(
        c, stream, sig,
        [&](Launch &l) -> int {
            int rc2 = enqueue(l);
            if (rc2 == WS_OK && !c->capturing) note_sweeps(c, sig);
            return rc2;
        },
        [&](void **owned, size_t *owned_n) -> int {
            int v = prep_sweeps(c, sig);
            if (v != WS_OK) return v;
            if (c->budget && c->held + total > c->budget) return kRerun;
            hipError_t e = hipMalloc(owned, total);
            ++c->stats[5];
            if (e != hipSuccess) {
                (void)hipGetLastError();
                *owned = nullptr;
                return kRerun;
            }
            *owned_n = total;
            c->held += total;
            if ((e = hipMemcpy(*owned, host.data(), total, hipMemcpyHostToDevice)) != hipSuccess)
                return hip_fail(c, e, "hipMemcpy");
            cap_tab = *owned;
            return WS_OK;
        },
        [&](const ws_ctx::Graph &gr) { return check_sweeps(c, gr, stream); });
}

int ws_timing_reset(ws_ctx *c) {
    if (!c) return WS_EINVAL;
    for (auto &r : c->sink.recs) {
        c->sink.pool.push_back(r.a);
        c->sink.pool.push_back(r.b);
    }
    c->sink.recs.clear();
    return WS_OK;
}

int ws_timing_read(ws_ctx *c, char *names, int name_len, double *total_ms, int64_t *launches, int cap) {
    if (!c) return WS_EINVAL;
    std::map<std::string, std::pair<double, int64_t>> agg;
    std::vector<std::string> order;
    for (auto &r : c->sink.recs) {
        hipError_t e = hipEventSynchronize(r.b);
        if (e != hipSuccess) return hip_fail(c, e, "hipEventSynchronize");
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess) return hip_fail(c, e, "hipEventElapsedTime");
        if (!agg.count(r.name)) order.push_back(r.name);
        agg[r.name].first += ms;
        agg[r.name].second += 1;
    }
    int i = 0;
    for (auto &nm : order) {
        if (i < cap) {
            if (names && name_len > 0) {
                strncpy(names + (size_t)i * name_len, nm.c_str(), name_len - 1);
                names[(size_t)i * name_len + name_len - 1] = 0;
            }
            if (total_ms) total_ms[i] = agg[nm].first;
            if (launches) launches[i] = agg[nm].second;
        }
        ++i;
    }
    return i;
}

}  // extern "C"
