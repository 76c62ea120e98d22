// Streaming server: many links' ATVC pools resident in device memory,
// admitted against an HBM budget, their uneven slices batched into one step
// graph replayed per step.
//
// Per step the host turns every link's queued events (chunks of pairs, slice
// ends) into one descriptor table.  The captured graph then runs two branches
// concurrently:
//   ingest: batched lazy preserve of opening slices, then the batched scan of
//           every queued chunk of every link;
//   close:  batched close, super lists, restore (budget rule, join, sort),
//           features + plain estimates of candidates and watch hosts, and
//           the learned correction;
// then writes the used rows of the results straight into mapped pinned host
// memory.  A link whose chunks the graph scans is closed in the following
// step, so the two branches never touch the same pool.
//
// A link whose queued pairs in a step are many next to its pool takes the
// tiled scan instead (stores grouped per 64 KiB tile and applied in LDS, the
// pool streamed once).  The step's tiled links share launches outside the
// graph (their grids depend on the step's pair counts), one grid row per
// link.  A launch's record passes touch no pool and run on a stream of their
// own; its tile pass, which opens the slice (the preserve runs there) and,
// when the slice's end is queued behind its chunks, writes the window's
// weights, runs on the graph's stream ahead of the graph, so such a slice is
// scanned and closed in one step.  When the next step will be tiled scans and
// their closes only, it is planned and its launches queued before the host
// waits for the current graph: its record passes then run beside that graph,
// and the GPU goes from the graph straight to its tile pass.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <thread>
#include <cstdint>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <vector>

#include "at.h"
#include "atpool.hpp"

using atp::ChunkDesc;
using atp::CloseDesc;
using atp::Geometry;
using atp::LinkSlot;
using atp::OpenDesc;
using atp::ServeState;
using atp::StepDesc;

namespace {

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

template <typename T>
int dalloc(T** p, uint64_t count) {
    *p = nullptr;
    hipError_t e = hipMalloc((void**)p, (count ? count : 1) * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return e == hipErrorOutOfMemory ? AT_E_NOMEM : AT_E_DEVICE;
    }
    return AT_OK;
}

enum LinkState { L_WAITING = 0, L_ACTIVE = 1, L_CLOSED = 2 };

struct Event {
    bool end;
    const uint32_t* aip;
    const uint32_t* bip;
    uint64_t n;
    uint32_t kprime;
    double t_arrival;
};

struct Link {
    uint32_t id = 0;
    int state = L_WAITING;
    at_params p{};
    Geometry G{};
    uint64_t bytes = 0;
    int slot = -1;
    // device buffers
    uint8_t* pool = nullptr;
    uint32_t* w = nullptr;
    uint64_t* aat = nullptr;
    uint32_t* sa = nullptr;
    uint32_t* sa_cnt = nullptr;
    uint32_t* cand = nullptr;
    uint64_t* frame_prefix = nullptr;
    uint32_t* watch = nullptr;
    uint32_t n_watch = 0;
    // clock
    uint64_t t = 0;          // slices closed
    bool open = false;
    uint32_t c0 = 0;
    std::deque<Event> q;
    uint64_t consumed = 0;   // events consumed (chunks + ends)
};

struct Result {
    at_serve_result r;
    std::vector<uint32_t> cand;
    std::vector<double> cand_est, cand_learned;
    std::vector<uint8_t> cand_flags;
    std::vector<double> watch_plain, watch_learned;
    std::vector<uint8_t> watch_flags;
};

}  // namespace

// One link's chunks of a step, scanned by the tiled scan.
struct TiledChunk {
    const uint32_t* aip;
    const uint32_t* bip;
    uint64_t n;
};
struct TiledJob {
    Link* L;
    std::vector<TiledChunk> chunks;  // copied: the queue's records may be retired before the launch
    uint64_t n;
    bool opens;     // the scan opens the slice: the tile pass runs its preserve
    bool weights;   // the slice's end is queued behind its chunks: the tile pass counts window kq
    uint32_t kq;
    uint32_t c0;    // block clock of the scanned slice
};

struct CloseRec {
    Link* L;
    uint32_t kq;
    double t_arrival;
    uint64_t slice;
};

struct at_serve {
    at_serve_config cfg{};
    hipStream_t s0 = nullptr, s1 = nullptr;  // s0: scan branch and graph launch; s1: close branch
    hipStream_t s2 = nullptr;                // record passes of the tiled scans
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    std::mutex step_mu;  // held while device state may be in use (steps, admissions, watch lists)
    std::mutex mu;       // guards the host-side queues; never held while the GPU works
    std::vector<Link*> links;             // by id
    std::deque<uint32_t> waiting;         // admission FIFO
    std::vector<int> slot_used;           // slot -> link id or -1
    uint64_t used_bytes = 0;
    uint64_t per_link_bytes = 0;
    Geometry shape{};
    uint64_t n_atv = 0;
    // device
    StepDesc* d_desc = nullptr;
    LinkSlot* d_slots = nullptr;
    ServeState* d_state = nullptr;
    uint32_t* d_hosts = nullptr;
    float* d_feat = nullptr;
    double* d_est = nullptr;
    uint8_t* d_pflags = nullptr;
    float* d_y = nullptr;
    uint8_t* d_act = nullptr;     // per close: block timestamp of every AT position
    uint64_t max_hosts = 0;
    // pinned host: the step descriptor, and two sets of mapped result arrays
    // (the export kernel writes step s's results into set s mod 2, so the
    // native thread reads one step's results while the next one runs)
    StepDesc* h_desc = nullptr;
    struct ResultSet {
        ServeState* state = nullptr;
        uint32_t* hosts = nullptr;
        double* est = nullptr;
        double* estl = nullptr;
        uint8_t* flags = nullptr;
        atp::ServeExport xp{};  // their device addresses
    } rs[2];
    int cur_set = 0;
    // graph
    at_mlp* mlp = nullptr;
    const void* mlp_key = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // native stepping thread
    std::thread worker;
    std::condition_variable cv;
    bool stop = false;
    bool running = false;
    int device = 0;
    int worker_rc = AT_OK;
    // results
    std::deque<Result> results;
    // closes of the last step whose results are not yet published (in set pend_set)
    struct PendingClose {
        uint32_t link, kq;
        double t_arrival;
        uint64_t slice;
    };
    std::vector<PendingClose> pending;
    // a step planned ahead: its tiled scans already queued behind the last
    // step's graph, its closes for the next step's graph
    struct Ahead {
        bool valid = false;
        std::vector<TiledJob> tiled;
        std::vector<CloseDesc> cds;
        std::vector<CloseRec> closes;
        uint64_t pairs = 0;
        int tset = 0;
        uint32_t n_timed = 0, n_jobs = 0;
    } ahead;
    int tset = 0;                  // timing-event set of the next step's tiled launches
    hipEvent_t ev_done = nullptr;  // recorded after a step's graph: its results are complete
    hipEvent_t ev_apply[2] = {};   // per scratch set, recorded after each tile pass: its slots are free
    int pend_set = 0;
    bool pend_mlp = false;
    double pend_step_ms = 0.0;
    uint64_t steps = 0;
    double last_step_ms = 0.0;
    uint64_t pairs_ingested = 0;
    // tiled scans: stream, scratch, timing
    bool tiled_ok = false;
    uint64_t pool_bytes = 0;
    // two scratch sets, used by alternate steps, so that a step's record passes
    // can run while the previous step's tile pass still reads its set
    atp::TileBufs tb[2][atp::kTileJobsMax] = {};    // scratch of each job of a batched launch
    uint32_t* stage_a[2][atp::kTileJobsMax] = {};   // gathered chunks of a job's link
    uint32_t* stage_b[2][atp::kTileJobsMax] = {};
    uint64_t stage_cap[2][atp::kTileJobsMax] = {};
    int tbuf = 0;                                   // the set of the next step with tiled scans
    std::vector<hipEvent_t> tev[2];  // start/end event pairs of a step's tiled launches (two steps in flight)
    uint64_t tiled_calls = 0, tiled_jobs = 0, tiled_pairs = 0, planned_ahead = 0;
    double tiled_ms = 0.0;
};

namespace atp {
// MLP operands of a network (capi.hip)
bool mlp_operands(const at_mlp* m, MlpDev* out);
}

namespace {

void free_link_device(Link* L) {
    void* b[] = {L->pool, L->w, L->aat, L->sa, L->sa_cnt, L->cand, L->frame_prefix, L->watch};
    for (void* p : b)
        if (p) (void)hipFree(p);
    L->pool = nullptr;
    L->w = nullptr;
    L->aat = nullptr;
    L->sa = nullptr;
    L->sa_cnt = nullptr;
    L->cand = nullptr;
    L->frame_prefix = nullptr;
    L->watch = nullptr;
}

uint64_t link_bytes(const at_serve* S) {
    const uint64_t ngroups = (uint64_t)(S->shape.umask + 1) * S->shape.r;
    return (S->n_atv << S->shape.log2g) + S->n_atv * 8 + ngroups * 12 + (uint64_t)S->cfg.cand_cap * 4 +
           ((uint64_t)S->shape.umask + 2) * 8 + (uint64_t)S->cfg.watch_cap * 4;
}

// Allocate and initialise a link's pool; publish its slot.  Caller holds mu.
int admit(at_serve* S, Link* L) {
    int slot = -1;
    for (uint32_t i = 0; i < S->slot_used.size(); i++)
        if (S->slot_used[i] < 0) {
            slot = (int)i;
            break;
        }
    if (slot < 0) return AT_E_NOMEM;
    const uint64_t ngroups = (uint64_t)(S->shape.umask + 1) * S->shape.r;
    int rc;
    if ((rc = dalloc(&L->pool, S->n_atv << S->shape.log2g)) || (rc = dalloc(&L->w, S->n_atv)) ||
        (rc = dalloc(&L->aat, ngroups)) || (rc = dalloc(&L->sa, S->n_atv)) || (rc = dalloc(&L->sa_cnt, ngroups)) ||
        (rc = dalloc(&L->cand, S->cfg.cand_cap)) || (rc = dalloc(&L->frame_prefix, S->shape.umask + 2)) ||
        (rc = dalloc(&L->watch, S->cfg.watch_cap))) {
        free_link_device(L);
        return rc;
    }
    hipError_t e = atp::launch_fill_u8(L->pool, S->n_atv << S->shape.log2g, (uint8_t)L->G.twok, S->s0);
    LinkSlot ls{};
    ls.G = L->G;
    ls.pool = L->pool;
    ls.w = L->w;
    ls.aat = L->aat;
    ls.sa = L->sa;
    ls.sa_cnt = L->sa_cnt;
    ls.cand = L->cand;
    ls.frame_prefix = L->frame_prefix;
    ls.watch = L->watch;
    ls.n_watch = 0;
    ls.tuple_budget = L->p.tuple_budget ? L->p.tuple_budget : (1ull << 32);
    if (e == hipSuccess) e = hipMemcpyAsync(S->d_slots + slot, &ls, sizeof(ls), hipMemcpyHostToDevice, S->s0);
    if (e == hipSuccess) e = hipStreamSynchronize(S->s0);
    if (e != hipSuccess) {
        free_link_device(L);
        return AT_E_DEVICE;
    }
    L->slot = slot;
    L->n_watch = 0;
    S->slot_used[slot] = (int)L->id;
    L->state = L_ACTIVE;
    S->used_bytes += L->bytes;
    return AT_OK;
}

void admit_waiting(at_serve* S) {
    while (!S->waiting.empty()) {
        Link* L = S->links[S->waiting.front()];
        if (S->used_bytes + L->bytes > S->cfg.hbm_budget) break;
        if (admit(S, L) != AT_OK) break;
        S->waiting.pop_front();
    }
}

int capture_graph(at_serve* S) {
    atp::ServeBufs B{};
    B.desc = S->d_desc;
    B.slots = S->d_slots;
    B.state = S->d_state;
    B.hosts = S->d_hosts;
    B.feat = S->d_feat;
    B.est = S->d_est;
    B.pflags = S->d_pflags;
    B.y = S->d_y;
    B.act = S->d_act;
    B.max_hosts = S->max_hosts;
    B.cand_cap = S->cfg.cand_cap;
    atp::MlpDev P{};
    const bool have_mlp = S->mlp && atp::mlp_operands(S->mlp, &P);
    if (S->exec) {
        (void)hipGraphExecDestroy(S->exec);
        S->exec = nullptr;
    }
    if (S->graph) {
        (void)hipGraphDestroy(S->graph);
        S->graph = nullptr;
    }
    hipError_t e = hipStreamBeginCapture(S->s0, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return AT_E_DEVICE;
    hipError_t ec = hipMemcpyAsync(S->d_desc, S->h_desc, sizeof(StepDesc), hipMemcpyHostToDevice, S->s0);
    if (ec == hipSuccess) ec = hipEventRecord(S->ev_fork, S->s0);
    if (ec == hipSuccess) ec = hipStreamWaitEvent(S->s1, S->ev_fork, 0);
    // branch 1: close of slices whose chunks are all scanned (in earlier steps, or
    // by this step's tiled launches, queued ahead of the graph)
    if (ec == hipSuccess) ec = atp::launch_serve_close_branch(B, S->shape, S->n_atv, S->s1);
    if (ec == hipSuccess && have_mlp)
        ec = atp::launch_mlp_forward_devn(S->d_feat, &S->d_state->n_hosts, S->max_hosts, P, S->d_y, S->s1);
    if (ec == hipSuccess)
        ec = have_mlp ? atp::launch_serve_export_learned(B, std::log(16.0) - 0.5, std::log(262144.0) + 0.5,
                                                         S->cfg.theta, S->s1)
                      : atp::launch_serve_export(B, S->s1);
    if (ec == hipSuccess) ec = hipEventRecord(S->ev_join, S->s1);
    // branch 0: open + scan
    if (ec == hipSuccess) ec = atp::launch_serve_ingest_branch(B, S->shape, S->s0);
    if (ec == hipSuccess) ec = hipStreamWaitEvent(S->s0, S->ev_join, 0);
    e = hipStreamEndCapture(S->s0, &S->graph);
    if (ec != hipSuccess || e != hipSuccess) {
        if (S->graph) (void)hipGraphDestroy(S->graph);
        S->graph = nullptr;
        (void)hipGetLastError();
        return AT_E_DEVICE;
    }
    e = hipGraphInstantiate(&S->exec, S->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        S->exec = nullptr;
        return AT_E_DEVICE;
    }
    S->mlp_key = have_mlp ? (const void*)S->mlp : nullptr;
    return AT_OK;
}

void free_server(at_serve* S) {
    if (S->exec) (void)hipGraphExecDestroy(S->exec);
    if (S->graph) (void)hipGraphDestroy(S->graph);
    for (Link* L : S->links) {
        if (L) {
            free_link_device(L);
            delete L;
        }
    }
    void* d[] = {S->d_desc, S->d_slots, S->d_state, S->d_hosts, S->d_feat, S->d_est, S->d_pflags, S->d_y, S->d_act};
    for (void* p : d)
        if (p) (void)hipFree(p);
    void* h[] = {S->h_desc,        S->rs[0].state, S->rs[0].hosts, S->rs[0].est, S->rs[0].estl, S->rs[0].flags,
                 S->rs[1].state,   S->rs[1].hosts, S->rs[1].est,   S->rs[1].estl, S->rs[1].flags};
    for (void* p : h)
        if (p) (void)hipHostFree(p);
    for (uint32_t q = 0; q < atp::kTileJobsMax; q++) {
        for (int x = 0; x < 2; x++) {
            const atp::TileBufs& B = S->tb[x][q];
            void* t[] = {B.rec, B.cnt, B.pre, B.csum, B.base, B.act, S->stage_a[x][q], S->stage_b[x][q]};
            for (void* p : t)
                if (p) (void)hipFree(p);
        }
    }
    for (const std::vector<hipEvent_t>& v : S->tev)
        for (hipEvent_t e : v) (void)hipEventDestroy(e);
    if (S->ev_fork) (void)hipEventDestroy(S->ev_fork);
    if (S->ev_done) (void)hipEventDestroy(S->ev_done);
    for (hipEvent_t ev : S->ev_apply)
        if (ev) (void)hipEventDestroy(ev);
    if (S->ev_join) (void)hipEventDestroy(S->ev_join);
    if (S->s2) (void)hipStreamDestroy(S->s2);
    if (S->s1) (void)hipStreamDestroy(S->s1);
    if (S->s0) (void)hipStreamDestroy(S->s0);
}

// The tiled scan streams the pool once per call; straight byte stores cost a
// partial-line write-back each, about 12 bytes' worth while the pools stay in
// the 256 MiB last-level cache and about 30 once they do not.  So a link's
// step goes tiled when its r*n stores times that cost reach its pool size.
constexpr uint64_t kLastLevelCache = 256ull << 20;
constexpr uint64_t kTileBatch = 8ull << 20;  // pairs per tiled launch

bool take_tiled(const at_serve* S, uint64_t n) {  // caller holds mu
    if (!S->tiled_ok || n == 0) return false;
    uint64_t resident = 0;
    for (int id : S->slot_used)
        if (id >= 0) resident += S->pool_bytes;
    const uint64_t per_store = resident > kLastLevelCache ? 30 : 12;
    return n * S->shape.r * per_store >= S->pool_bytes;
}

int tiled_buffers(at_serve* S, int set, uint32_t slot, uint64_t n) {
    const atp::TileSizes z = atp::tiled_sizes(std::min<uint64_t>(n, kTileBatch), S->pool_bytes, S->shape);
    atp::TileBufs& B = S->tb[set][slot];
    int rc;
    if (z.recs > B.rec_cap) {
        if (B.rec) (void)hipFree(B.rec);
        B.rec_cap = 0;
        if ((rc = dalloc(&B.rec, z.recs))) return rc;
        B.rec_cap = z.recs;
    }
    if (z.table > B.table_cap) {
        if (B.cnt) (void)hipFree(B.cnt);
        if (B.pre) (void)hipFree(B.pre);
        B.cnt = nullptr;
        B.pre = nullptr;
        B.table_cap = 0;
        if ((rc = dalloc(&B.cnt, z.table)) || (rc = dalloc(&B.pre, z.table))) return rc;
        B.table_cap = z.table;
    }
    if (z.nchunk + 2 > B.chunk_cap) {
        if (B.csum) (void)hipFree(B.csum);
        B.chunk_cap = 0;
        if ((rc = dalloc(&B.csum, (uint64_t)(z.nchunk + 2) * 4096))) return rc;
        B.chunk_cap = z.nchunk + 2;
    }
    if (!B.base && (rc = dalloc(&B.base, 4097))) return rc;
    if (!B.act && (rc = dalloc(&B.act, (uint64_t)S->shape.g))) return rc;
    return AT_OK;
}

int stage_buffers(at_serve* S, int set, uint32_t slot, uint64_t n) {
    if (n <= S->stage_cap[set][slot]) return AT_OK;
    if (S->stage_a[set][slot]) (void)hipFree(S->stage_a[set][slot]);
    if (S->stage_b[set][slot]) (void)hipFree(S->stage_b[set][slot]);
    S->stage_a[set][slot] = S->stage_b[set][slot] = nullptr;
    S->stage_cap[set][slot] = 0;
    int rc;
    if ((rc = dalloc(&S->stage_a[set][slot], n)) || (rc = dalloc(&S->stage_b[set][slot], n))) return rc;
    S->stage_cap[set][slot] = n;
    return AT_OK;
}

// One link's chunks of a step, scanned by the tiled scan.

// One tiled launch of the given jobs between a pair of timing events.
// One batch of tiled jobs on scratch set `set`.  Its record passes go on s2
// once the last tile pass that read that set is done; its tile pass goes on
// s0 behind them and behind whatever s0 holds before (the previous step's
// graph, whose closes read the pools).  The record passes touch no pool, so
// on s2 they run beside that graph and the previous step's tile pass, which
// reads the other set.  Events around each half time it.
int launch_timed(at_serve* S, const atp::TileJobSpec* js, uint32_t nj, int set, int tset, uint32_t* n_timed) {
    std::vector<hipEvent_t>& tev = S->tev[tset];
    while (tev.size() < 4 * (*n_timed + 1)) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return AT_E_DEVICE;
        tev.push_back(e);
    }
    hipEvent_t* ev = &tev[4 * *n_timed];
    hipError_t r = hipStreamWaitEvent(S->s2, S->ev_apply[set], 0);
    if (r == hipSuccess) r = hipEventRecord(ev[0], S->s2);
    if (r == hipSuccess) r = atp::launch_ingest_tiled_records(js, nj, S->s2);
    if (r == hipSuccess) r = hipEventRecord(ev[1], S->s2);
    if (r == hipSuccess) r = hipStreamWaitEvent(S->s0, ev[1], 0);
    if (r == hipSuccess) r = hipEventRecord(ev[2], S->s0);
    if (r == hipSuccess) r = atp::launch_ingest_tiled_apply(js, nj, S->s0);
    if (r == hipSuccess) r = hipEventRecord(ev[3], S->s0);
    if (r == hipSuccess) r = hipEventRecord(S->ev_apply[set], S->s0);
    if (r != hipSuccess) return AT_E_DEVICE;
    ++*n_timed;
    return AT_OK;
}

// Launch a step's tiled jobs, their tile passes on s0 ahead of the step
// graph whose closes read these pools.  Jobs share launches, up to
// kTileJobsMax per launch, each with its own scratch slot; a job of more than
// kTileBatch pairs takes launches of its own, one per kTileBatch pairs.
// Gathered chunks are staged on s2, where the record passes read them.
int run_tiled(at_serve* S, std::vector<TiledJob>& jobs, int tset, uint32_t* n_timed, uint32_t* n_jobs) {
    *n_timed = 0;
    *n_jobs = 0;
    if (jobs.empty()) return AT_OK;
    const int set = S->tbuf;  // this step's scratch set; the next step takes the other
    S->tbuf ^= 1;
    atp::TileJobSpec batch[atp::kTileJobsMax];
    uint32_t nb = 0;
    auto flush = [&]() -> int {
        if (nb == 0) return AT_OK;
        const int rc = launch_timed(S, batch, nb, set, tset, n_timed);
        *n_jobs += nb;
        nb = 0;
        return rc;
    };
    for (TiledJob& J : jobs) {
        Link* L = J.L;
        int rc;
        const bool single = J.n <= kTileBatch;
        if (!single || nb == atp::kTileJobsMax)
            if ((rc = flush())) return rc;
        const uint32_t slot = nb;
        rc = tiled_buffers(S, set, slot, J.n);
        if (!rc && J.chunks.size() > 1) rc = stage_buffers(S, set, slot, J.n);
        if (rc) return rc;
        const uint32_t* a = J.chunks[0].aip;
        const uint32_t* b = J.chunks[0].bip;
        if (J.chunks.size() > 1) {
            atp::GatherList G{};
            uint64_t off = 0;
            for (size_t c = 0; c < J.chunks.size(); c++) {
                G.aip[G.n] = J.chunks[c].aip;
                G.bip[G.n] = J.chunks[c].bip;
                G.cnt[G.n] = J.chunks[c].n;
                G.off[G.n] = off;
                off += J.chunks[c].n;
                if (++G.n == atp::kGatherMax || c + 1 == J.chunks.size()) {
                    if (atp::launch_gather_pairs(G, S->stage_a[set][slot], S->stage_b[set][slot], S->s2) != hipSuccess)
                        return AT_E_DEVICE;
                    G.n = 0;
                }
            }
            a = S->stage_a[set][slot];
            b = S->stage_b[set][slot];
        }
        for (uint64_t off = 0; off < J.n; off += kTileBatch) {
            const uint64_t m = std::min<uint64_t>(kTileBatch, J.n - off);
            const bool first = off == 0;
            const bool w = J.weights && single;
            batch[nb++] = atp::TileJobSpec{L->pool, S->pool_bytes, a + off, b + off, m, L->G, J.c0, J.opens && first,
                                           w ? L->w : nullptr, J.kq, S->tb[set][slot]};
            if (!single && (rc = flush())) return rc;
        }
    }
    return flush();
}

}  // namespace

extern "C" {

int at_serve_create(const at_serve_config* cfg, at_serve** out) {
    if (!out || !cfg) return AT_E_INVAL;
    *out = nullptr;
    at_params shp{};
    shp.k = 1;
    shp.r = cfg->r;
    shp.c = cfg->c;
    shp.s = cfg->s;
    shp.u = cfg->u;
    shp.log2g = cfg->log2g;
    shp.theta = cfg->theta;
    if (cfg->max_links < 1 || cfg->max_links > atp::kServeMaxLinks || cfg->cand_cap < 1 || cfg->cand_cap > 2048 ||
        cfg->u > 8 || cfg->watch_cap > 16384)
        return AT_E_INVAL;
    {  // the geometry rules of at_create
        const uint32_t W = 32 - shp.u;
        if (shp.r < 1 || shp.r > (uint32_t)atp::kMaxRows || shp.c < 1 || shp.c > 20 || shp.s < 1 || shp.s > shp.c ||
            shp.c > W || shp.c + shp.s * (shp.r - 1) < W || shp.c * shp.r <= W || shp.s * (shp.r - 1) >= W ||
            shp.log2g < 4 || shp.log2g > 15 || !(shp.theta > 0))
            return AT_E_INVAL;
    }
    at_serve* S = new (std::nothrow) at_serve();
    if (!S) return AT_E_NOMEM;
    S->cfg = *cfg;
    S->shape = atp::derive_geometry(shp);
    S->n_atv = ((uint64_t)(S->shape.umask + 1) * S->shape.r) << S->shape.c;
    S->per_link_bytes = link_bytes(S);
    S->pool_bytes = S->n_atv << S->shape.log2g;
    {
        int dev = 0, lds = 0;
        S->tiled_ok = hipGetDevice(&dev) == hipSuccess &&
                      hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
                      (size_t)lds >= atp::tiled_lds_bytes(4096) + 1024 && atp::tiled_fits(S->pool_bytes);
    }
    S->slot_used.assign(cfg->max_links, -1);
    S->max_hosts = (uint64_t)cfg->max_links * (cfg->cand_cap + cfg->watch_cap);
    int rc = AT_OK;
    hipError_t e = hipStreamCreateWithFlags(&S->s0, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->s1, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->s2, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&S->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&S->ev_done, hipEventDisableTiming);
    for (hipEvent_t& ev : S->ev_apply)
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&S->ev_join, hipEventDisableTiming);
    if (e != hipSuccess) rc = AT_E_DEVICE;
    if (!rc && ((rc = dalloc(&S->d_desc, 1)) || (rc = dalloc(&S->d_slots, atp::kServeMaxLinks)) ||
                (rc = dalloc(&S->d_state, 1)) || (rc = dalloc(&S->d_hosts, S->max_hosts)) ||
                (rc = dalloc(&S->d_feat, S->max_hosts * 64)) || (rc = dalloc(&S->d_est, S->max_hosts)) ||
                (rc = dalloc(&S->d_pflags, S->max_hosts)) || (rc = dalloc(&S->d_y, S->max_hosts)) ||
                (rc = dalloc(&S->d_act, (uint64_t)atp::kServeMaxLinks * S->shape.g)))) {
    }
    if (!rc) {
        if (hipHostMalloc((void**)&S->h_desc, sizeof(StepDesc), 0) != hipSuccess) rc = AT_E_NOMEM;
        const unsigned mf = hipHostMallocMapped;
        for (int q = 0; q < 2 && !rc; q++) {
            at_serve::ResultSet& R = S->rs[q];
            if (hipHostMalloc((void**)&R.state, sizeof(ServeState), mf) != hipSuccess ||
                hipHostMalloc((void**)&R.hosts, S->max_hosts * 4, mf) != hipSuccess ||
                hipHostMalloc((void**)&R.est, S->max_hosts * 8, mf) != hipSuccess ||
                hipHostMalloc((void**)&R.estl, S->max_hosts * 8, mf) != hipSuccess ||
                hipHostMalloc((void**)&R.flags, S->max_hosts, mf) != hipSuccess)
                rc = AT_E_NOMEM;
            R.xp.max_hosts = S->max_hosts;
            if (!rc && (hipHostGetDevicePointer((void**)&R.xp.state, R.state, 0) != hipSuccess ||
                        hipHostGetDevicePointer((void**)&R.xp.hosts, R.hosts, 0) != hipSuccess ||
                        hipHostGetDevicePointer((void**)&R.xp.est, R.est, 0) != hipSuccess ||
                        hipHostGetDevicePointer((void**)&R.xp.est_l, R.estl, 0) != hipSuccess ||
                        hipHostGetDevicePointer((void**)&R.xp.flags, R.flags, 0) != hipSuccess))
                rc = AT_E_DEVICE;
        }
    }
    if (rc) {
        free_server(S);
        delete S;
        return rc;
    }
    memset(S->h_desc, 0, sizeof(StepDesc));
    *out = S;
    return AT_OK;
}

int at_serve_stop(at_serve* S);

int at_serve_destroy(at_serve* S) {
    if (!S) return AT_OK;
    at_serve_stop(S);
    { std::lock_guard<std::mutex> sg(S->step_mu); }
    (void)hipStreamSynchronize(S->s0);
    (void)hipStreamSynchronize(S->s1);
    (void)hipStreamSynchronize(S->s2);
    free_server(S);
    delete S;
    return AT_OK;
}

int at_serve_set_mlp(at_serve* S, at_mlp* m) {
    if (!S) return AT_E_INVAL;
    std::lock_guard<std::mutex> sg(S->step_mu);
    std::lock_guard<std::mutex> g(S->mu);
    S->mlp = m;
    return AT_OK;
}

int at_serve_open_link(at_serve* S, uint32_t k, uint64_t seed, uint64_t tuple_budget, uint32_t* link_id,
                       int* admitted) {
    if (!S || !link_id) return AT_E_INVAL;
    if (k < 1 || k > 127) return AT_E_INVAL;
    std::lock_guard<std::mutex> sg(S->step_mu);
    std::lock_guard<std::mutex> g(S->mu);
    Link* L = new (std::nothrow) Link();
    if (!L) return AT_E_NOMEM;
    L->id = (uint32_t)S->links.size();
    L->p.k = k;
    L->p.r = S->cfg.r;
    L->p.c = S->cfg.c;
    L->p.s = S->cfg.s;
    L->p.u = S->cfg.u;
    L->p.log2g = S->cfg.log2g;
    L->p.theta = S->cfg.theta;
    L->p.seed = seed;
    L->p.tuple_budget = tuple_budget;
    L->G = atp::derive_geometry(L->p);
    L->bytes = S->per_link_bytes;
    S->links.push_back(L);
    *link_id = L->id;
    if (L->bytes > S->cfg.hbm_budget) {
        L->state = L_CLOSED;
        return AT_E_NOMEM;
    }
    if (S->waiting.empty() && S->used_bytes + L->bytes <= S->cfg.hbm_budget) {
        int rc = admit(S, L);
        if (rc == AT_OK) {
            if (admitted) *admitted = 1;
            return AT_OK;
        }
    }
    L->state = L_WAITING;
    S->waiting.push_back(L->id);
    if (admitted) *admitted = 0;
    return AT_OK;
}

int at_serve_link_state(at_serve* S, uint32_t link_id, int* state, uint64_t* slices_closed, uint64_t* pending) {
    if (!S) return AT_E_INVAL;
    std::lock_guard<std::mutex> g(S->mu);
    if (link_id >= S->links.size()) return AT_E_INVAL;
    const Link* L = S->links[link_id];
    if (state) *state = L->state;
    if (slices_closed) *slices_closed = L->t;
    if (pending) *pending = L->q.size();
    return AT_OK;
}

int at_serve_close_link(at_serve* S, uint32_t link_id) {
    if (!S) return AT_E_INVAL;
    std::lock_guard<std::mutex> sg(S->step_mu);
    std::lock_guard<std::mutex> g(S->mu);
    if (link_id >= S->links.size()) return AT_E_INVAL;
    Link* L = S->links[link_id];
    if (L->state == L_CLOSED) return AT_E_STATE;
    if (L->state == L_WAITING) {
        for (auto it = S->waiting.begin(); it != S->waiting.end(); ++it)
            if (*it == link_id) {
                S->waiting.erase(it);
                break;
            }
    } else {
        (void)hipStreamSynchronize(S->s0);
        S->slot_used[L->slot] = -1;
        free_link_device(L);
        S->used_bytes -= L->bytes;
        L->slot = -1;
    }
    L->state = L_CLOSED;
    L->q.clear();
    admit_waiting(S);
    return AT_OK;
}

int at_serve_set_watch(at_serve* S, uint32_t link_id, const uint32_t* hosts_host, uint32_t n) {
    if (!S || (n && !hosts_host)) return AT_E_INVAL;
    std::lock_guard<std::mutex> sg(S->step_mu);
    std::lock_guard<std::mutex> g(S->mu);
    if (link_id >= S->links.size() || n > S->cfg.watch_cap) return AT_E_INVAL;
    Link* L = S->links[link_id];
    if (L->state != L_ACTIVE) return AT_E_STATE;
    hipError_t e = hipSuccess;
    if (n) e = hipMemcpyAsync(L->watch, hosts_host, n * 4, hipMemcpyHostToDevice, S->s0);
    const size_t off = offsetof(LinkSlot, n_watch);
    uint32_t nw = n;
    if (e == hipSuccess)
        e = hipMemcpyAsync(reinterpret_cast<uint8_t*>(S->d_slots + L->slot) + off, &nw, sizeof(nw),
                           hipMemcpyHostToDevice, S->s0);
    if (e == hipSuccess) e = hipStreamSynchronize(S->s0);
    if (e != hipSuccess) return AT_E_DEVICE;
    L->n_watch = n;
    return AT_OK;
}

int at_serve_submit(at_serve* S, uint32_t link_id, const uint32_t* aip_dev, const uint32_t* bip_dev, uint64_t n) {
    if (!S || (n && (!aip_dev || !bip_dev))) return AT_E_INVAL;
    std::lock_guard<std::mutex> g(S->mu);
    if (link_id >= S->links.size()) return AT_E_INVAL;
    Link* L = S->links[link_id];
    if (L->state != L_ACTIVE) return AT_E_STATE;
    if (n == 0) return AT_OK;
    L->q.push_back(Event{false, aip_dev, bip_dev, n, 0, 0.0});
    S->cv.notify_one();
    return AT_OK;
}

int at_serve_end_slice(at_serve* S, uint32_t link_id, uint32_t kprime) {
    if (!S) return AT_E_INVAL;
    const double t = now_ms();
    std::lock_guard<std::mutex> g(S->mu);
    if (link_id >= S->links.size()) return AT_E_INVAL;
    Link* L = S->links[link_id];
    if (L->state != L_ACTIVE) return AT_E_STATE;
    if (kprime < 1 || kprime > L->p.k) return AT_E_INVAL;
    L->q.push_back(Event{true, nullptr, nullptr, 0, kprime, t});
    S->cv.notify_one();
    return AT_OK;
}

int at_serve_submit_last(at_serve* S, uint32_t link_id, const uint32_t* aip_dev, const uint32_t* bip_dev,
                         uint64_t n, uint32_t kprime) {
    if (!S || (n && (!aip_dev || !bip_dev))) return AT_E_INVAL;
    const double t = now_ms();
    std::lock_guard<std::mutex> g(S->mu);
    if (link_id >= S->links.size()) return AT_E_INVAL;
    Link* L = S->links[link_id];
    if (L->state != L_ACTIVE) return AT_E_STATE;
    if (kprime < 1 || kprime > L->p.k) return AT_E_INVAL;
    if (n) L->q.push_back(Event{false, aip_dev, bip_dev, n, 0, 0.0});
    L->q.push_back(Event{true, nullptr, nullptr, 0, kprime, t});
    S->cv.notify_one();
    return AT_OK;
}

}  // extern "C"

namespace {

// The pending closes' results (from mapped set pend_set) into the result
// queue; returns how many.  Caller holds mu.
uint32_t publish_pending(at_serve* S) {
    const at_serve::ResultSet& X = S->rs[S->pend_set];
    const double now = now_ms();
    uint32_t produced = 0;
    for (uint32_t ci = 0; ci < S->pending.size(); ci++) {
        const at_serve::PendingClose& pc = S->pending[ci];
        const atp::CloseOut& o = X.state->out[ci];
        Result R{};
        R.r.link = pc.link;
        R.r.kprime = pc.kq;
        R.r.slice = pc.slice;
        R.r.restore_rc = o.rc;
        R.r.n_out = o.rc == AT_E_BUDGET ? o.U : o.m;
        R.r.n_cand = o.n_cand;
        R.r.n_watch = o.n_hosts - o.n_cand;
        R.r.latency_ms = now - pc.t_arrival;
        R.r.step_ms = S->pend_step_ms;
        const uint64_t h0 = o.host_off, nc = o.n_cand, nw = (uint64_t)o.n_hosts - nc;
        R.cand.assign(X.hosts + h0, X.hosts + h0 + nc);
        R.cand_est.assign(X.est + h0, X.est + h0 + nc);
        R.watch_plain.assign(X.est + h0 + nc, X.est + h0 + nc + nw);
        const uint8_t fb = S->pend_mlp ? 0 : (uint8_t)AT_F_FALLBACK;
        R.cand_flags.resize(nc);
        R.watch_flags.resize(nw);
        for (uint64_t q = 0; q < nc; q++) R.cand_flags[q] = X.flags[h0 + q] | fb;
        for (uint64_t q = 0; q < nw; q++) R.watch_flags[q] = X.flags[h0 + nc + q] | fb;
        if (S->pend_mlp) {
            R.cand_learned.assign(X.estl + h0, X.estl + h0 + nc);
            R.watch_learned.assign(X.estl + h0 + nc, X.estl + h0 + nc + nw);
        } else {
            R.cand_learned = R.cand_est;
            R.watch_learned = R.watch_plain;
        }
        S->results.push_back(std::move(R));
        produced++;
    }
    S->pending.clear();
    return produced;
}


// Every active link with queued work can go into a step of tiled scans and
// their closes only (no direct-path chunk, no close of a slice scanned
// earlier, no empty slice to open): such a step can be planned and its scans
// launched before the previous step's graph has finished.  Caller holds mu.
bool tiled_only(const at_serve* S) {
    bool any = false;
    for (const Link* L : S->links) {
        if (!L || L->state != L_ACTIVE || L->q.empty()) continue;
        if (L->q.front().end) return false;
        uint64_t n = 0;
        for (const Event& ev : L->q) {
            if (ev.end) break;
            if (ev.aip) n += ev.n;
        }
        if (!take_tiled(S, n)) return false;
        any = true;
    }
    return any;
}

// Plan one step from the queues (caller holds mu): the tiled jobs, the
// closes (descriptors and records) and, when D is given, the direct-path
// opens and chunks.  The step's effects on the queues and the link clocks
// are applied at once -- handed chunks and closed ends leave the queues, a
// closed link's clock advances -- since they do not depend on the GPU.
void plan_step(at_serve* S, StepDesc* D, std::vector<TiledJob>& tiled, std::vector<CloseDesc>& cds,
               std::vector<CloseRec>& closes, uint64_t& pairs) {
    for (Link* L : S->links) {
        if (!L || L->state != L_ACTIVE || L->q.empty()) continue;
        const Event& first = L->q.front();
        if (first.end && L->open) {
            // every chunk of this slice was scanned in an earlier step: close it now
            CloseDesc c{};
            c.slot = (uint32_t)L->slot;
            c.c0 = L->c0;
            c.kq = first.kprime;
            c.ready = 0;  // its pairs went in over earlier steps: the close counts the window
            cds.push_back(c);
            closes.push_back(CloseRec{L, first.kprime, first.t_arrival, L->t});
            continue;  // the next slice waits for the next step
        }
        // the step's pairs of this link's current slice, and whether its end follows them
        uint64_t n = 0;
        const Event* end = nullptr;
        for (const Event& ev : L->q) {
            if (ev.end) {
                end = &ev;
                break;
            }
            if (ev.aip) n += ev.n;
        }
        if (take_tiled(S, n)) {
            // scanned ahead of the graph; with its end queued the slice also
            // closes in this step's graph, and a scan that opens it and takes
            // all its pairs (at most one launch) counts the window for it
            TiledJob J{L, {}, n, !L->open, false, end ? end->kprime : 0u, 0};
            if (!L->open) {
                L->open = true;
                L->c0 = (uint32_t)(L->t % L->G.twok);
            }
            J.c0 = L->c0;
            J.weights = J.opens && end && n <= kTileBatch;
            for (Event& ev : L->q) {
                if (ev.end) break;
                if (!ev.aip) continue;
                J.chunks.push_back(TiledChunk{ev.aip, ev.bip, ev.n});
                ev.aip = nullptr;  // handed to this step
            }
            pairs += n;
            if (end) {
                CloseDesc c{};
                c.slot = (uint32_t)L->slot;
                c.c0 = L->c0;
                c.kq = end->kprime;
                c.ready = J.weights ? 1u : 0u;
                cds.push_back(c);
                closes.push_back(CloseRec{L, end->kprime, end->t_arrival, L->t});
            }
            tiled.push_back(std::move(J));
            continue;
        }
        if (!D) continue;  // a tiled-only step never gets here (tiled_only)
        // open the slice if needed, then queue its chunks (stopping at its end)
        if (!L->open) {
            OpenDesc& o = D->open[D->n_open];
            o.slot = (uint32_t)L->slot;
            o.c0 = (uint32_t)(L->t % L->G.twok);
            o.S = atp::preserve_spans(L->G, o.c0);
            D->open_prefix[D->n_open + 1] = D->open_prefix[D->n_open] + S->n_atv * (o.S.nw0 + o.S.nw1);
            D->n_open++;
            L->open = true;
            L->c0 = o.c0;
        }
        for (auto it = L->q.begin(); it != L->q.end() && !it->end; ++it) {
            if (D->n_chunks == atp::kServeMaxChunks) break;
            if (it->aip == nullptr) continue;  // already handed to a step
            ChunkDesc& cd = D->chunk[D->n_chunks++];
            cd.aip = it->aip;
            cd.bip = it->bip;
            cd.n = it->n;
            cd.unit0 = D->n_units;
            cd.slot = (uint32_t)L->slot;
            cd.c0 = L->c0;
            cd.vec = ((reinterpret_cast<uintptr_t>(it->aip) | reinterpret_cast<uintptr_t>(it->bip)) & 15u) == 0;
            D->n_units += (it->n + atp::kServeUnit - 1) / atp::kServeUnit;
            pairs += it->n;
            it->aip = nullptr;  // handed to this step
        }
    }
    // retire handed chunks, then the ends this step closes
    for (Link* L : S->links) {
        if (!L || L->state != L_ACTIVE) continue;
        while (!L->q.empty() && !L->q.front().end && L->q.front().aip == nullptr) {
            L->q.pop_front();
            L->consumed++;
        }
    }
    for (const CloseRec& cr : closes) {
        Link* L = cr.L;
        L->q.pop_front();  // the end event
        L->consumed++;
        L->t += 1;
        L->open = false;
    }
}

// One step.  Its scans and graph go on s0; without `flush`, when the next
// step can be tiled-only its scans are planned and queued at once behind this
// step's graph (the GPU goes on with them while the host collects this step),
// and the previous step's results are published while this one runs; with
// `flush` this step's own results are published before returning.
int serve_step(at_serve* S, uint32_t* n_results, bool flush) {
    if (n_results) *n_results = 0;
    std::lock_guard<std::mutex> sg(S->step_mu);
    std::unique_lock<std::mutex> lk(S->mu);
    if (!S->exec || S->mlp_key != (const void*)S->mlp) {
        int rc = capture_graph(S);
        if (rc) return rc;
    }
    StepDesc& D = *S->h_desc;
    D.n_open = D.n_chunks = D.n_close = 0;
    D.n_units = 0;
    D.open_prefix[0] = 0;
    const int set = S->cur_set;  // this step's results go to mapped set `set`
    D.xp = S->rs[set].xp;
    std::vector<TiledJob> tiled;
    std::vector<CloseDesc> cds;
    std::vector<CloseRec> closes;
    uint64_t pairs = 0;
    at_serve::Ahead& A = S->ahead;
    const bool from_ahead = A.valid;
    int tset = S->tset;
    uint32_t n_timed = 0, n_jobs = 0;
    if (from_ahead) {
        // planned by the previous step, its scans already queued behind that step's graph
        tiled = std::move(A.tiled);
        pairs = A.pairs;
        tset = A.tset;
        n_timed = A.n_timed;
        n_jobs = A.n_jobs;
        for (size_t q = 0; q < A.cds.size(); q++) {
            const Link* L = A.closes[q].L;
            if (L->state != L_ACTIVE || L->slot != (int)A.cds[q].slot) continue;  // closed meanwhile
            cds.push_back(A.cds[q]);
            closes.push_back(A.closes[q]);
        }
        A = at_serve::Ahead{};
    } else {
        plan_step(S, &D, tiled, cds, closes, pairs);
    }
    for (const CloseDesc& c : cds) D.close[D.n_close++] = c;
    lk.unlock();

    const double t0 = now_ms();
    // the tiled scans first: the graph's closes read what they store
    int trc = from_ahead ? AT_OK : run_tiled(S, tiled, tset, &n_timed, &n_jobs);
    hipError_t e = trc ? hipSuccess : hipGraphLaunch(S->exec, S->s0);
    if (e == hipSuccess && !trc) e = hipEventRecord(S->ev_done, S->s0);
    if (e == hipSuccess && !trc && !flush) {
        // the next step, if it is tiled scans and their closes only
        lk.lock();
        if (tiled_only(S)) {
            A.valid = true;
            S->planned_ahead++;
            A.tset = tset ^ 1;
            plan_step(S, nullptr, A.tiled, A.cds, A.closes, A.pairs);
        }
        lk.unlock();
        if (A.valid) trc = run_tiled(S, A.tiled, A.tset, &A.n_timed, &A.n_jobs);
    }
    uint32_t produced = 0;
    {  // the previous step's results (the other mapped set) while this one runs
        std::lock_guard<std::mutex> g(S->mu);
        produced += publish_pending(S);
    }
    if (e == hipSuccess) e = hipEventSynchronize(S->ev_done);
    const double t1 = now_ms();
    if (e != hipSuccess) return AT_E_DEVICE;
    if (trc) return trc;
    float tms = 0.f;
    for (uint32_t q = 0; q < n_timed; q++) {  // record passes plus tile pass of each launch
        const hipEvent_t* ev = &S->tev[tset][4 * q];
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess) tms += ms;
        if (hipEventElapsedTime(&ms, ev[2], ev[3]) == hipSuccess) tms += ms;
    }
    S->tset = tset ^ 1;

    lk.lock();
    S->tiled_ms += tms;
    S->tiled_calls += n_timed;
    S->tiled_jobs += n_jobs;
    S->steps++;
    S->last_step_ms = t1 - t0;
    S->pairs_ingested += pairs;
    for (const TiledJob& J : tiled) S->tiled_pairs += J.n;
    // this step's closes: their results are in set `set`, published by the next
    // step (or below with flush)
    S->pending.clear();
    for (const CloseRec& cr : closes)
        S->pending.push_back(at_serve::PendingClose{cr.L->id, cr.kq, cr.t_arrival, cr.slice});
    S->pend_set = set;
    S->pend_mlp = S->mlp_key != nullptr;
    S->pend_step_ms = t1 - t0;
    S->cur_set = set ^ 1;
    if (flush) produced += publish_pending(S);
    if (n_results) *n_results = produced;
    return AT_OK;
}

}  // namespace

extern "C" {

int at_serve_step(at_serve* S, uint32_t* n_results) {
    if (!S) return AT_E_INVAL;
    return serve_step(S, n_results, true);
}

}  // extern "C"

namespace {

bool has_work(const at_serve* S) {  // caller holds mu
    if (S->ahead.valid) return true;  // a step planned ahead still needs its graph
    for (const Link* L : S->links)
        if (L && L->state == L_ACTIVE && !L->q.empty()) return true;
    return false;
}

void worker_loop(at_serve* S) {
    (void)hipSetDevice(S->device);
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(S->mu);
            if (!has_work(S)) publish_pending(S);  // no step to overlap them with
            S->cv.wait(lk, [&] { return S->stop || has_work(S); });
            if (S->stop && !has_work(S)) return;
        }
        uint32_t n = 0;
        int rc = serve_step(S, &n, false);
        if (rc != AT_OK) {
            std::lock_guard<std::mutex> lk(S->mu);
            S->worker_rc = rc;
            return;
        }
    }
}

}  // namespace

extern "C" {

int at_serve_start(at_serve* S) {
    if (!S) return AT_E_INVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->running) return AT_E_STATE;
    if (hipGetDevice(&S->device) != hipSuccess) return AT_E_DEVICE;
    S->stop = false;
    S->worker_rc = AT_OK;
    S->worker = std::thread(worker_loop, S);
    S->running = true;
    return AT_OK;
}

int at_serve_stop(at_serve* S) {
    if (!S) return AT_E_INVAL;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (!S->running) return AT_OK;
        S->stop = true;
    }
    S->cv.notify_all();
    S->worker.join();
    std::lock_guard<std::mutex> lk(S->mu);
    S->running = false;
    return S->worker_rc;
}

int at_serve_next_result(at_serve* S, at_serve_result* out, uint32_t* cand, double* cand_plain,
                         double* cand_learned, uint8_t* cand_flags, uint32_t cand_cap, double* watch_plain,
                         double* watch_learned, uint8_t* watch_flags, uint32_t watch_cap) {
    if (!S || !out) return AT_E_INVAL;
    std::lock_guard<std::mutex> g(S->mu);
    if (S->results.empty()) return AT_E_STATE;
    Result& R = S->results.front();
    if (R.cand.size() > cand_cap || R.watch_plain.size() > watch_cap) return AT_E_OVERFLOW;
    *out = R.r;
    for (size_t i = 0; i < R.cand.size(); i++) {
        if (cand) cand[i] = R.cand[i];
        if (cand_plain) cand_plain[i] = R.cand_est[i];
        if (cand_learned) cand_learned[i] = R.cand_learned[i];
        if (cand_flags) cand_flags[i] = R.cand_flags[i];
    }
    for (size_t i = 0; i < R.watch_plain.size(); i++) {
        if (watch_plain) watch_plain[i] = R.watch_plain[i];
        if (watch_learned) watch_learned[i] = R.watch_learned[i];
        if (watch_flags) watch_flags[i] = R.watch_flags[i];
    }
    S->results.pop_front();
    return AT_OK;
}

int at_serve_stats(at_serve* S, uint64_t* out4) {
    if (!S || !out4) return AT_E_INVAL;
    std::lock_guard<std::mutex> g(S->mu);
    out4[0] = S->steps;
    out4[1] = S->pairs_ingested;
    out4[2] = S->used_bytes;
    out4[3] = S->waiting.size();
    return AT_OK;
}

int at_serve_tiled_stats(at_serve* S, uint64_t* calls, uint64_t* pairs, double* device_ms, uint64_t* jobs,
                         uint64_t* planned_ahead) {
    if (!S) return AT_E_INVAL;
    std::lock_guard<std::mutex> g(S->mu);
    if (planned_ahead) *planned_ahead = S->planned_ahead;
    if (calls) *calls = S->tiled_calls;
    if (jobs) *jobs = S->tiled_jobs;
    if (pairs) *pairs = S->tiled_pairs;
    if (device_ms) *device_ms = S->tiled_ms;
    return AT_OK;
}

int at_serve_read_pool(at_serve* S, uint32_t link_id, uint8_t* host_out) {
    if (!S || !host_out) return AT_E_INVAL;
    std::lock_guard<std::mutex> sg(S->step_mu);
    std::lock_guard<std::mutex> g(S->mu);
    if (link_id >= S->links.size()) return AT_E_INVAL;
    Link* L = S->links[link_id];
    if (L->state != L_ACTIVE) return AT_E_STATE;
    hipError_t e = hipMemcpyAsync(host_out, L->pool, S->n_atv << S->shape.log2g, hipMemcpyDeviceToHost, S->s0);
    if (e == hipSuccess) e = hipStreamSynchronize(S->s0);
    return e == hipSuccess ? AT_OK : AT_E_DEVICE;
}

}  // extern "C"
