// Batched stepping of many grids (one persistent launch per phase, optional
// HIP graph replay) and the request server built on it (include/vlasov.h).
//
// The host plans each cycle of every member grid with the same state machine
// as vlasov_step: a first half drift (with density partial sums) opens step 1;
// every later cycle closes step s and opens step s + 1 with the fused pair of
// half drifts; the last cycle closes the last step with a single half drift.
// Cycles that open a step also run the density, force and kick of that step.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "vlasov_internal.hpp"

using namespace vlasov_detail;

namespace {

// Persistent launch widths (workgroups) of the four batched phases.
constexpr int KB_FORCE_NT = 1024;

size_t set_bytes(int K) { return align_up(sizeof(vk::GridDesc) * vk::BATCH_MAX + sizeof(vk::Cycle) * (size_t)K); }

struct Member {
    vlasov_ctx *c;
    int64_t total, started, closed;
    // the open step has its first half drift but not yet its kick (after a
    // fused kick and drift pair)
    bool half_open = false;
    bool done() const { return closed == total; }
};

// The fused kick and drift pair runs on a member whose drift offsets vary
// little enough inside its 16-row tiles (tables built for one block per
// tile) and whose p axis is periodic: spreads up to 8 columns on tiles of 230
// columns, up to 56 on tiles of 182.
bool fusable(const vlasov_ctx *c)
{
    return c->kd_spread[0] <= vk::KD_SPR_WIDE && c->kd_rb == 1 && c->P.bc_p == VLASOV_BC_PERIODIC;
}

bool kd_wide(const vlasov_ctx *c) { return c->kd_spread[0] > vk::KD_SPR; }

// The batched fused kernel runs tiles of one 16-row block: a member's fused
// tables must be built for that height (vlasov_set_tuning rebuilds them).
int one_block_tiles(vlasov_ctx *c)
{
    if (c->kd_rb == 1) return VLASOV_OK;
    vlasov_tuning t = c->tune;
    t.kick_drift_blocks = 1;
    return vlasov_set_tuning(c, &t);
}

int kd_tiles(const vlasov_ctx *c)
{
    const int tw = kd_wide(c) ? vk::KB_KD_TW_WIDE : vk::KB_KD_TW;
    return (int)((c->P.nx + tw - 1) / tw) * (int)c->nblk;
}

int drift_tiles(const vlasov_ctx *c)
{
    constexpr int TW = vk::DriftGeom<1, DRIFT_NT, DRIFT_V, 0>::TW;
    return (int)((c->P.nx + TW - 1) / TW) * (int)c->nblk;
}

int kick_tiles(const vlasov_ctx *c)
{
    const int R = c->P.storage == VLASOV_F32 ? kick_rows<float>() : kick_rows<double>();
    return (int)((c->P.nx + 255) / 256) * (int)((c->P.np + R - 1) / R);
}

int force_items(const vlasov_ctx *c)
{
    switch (c->P.model) {
    case VLASOV_MODEL_HMF:
    case VLASOV_MODEL_SHEET:
        return 1;
    case VLASOV_MODEL_RING:
        return (int)((c->P.nx + 15) / 16) + 1;
    default:
        return 0;
    }
}

vk::GridDesc describe(const vlasov_ctx *c)
{
    vk::GridDesc g{};
    g.f[0] = c->f[0];
    g.f[1] = c->f[1];
    g.dm = c->at<int32_t>(c->L.drift_m);
    g.dw = c->at<double4>(c->L.drift_w);
    g.part = c->at<double>(c->L.part);
    g.rho = c->at<double>(c->L.rho);
    g.F = c->at<double>(c->L.F);
    g.Fkick = force_ptr(c);
    g.cs = c->at<double>(c->L.cs);
    g.sn = c->at<double>(c->L.sn);
    g.K = c->at<double>(c->L.ringK);
    g.mxmy = c->at<double>(c->L.mxmy);
    g.hist = c->at<double>(c->L.hist);
    g.hcount = c->at<int64_t>(c->L.hcount);
    g.hcap = c->P.hist_cap;
    g.nx = (int32_t)c->P.nx;
    g.np = (int32_t)c->P.np;
    g.nblk = (int32_t)c->nblk;
    g.model = c->P.model;
    g.bc_x = c->P.bc_x;
    g.bc_p = c->P.bc_p;
    g.dx = c->dx;
    g.dp = c->dp;
    g.dt = c->P.dt;
    g.sheetK = ((2.0 * M_PI) * c->P.sheet_G) * c->dx;
    g.kbase = c->at<int32_t>(c->L.kd_base);
    g.krel = c->at<int32_t>(c->L.kd_rel);
    g.kd_wide = kd_wide(c) ? 1 : 0;
    return g;
}

// Plans and launches chunks of K cycles over a set of member grids.
class Engine {
  public:
    int init(char *dev, size_t bytes, hipStream_t st, int storage, int K, int flags)
    {
        const bool graph = (flags & VLASOV_BATCH_GRAPH) != 0;
        fuse_ = (flags & VLASOV_BATCH_FUSE) != 0;
        if (K < 1 || K > 4096) return fail(VLASOV_E_INVAL, "chunk_cycles must be in [1, 4096]");
        if (!dev || ((uintptr_t)dev % ALIGN) || bytes < 2 * set_bytes(K))
            return fail(VLASOV_E_INVAL, "batch scratch missing, misaligned or too small");
        dev_ = dev;
        st_ = st;
        storage_ = storage;
        K_ = K;
        graph_ = graph;
        // each persistent launch has as many workgroups as the chip holds at once
        int dev_id = 0, ncu = 0;
        HIP_TRY(hipGetDevice(&dev_id));
        HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev_id));
        if (storage == VLASOV_F32) {
            HIP_TRY(size_grids<float>(ncu));
        } else {
            HIP_TRY(size_grids<double>(ncu));
        }
        for (int s = 0; s < 2; ++s) {
            HIP_TRY(hipHostMalloc((void **)&host_[s], set_bytes(K), hipHostMallocDefault));
            HIP_TRY(hipEventCreateWithFlags(&ev_[s], hipEventDisableTiming));
        }
        // graphs are captured on a private stream (the caller's may be the null
        // stream, which cannot be captured) and launched on the caller's
        if (graph) HIP_TRY(hipStreamCreateWithFlags(&cap_, hipStreamNonBlocking));
        return VLASOV_OK;
    }

    void release()
    {
        if (st_ || dev_) (void)hipStreamSynchronize(st_);
        for (int s = 0; s < 2; ++s) {
            if (exec_[s]) (void)hipGraphExecDestroy(exec_[s]);
            if (ev_[s]) (void)hipEventDestroy(ev_[s]);
            if (host_[s]) (void)hipHostFree(host_[s]);
            exec_[s] = nullptr;
            ev_[s] = nullptr;
            host_[s] = nullptr;
        }
        if (cap_) (void)hipStreamDestroy(cap_);
        cap_ = nullptr;
    }

    // Plans K cycles of the members (advancing their state and their contexts'
    // current buffer) and enqueues them.
    int chunk(std::vector<Member *> &ms)
    {
        const int set = set_;
        set_ ^= 1;
        HIP_TRY(hipEventSynchronize(ev_[set]));  // the last upload from this host set is done
        vk::GridDesc *hd = reinterpret_cast<vk::GridDesc *>(host_[set]);
        vk::Cycle *hc = reinterpret_cast<vk::Cycle *>(host_[set] + sizeof(vk::GridDesc) * vk::BATCH_MAX);
        const int n = (int)ms.size();
        for (int a = 0; a < n; ++a) hd[a] = describe(ms[a]->c);
        for (int k = 0; k < K_; ++k) {
            vk::Cycle &cy = hc[k];
            cy.n = n;
            cy.off_drift[0] = cy.off_dens[0] = cy.off_force[0] = cy.off_kick[0] = cy.off_kd[0] = 0;
            for (int a = 0; a < n; ++a) {
                Member &m = *ms[a];
                vlasov_ctx *c = m.c;
                // drift phase: the first half drift of the first step, the
                // pair closing one step and opening the next, or the last
                // half drift; none when the open step has its first half drift
                int kind = vk::DRIFT_NONE, kick = 0, fused = 0;
                if (!m.done()) {
                    if (m.started == m.closed) {
                        kind = vk::DRIFT_FIRST;
                        kick = 1;
                        ++m.started;
                    } else if (m.half_open) {
                        kick = 1;
                    } else if (m.started < m.total) {
                        kind = vk::DRIFT_PAIR;
                        kick = 1;
                        ++m.closed;
                        ++m.started;
                    } else {
                        kind = vk::DRIFT_LAST;
                        ++m.closed;
                    }
                    // kick phase: with a next step to open, the fused kick and
                    // drift pair where the member allows it
                    if (kick && fuse_ && m.started < m.total && fusable(c)) {
                        fused = 1;
                        ++m.closed;
                        ++m.started;
                    }
                    m.half_open = fused != 0;
                }
                cy.slot[a] = a;
                cy.drift[a] = (int8_t)kind;
                cy.kick[a] = (int8_t)kick;
                cy.cur[a] = (int8_t)c->cur;
                cy.kin[a] = (int8_t)(c->cur ^ (kind ? 1 : 0));
                cy.off_drift[a + 1] = cy.off_drift[a] + (kind ? drift_tiles(c) : 0);
                cy.off_dens[a + 1] = cy.off_dens[a] + (kick ? (int)((c->P.nx + 15) / 16) : 0);
                cy.off_force[a + 1] = cy.off_force[a] + (kick ? force_items(c) : 0);
                cy.off_kick[a + 1] = cy.off_kick[a] + (kick && !fused ? kick_tiles(c) : 0);
                cy.off_kd[a + 1] = cy.off_kd[a] + (fused ? kd_tiles(c) : 0);
                if (kind) c->cur ^= 1;
                if (kick) {
                    c->cur ^= 1;
                    c->have_force = true;
                }
            }
        }
        if (fail_at_ >= 0 && chunks_++ == fail_at_)
            return fail(VLASOV_E_HIP, "injected failure of a chunk (VLASOV_TEST_FAIL_CHUNK)");
        char *dset = dev_ + (size_t)set * set_bytes(K_);
        HIP_TRY(hipMemcpyAsync(dset, host_[set], set_bytes(K_), hipMemcpyHostToDevice, st_));
        HIP_TRY(hipEventRecord(ev_[set], st_));
        if (!graph_) return launch_cycles(dset, st_);
        if (!exec_[set]) {
            hipGraph_t g = nullptr;
            HIP_TRY(hipStreamBeginCapture(cap_, hipStreamCaptureModeThreadLocal));
            int rc = launch_cycles(dset, cap_);
            hipError_t e = hipStreamEndCapture(cap_, &g);
            if (rc != VLASOV_OK) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (e != hipSuccess) return fail(VLASOV_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
            e = hipGraphInstantiate(&exec_[set], g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return fail(VLASOV_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
        }
        HIP_TRY(hipGraphLaunch(exec_[set], st_));
        return VLASOV_OK;
    }

  private:
    // Resident workgroups of each persistent kernel (occupancy times CUs).
    template <typename K>
    static hipError_t resident(K kernel, int threads, int ncu, int &out)
    {
        int nb = 0;
        const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, 0);
        out = std::max(1, nb) * ncu;
        return e;
    }

    template <typename T>
    hipError_t size_grids(int ncu)
    {
        hipError_t e = resident(vk::kb_drift<T, DRIFT_NT, DRIFT_V, DRIFT_PF>, DRIFT_NT, ncu, wg_drift_);
        if (e == hipSuccess) e = resident(vk::kb_density, 256, ncu, wg_dens_);
        if (e == hipSuccess) e = resident(vk::kb_force, KB_FORCE_NT, ncu, wg_force_);
        if (e == hipSuccess) e = resident(vk::kb_kick<T, kick_rows<T>()>, 256, ncu, wg_kick_);
        if (e == hipSuccess)
            e = resident(vk::kb_kick_drift<T, kd_pf<T>()>, vk::KDGeom<vk::KB_KD_TW>::NT, ncu, wg_kd_);
        return e;
    }

    template <typename T>
    void launch_cycles_t(char *dset, hipStream_t st)
    {
        const vk::GridDesc *gd = reinterpret_cast<const vk::GridDesc *>(dset);
        const vk::Cycle *cy = reinterpret_cast<const vk::Cycle *>(dset + sizeof(vk::GridDesc) * vk::BATCH_MAX);
        for (int k = 0; k < K_; ++k) {
            vk::kb_drift<T, DRIFT_NT, DRIFT_V, DRIFT_PF><<<wg_drift_, DRIFT_NT, 0, st>>>(gd, cy + k);
            vk::kb_density<<<wg_dens_, 256, 0, st>>>(gd, cy + k);
            vk::kb_force<<<wg_force_, KB_FORCE_NT, 0, st>>>(gd, cy + k);
            vk::kb_kick<T, kick_rows<T>()><<<wg_kick_, 256, 0, st>>>(gd, cy + k);
            if (fuse_) vk::kb_kick_drift<T, kd_pf<T>()><<<wg_kd_, vk::KDGeom<vk::KB_KD_TW>::NT, 0, st>>>(gd, cy + k);
        }
    }

    int launch_cycles(char *dset, hipStream_t st)
    {
        if (storage_ == VLASOV_F32)
            launch_cycles_t<float>(dset, st);
        else
            launch_cycles_t<double>(dset, st);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(VLASOV_E_HIP, std::string("batched launch: ") + hipGetErrorString(e));
        return VLASOV_OK;
    }

    char *dev_ = nullptr;
    hipStream_t st_ = nullptr;
    int storage_ = 0, K_ = 1;
    bool graph_ = false;
    char *host_[2] = {nullptr, nullptr};
    hipEvent_t ev_[2] = {nullptr, nullptr};
    hipGraphExec_t exec_[2] = {nullptr, nullptr};
    hipStream_t cap_ = nullptr;
    int set_ = 0;
    bool fuse_ = false;  // the fused kick and drift pair for the members that allow it
    int wg_drift_ = 1, wg_dens_ = 1, wg_force_ = 1, wg_kick_ = 1, wg_kd_ = 1;  // persistent grid sizes

  public:
    // failure handling tests: the chunk with this index (from 0) fails after
    // its planning, before anything is enqueued (-1: never)
    int64_t fail_at_ = -1, chunks_ = 0;
};

double seconds_since(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

// ---------------------------------------------------------------------------
// Server
// ---------------------------------------------------------------------------
struct vlasov_server {
    char *arena = nullptr;
    size_t arena_bytes = 0, table_bytes = 0;
    hipStream_t stream = nullptr;
    // admissions (tables, initial condition) and retirements (diagnostics,
    // final f) run on streams of their own, beside the chunk on `stream`
    hipStream_t adm = nullptr, ret = nullptr;
    hipEvent_t cev[2] = {nullptr, nullptr};  // end of the last two chunks
    int64_t chunk_seq = 0, completed = -1;   // chunks enqueued, last one known complete
    int storage = 0, max_slots = 0, K = 1;
    int flags = 0;
    std::chrono::steady_clock::time_point t0;

    struct Pending {
        uint64_t ticket;
        vlasov_request req;
        std::vector<double> f0;
        double t_submit;
    };
    struct Entry {
        bool done = false;
        vlasov_result res{};
        std::vector<double> f;
    };
    struct Active {
        uint64_t ticket;
        vlasov_ctx *ctx;
        size_t off, bytes;
        Member m;
        bool keep_f;
        double t_submit, t_admit;
        int32_t failed = VLASOV_OK;  // error of the chunk this request was in
        int64_t closed_before = 0;   // steps finished before the current chunk
        int64_t fin_chunk = -1;      // the chunk that finishes it (-1: none yet)
        bool in_chunk = false;       // stepped by the chunk being enqueued
    };

    std::mutex mu;
    std::condition_variable cv;
    std::deque<Pending> queue;
    std::unordered_map<uint64_t, Entry> entries;
    uint64_t next_ticket = 1;
    bool stopping = false;
    int64_t n_running = 0;
    std::thread th;

    // first-fit allocator over [table_bytes, arena_bytes): offset -> size of free ranges
    std::map<size_t, size_t> free_;
    Engine eng;
    bool eng_ready = false;
    std::vector<Active> active;

    size_t alloc(size_t bytes)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const size_t off = it->first, rest = it->second - bytes;
                free_.erase(it);
                if (rest) free_[off + bytes] = rest;
                return off;
            }
        }
        return (size_t)-1;
    }

    void release(size_t off, size_t bytes)
    {
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

    void finish(uint64_t ticket, const vlasov_result &r, std::vector<double> &&f)
    {
        std::lock_guard<std::mutex> lk(mu);
        Entry &e = entries[ticket];
        e.done = true;
        e.res = r;
        e.f = std::move(f);
    }

    void run();
};

namespace {

// Admits queued requests (FIFO) while a slot and arena space are free.
void admit(vlasov_server *s)
{
    for (;;) {
        vlasov_server::Pending p;
        size_t off = 0, bytes = 0;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            if (s->queue.empty() || (int)s->active.size() >= s->max_slots) return;
            bytes = vlasov_request_footprint(&s->queue.front().req.p);
            off = s->alloc(bytes);
            if (off == (size_t)-1) return;
            p = std::move(s->queue.front());
            s->queue.pop_front();
            ++s->n_running;
        }
        const size_t fb = vlasov_f_bytes(&p.req.p);
        vlasov_ctx *c = nullptr;
        const bool gen = p.req.ic.kind != VLASOV_IC_HOST;
        int rc = vlasov_init(&p.req.p, gen ? nullptr : p.f0.data(), s->arena + off, s->arena + off + align_up(fb),
                             s->adm, &c);
        if (rc == VLASOV_OK && gen) rc = vlasov_generate_ic(c, &p.req.ic);
        if (rc == VLASOV_OK && (s->flags & VLASOV_BATCH_FUSE)) rc = one_block_tiles(c);
        if (rc != VLASOV_OK && c) {
            vlasov_destroy(c);
            c = nullptr;
        }
        // init and generation synchronised the admission stream; from now on
        // the context's work is enqueued on the chunk stream
        if (c) c->stream = s->stream;
        const double t_admit = seconds_since(s->t0);
        if (rc != VLASOV_OK) {
            vlasov_result r{};
            r.status = rc;
            r.t_submit = p.t_submit;
            r.t_admit = r.t_done = t_admit;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                s->release(off, bytes);
                --s->n_running;
            }
            s->finish(p.ticket, r, {});
            continue;
        }
        vlasov_server::Active a;
        a.ticket = p.ticket;
        a.ctx = c;
        a.off = off;
        a.bytes = bytes;
        a.m = Member{c, p.req.nsteps, 0, 0};
        a.keep_f = p.req.keep_f != 0;
        a.t_submit = p.t_submit;
        a.t_admit = t_admit;
        s->active.push_back(a);
    }
}

// Retires finished members: diagnostics, optional final f, arena space back.
// Retires the members whose last chunk is complete (diagnostics and the
// final f on the retire stream, beside the chunk that may be running).
void retire(vlasov_server *s)
{
    std::vector<vlasov_server::Active> keep;
    for (auto &a : s->active) {
        if (!a.m.done() || a.fin_chunk > s->completed) {
            keep.push_back(a);
            continue;
        }
        a.ctx->stream = s->ret;
        vlasov_result r{};
        std::vector<double> f;
        if (a.failed != VLASOV_OK) {
            // the chunk's kernels may not have run (planning already moved the
            // context to its output buffer): no diagnostics, no f
            r.status = a.failed;
            r.steps_done = a.closed_before;
        } else {
            r.status = vlasov_moments(a.ctx, &r.m);
            r.steps_done = a.m.closed;
        }
        if (a.keep_f && a.failed == VLASOV_OK) {
            f.resize((size_t)a.ctx->P.nx * (size_t)a.ctx->P.np);
            int rc = vlasov_read_f(a.ctx, f.data());
            if (rc != VLASOV_OK && r.status == VLASOV_OK) r.status = rc;
        }
        r.t_submit = a.t_submit;
        r.t_admit = a.t_admit;
        r.t_done = seconds_since(s->t0);
        vlasov_destroy(a.ctx);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->release(a.off, a.bytes);
            --s->n_running;
        }
        s->finish(a.ticket, r, std::move(f));
    }
    s->active.swap(keep);
}

}  // namespace

void vlasov_server::run()
{
    int dev = 0;
    bool dev_set = false;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait(lk, [&] { return stopping || !queue.empty() || !active.empty(); });
            if (stopping && queue.empty() && active.empty()) break;
        }
        if (!dev_set) {
            (void)hipPointerGetAttribute(&dev, HIP_POINTER_ATTRIBUTE_DEVICE_ORDINAL, (hipDeviceptr_t)arena);
            (void)hipSetDevice(dev);
            dev_set = true;
        }
        if (!eng_ready) {
            int rc = eng.init(arena, table_bytes, stream, storage, K, flags);
            if (rc == VLASOV_OK &&
                (hipStreamCreateWithFlags(&adm, hipStreamNonBlocking) != hipSuccess ||
                 hipStreamCreateWithFlags(&ret, hipStreamNonBlocking) != hipSuccess ||
                 hipEventCreateWithFlags(&cev[0], hipEventDisableTiming) != hipSuccess ||
                 hipEventCreateWithFlags(&cev[1], hipEventDisableTiming) != hipSuccess))
                rc = fail(VLASOV_E_HIP, "server streams");
            if (rc != VLASOV_OK) {
                // fail every queued request
                std::unique_lock<std::mutex> lk(mu);
                const std::string why = vlasov_last_error();
                for (auto &p : queue) {
                    Entry &e = entries[p.ticket];
                    e.done = true;
                    e.res.status = VLASOV_E_HIP;
                    e.res.t_submit = p.t_submit;
                }
                queue.clear();
                continue;
            }
            eng_ready = true;
        }
        admit(this);
        if (active.empty()) {
            // nothing fits (can only happen transiently): wait for more work
            std::this_thread::sleep_for(std::chrono::microseconds(200));
            continue;
        }
        // One chunk ahead: chunk n is enqueued before the host waits for
        // chunk n - 1 and retires the requests it finished, so the GPU runs
        // while the host retires and admits.
        std::vector<Member *> ms;
        for (auto &a : active) {
            a.in_chunk = !a.m.done();  // else finishing in an earlier chunk, or nothing to do
            if (!a.in_chunk) continue;
            a.closed_before = a.m.closed;
            ms.push_back(&a.m);
        }
        bool launched = false;
        if (!ms.empty()) {
            int rc = eng.chunk(ms);
            if (rc == VLASOV_OK) {
                const hipError_t e = hipEventRecord(cev[chunk_seq & 1], stream);
                if (e != hipSuccess) rc = fail(VLASOV_E_HIP, std::string("chunk event: ") + hipGetErrorString(e));
            }
            if (rc != VLASOV_OK) {
                // the requests of this chunk fail with its error and leave
                (void)hipStreamSynchronize(stream);
                for (auto &a : active) {
                    if (!a.in_chunk) continue;
                    a.failed = rc;
                    a.m.closed = a.m.total;
                    a.fin_chunk = -1;
                }
                completed = chunk_seq - 1;
            } else {
                for (auto &a : active)
                    if (a.m.done() && a.fin_chunk < 0 && a.closed_before < a.m.closed) a.fin_chunk = chunk_seq;
                launched = true;
            }
            ++chunk_seq;
        }
        const int64_t want = launched ? chunk_seq - 2 : chunk_seq - 1;
        if (want > completed) {
            if (hipEventSynchronize(cev[want & 1]) != hipSuccess) {
                (void)hipStreamSynchronize(stream);
                // a device error: every running request fails and leaves
                for (auto &a : active) {
                    if (!a.m.done() || a.fin_chunk >= 0) a.failed = VLASOV_E_HIP;
                    a.m.closed = a.m.total;
                    a.fin_chunk = -1;
                }
            }
            completed = want;
        }
        retire(this);
    }
    if (chunk_seq > 0) (void)hipStreamSynchronize(stream);
    if (eng_ready) eng.release();
    for (auto e : cev)
        if (e) (void)hipEventDestroy(e);
    if (adm) (void)hipStreamDestroy(adm);
    if (ret) (void)hipStreamDestroy(ret);
}

extern "C" {

size_t vlasov_batch_scratch_bytes(int32_t chunk_cycles)
{
    if (chunk_cycles < 1 || chunk_cycles > 4096) return 0;
    return 2 * set_bytes(chunk_cycles);
}

int vlasov_batch_step(vlasov_ctx *const *ctxs, int32_t n, const int64_t *nsteps, void *scratch_dev,
                      size_t scratch_bytes, int32_t chunk_cycles, int32_t flags)
{
    if (!ctxs || !nsteps || n < 1 || n > vk::BATCH_MAX) return fail(VLASOV_E_INVAL, "need 1..VLASOV_BATCH_MAX (256) contexts");
    for (int a = 0; a < n; ++a) {
        if (!ctxs[a]) return fail(VLASOV_E_INVAL, "NULL context");
        if (nsteps[a] < 0) return fail(VLASOV_E_INVAL, "nsteps must be >= 0");
        if (ctxs[a]->P.storage != ctxs[0]->P.storage) return fail(VLASOV_E_INVAL, "mixed storage types");
        if (ctxs[a]->stream != ctxs[0]->stream) return fail(VLASOV_E_INVAL, "contexts on different streams");
        if (ctxs[a]->P.spline != VLASOV_SPLINE_FD) return fail(VLASOV_E_INVAL, "batches run the local spline only");
        if (ctxs[a]->P.splitting != VLASOV_SPLIT_STRANG || ctxs[a]->P.filter_every != 0)
            return fail(VLASOV_E_INVAL, "batches run the Strang splitting without filter only");
        for (int b = 0; b < a; ++b)
            if (ctxs[b] == ctxs[a]) return fail(VLASOV_E_INVAL, "a context appears twice");
    }
    if (flags & VLASOV_BATCH_FUSE)
        for (int a = 0; a < n; ++a) {
            const int rt = one_block_tiles(ctxs[a]);
            if (rt != VLASOV_OK) return rt;
        }
    Engine eng;
    int rc = eng.init((char *)scratch_dev, scratch_bytes, ctxs[0]->stream, ctxs[0]->P.storage, chunk_cycles, flags);
    if (rc != VLASOV_OK) {
        eng.release();
        return rc;
    }
    std::vector<Member> mem((size_t)n);
    std::vector<Member *> ms;
    for (int a = 0; a < n; ++a) {
        mem[a] = Member{ctxs[a], nsteps[a], 0, 0};
        ms.push_back(&mem[a]);
    }
    for (;;) {
        bool all = true;
        for (auto *m : ms) all = all && m->done();
        if (all) break;
        if ((rc = eng.chunk(ms)) != VLASOV_OK) break;
    }
    eng.release();
    if (rc == VLASOV_OK)
        for (int a = 0; a < n; ++a) ctxs[a]->steps_done += nsteps[a];
    return rc;
}

size_t vlasov_request_footprint(const vlasov_params *p)
{
    const size_t fb = vlasov_f_bytes(p), wb = vlasov_workspace_bytes(p);
    if (!fb || !wb) return 0;
    return align_up(fb) + align_up(wb);
}

size_t vlasov_server_table_bytes(int32_t chunk_cycles) { return vlasov_batch_scratch_bytes(chunk_cycles); }

int vlasov_server_create(void *arena_dev, size_t arena_bytes, void *hip_stream, int32_t storage, int32_t max_slots,
                         int32_t chunk_cycles, int32_t flags, vlasov_server **out)
{
    if (!arena_dev || !out || ((uintptr_t)arena_dev % ALIGN)) return fail(VLASOV_E_INVAL, "bad arena or output");
    if (storage != VLASOV_F64 && storage != VLASOV_F32) return fail(VLASOV_E_INVAL, "unknown storage");
    if (max_slots < 1 || max_slots > vk::BATCH_MAX) return fail(VLASOV_E_INVAL, "max_slots must be in [1, VLASOV_BATCH_MAX = 256]");
    const size_t tb = vlasov_server_table_bytes(chunk_cycles);
    if (!tb) return fail(VLASOV_E_INVAL, "chunk_cycles must be in [1, 4096]");
    if (arena_bytes <= tb) return fail(VLASOV_E_INVAL, "arena smaller than the server tables");
    vlasov_server *s = new vlasov_server();
    s->arena = (char *)arena_dev;
    s->arena_bytes = arena_bytes;
    s->table_bytes = tb;
    s->stream = (hipStream_t)hip_stream;
    s->storage = storage;
    s->max_slots = max_slots;
    s->K = chunk_cycles;
    s->flags = flags;
    if (const char *v = getenv("VLASOV_TEST_FAIL_CHUNK")) s->eng.fail_at_ = strtoll(v, nullptr, 10);
    s->t0 = std::chrono::steady_clock::now();
    s->free_[tb] = (arena_bytes - tb) / ALIGN * ALIGN;
    s->th = std::thread([s] { s->run(); });
    *out = s;
    return VLASOV_OK;
}

int vlasov_submit(vlasov_server *s, const vlasov_request *r, const double *f0_host, uint64_t *ticket)
{
    if (!s || !r || !ticket) return fail(VLASOV_E_INVAL, "NULL argument");
    if (r->ic.kind == VLASOV_IC_HOST) {
        if (!f0_host) return fail(VLASOV_E_INVAL, "f0_host is NULL for a request without a generated initial condition");
    } else {
        const std::string bad = validate_ic(&r->ic);
        if (!bad.empty()) return fail(VLASOV_E_INVAL, bad);
    }
    const std::string why = validate(&r->p);
    if (!why.empty()) return fail(VLASOV_E_INVAL, why);
    if (r->p.storage != s->storage) return fail(VLASOV_E_INVAL, "request storage differs from the server's");
    if (r->p.hist_cap != 0) return fail(VLASOV_E_INVAL, "requests keep no magnetization history");
    if (r->p.spline != VLASOV_SPLINE_FD) return fail(VLASOV_E_INVAL, "the server runs the local spline only");
    if (r->p.splitting != VLASOV_SPLIT_STRANG || r->p.filter_every != 0)
        return fail(VLASOV_E_INVAL, "the server runs the Strang splitting without filter only");
    if (r->nsteps < 0) return fail(VLASOV_E_INVAL, "nsteps must be >= 0");
    const size_t bytes = vlasov_request_footprint(&r->p);
    if (bytes > s->arena_bytes - s->table_bytes) return fail(VLASOV_E_NOMEM, "request larger than the arena");
    vlasov_server::Pending p;
    p.req = *r;
    if (r->ic.kind == VLASOV_IC_HOST) p.f0.assign(f0_host, f0_host + (size_t)r->p.nx * (size_t)r->p.np);
    p.t_submit = seconds_since(s->t0);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stopping) return fail(VLASOV_E_STATE, "server is shutting down");
        p.ticket = s->next_ticket++;
        *ticket = p.ticket;
        s->entries[p.ticket] = vlasov_server::Entry{};
        s->queue.push_back(std::move(p));
    }
    s->cv.notify_one();
    return VLASOV_OK;
}

int vlasov_poll(vlasov_server *s, uint64_t ticket, vlasov_result *out, double *f_host)
{
    if (!s || !out) return fail(VLASOV_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->entries.find(ticket);
    if (it == s->entries.end()) return fail(VLASOV_E_NOTFOUND, "unknown ticket");
    if (!it->second.done) return VLASOV_PENDING;
    *out = it->second.res;
    if (f_host && !it->second.f.empty()) memcpy(f_host, it->second.f.data(), it->second.f.size() * sizeof(double));
    s->entries.erase(it);
    return VLASOV_OK;
}

int vlasov_server_stats(vlasov_server *s, int64_t *queued, int64_t *running, int64_t *done)
{
    if (!s) return fail(VLASOV_E_INVAL, "NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    int64_t d = 0;
    for (auto &kv : s->entries) d += kv.second.done ? 1 : 0;
    if (queued) *queued = (int64_t)s->queue.size();
    if (running) *running = s->n_running;
    if (done) *done = d;
    return VLASOV_OK;
}

int vlasov_server_destroy(vlasov_server *s)
{
    if (!s) return VLASOV_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv.notify_all();
    if (s->th.joinable()) s->th.join();
    delete s;
    return VLASOV_OK;
}

}  // extern "C"
