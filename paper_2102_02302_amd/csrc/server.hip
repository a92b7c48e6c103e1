// Served form, native: continuous batching of independent embedding
// requests on one GPU.
//
// Threads: callers submit requests (edge arrays) and poll completions.
// Builder threads, each with its own stream and pinned staging buffer, take
// a free slot (a library context) and form a *group* when they are free to
// build it: the waiting requests in arrival order, up to max_group, whose
// summed footprint fits the budget.  A builder packs the group's edges,
// copies them to the device once and builds the group as one block-diagonal
// graph (one build for all its members).  One scheduler thread steps every
// built group by one iteration per step, all groups in shared launches
// (step_contexts), and retires a group that reached k iterations by
// asynchronous copies of each member's rows to its output buffer.  A
// block-diagonal build gives every member the same bits as building it
// alone, so grouping changes speed, not results.  A slot is reused only
// after its result copies have completed.  Which requests form a group,
// on which slot, and what device memory that is charged is decided by the
// host-only policy of admission.hpp.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "admission.hpp"
#include "internal.hpp"

namespace {

struct SReq {
    int64_t ticket = 0;
    cleora_request r{};
    double submit_s = 0, admit_s = -1, ready_s = -1, done_s = -1;
    int64_t footprint = 0;  // charge: cleora_footprint_bytes plus staging
    int64_t row0 = 0;  // first row inside its group's block-diagonal graph
    int32_t status = CLEORA_OK;
    bool on_dev[3] = {false, false, false};  // src, dst, w in device memory
};

// Device memory is copied on the device; host memory (pageable, pinned or
// managed) is read by the builder thread.
bool is_device_ptr(const void *p)
{
    if (!p) return false;
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeArray;
}

struct Group {
    std::vector<SReq *> members;
    int slot = -1;
    int32_t iteration = 0;
    int64_t footprint = 0;
    int32_t status = CLEORA_OK;
};

double seconds_since(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// Pinned host staging of one builder thread (grow-only).
struct HostBuf {
    void *p = nullptr;
    size_t cap = 0;
    void ensure(size_t bytes)
    {
        if (bytes <= cap) return;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
        if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            throw cleora::Error(CLEORA_E_NOMEM, "pinned staging allocation failed");
        }
        cap = bytes;
    }
    ~HostBuf()
    {
        if (p) (void)hipHostFree(p);
    }
};

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Staging bytes a request adds to its group's buffer: src, dst and weights
// (4 bytes each per edge), its three table entries and the 256-byte
// alignment of the three arrays (a group's staging never exceeds the sum
// over its members).
int64_t staging_bytes(int64_t n_edges) { return 12 * n_edges + 1024; }

}  // namespace

struct cleora_server {
    int device = 0;
    int32_t dim = 0, dtype = 0, k = 0, max_group = 1;
    int32_t pack_threads = 4;  // threads that copy one large group's edges
    uint32_t flags = 0;
    int64_t budget = 0;
    std::vector<cleora_ctx *> ctxs;
    std::vector<cleora::DevBuf> staging;  // per slot: the group's edges and tables
    std::unique_ptr<cleora::Admission> policy;  // queue, slots and memory charges
    int64_t bound_exceeded = 0;  // builds that held more than they were charged

    std::mutex mu;
    std::condition_variable cv_sched, cv_build, cv_done;
    std::deque<SReq *> pending, done;  // pending mirrors the policy's queue
    std::vector<Group *> building, ready;
    int64_t next_ticket = 0, in_system = 0;
    bool stop = false;
    std::string fatal;

    // scheduler-thread state
    std::vector<Group *> active;
    std::vector<std::pair<hipEvent_t, Group *>> retiring;
    std::vector<hipEvent_t> ev_pool;
    int64_t steps = 0, stepped = 0;
    int32_t max_active = 0;

    std::thread sched;
    std::vector<std::thread> builders;
    hipStream_t main_s = nullptr;
    std::vector<hipStream_t> bstreams;
    std::chrono::steady_clock::time_point t0;

    // caller holds mu: complete every member of g, free the slot
    void finish(Group *g)
    {
        const double t = seconds_since(t0);
        for (SReq *q : g->members) {
            if (q->status == CLEORA_OK) q->status = g->status;
            q->done_s = t;
            done.push_back(q);
        }
        policy->release(g->slot);
        delete g;
        cv_done.notify_all();
        cv_build.notify_one();
    }

    // Build all members as one block-diagonal graph (members whose ids are
    // out of range are dropped first, with E_INPUT).
    void build_group(Group *g, hipStream_t s, HostBuf &host)
    {
        cleora::TraceRange trace_range("cleora_server build group");
        const size_t nm = g->members.size();
        bool any_w = false;
        int64_t m_total = 0, n_total = 0;
        for (SReq *q : g->members) {
            any_w = any_w || q->r.w != nullptr;
            m_total += q->r.n_edges;
            n_total += q->r.n_nodes;
        }
        const int64_t m1 = std::max<int64_t>(m_total, 1);
        const size_t off_src = 0, off_dst = align256(4 * (size_t)m1),
                     off_w = off_dst + align256(4 * (size_t)m1),
                     off_tab = off_w + (any_w ? align256(4 * (size_t)m1) : 0),
                     tab_bytes = 8 * (3 * nm + 2), total = off_tab + tab_bytes;
        host.ensure(total);
        char *h = static_cast<char *>(host.p);
        int64_t *row0 = reinterpret_cast<int64_t *>(h + off_tab), *eoff = row0 + nm + 1;
        uint64_t *seeds = reinterpret_cast<uint64_t *>(eoff + nm + 1);
        int64_t e = 0, r = 0;
        for (size_t i = 0; i < nm; ++i) {
            const cleora_request &q = g->members[i]->r;
            row0[i] = r;
            eoff[i] = e;
            seeds[i] = q.seed;
            g->members[i]->row0 = r;
            e += q.n_edges;
            r += q.n_nodes;
        }
        row0[nm] = r;
        eoff[nm] = e;
        // the members' host edge arrays into the pinned staging; a large
        // group is copied by several threads (the copy, not the GPU, bounds
        // the builders of a busy server)
        auto pack = [&](size_t i0, size_t i1) {
            for (size_t i = i0; i < i1; ++i) {
                const cleora_request &q = g->members[i]->r;
                const bool *dv = g->members[i]->on_dev;
                const int64_t at = eoff[i];
                if (q.n_edges <= 0) continue;
                if (!dv[0]) std::memcpy(h + off_src + 4 * at, q.src, 4 * (size_t)q.n_edges);
                if (!dv[1]) std::memcpy(h + off_dst + 4 * at, q.dst, 4 * (size_t)q.n_edges);
                if (any_w) {
                    float *wd = reinterpret_cast<float *>(h + off_w) + at;
                    if (!q.w) std::fill(wd, wd + q.n_edges, 1.0f);
                    else if (!dv[2]) std::memcpy(wd, q.w, 4 * (size_t)q.n_edges);
                }
            }
        };
        const int64_t pack_bytes = (any_w ? 12 : 8) * m_total;
        const size_t parts =
            std::min<size_t>(nm, pack_bytes >= (8 << 20) ? (size_t)pack_threads : 1);
        if (parts <= 1) {
            pack(0, nm);
        } else {
            // split the members into `parts` runs of about equal edge counts
            std::vector<std::thread> th;
            size_t i0 = 0;
            for (size_t p = 0; p < parts && i0 < nm; ++p) {
                const int64_t goal = (int64_t)((double)m_total * (double)(p + 1) / (double)parts);
                size_t i1 = i0 + 1;
                while (i1 < nm && eoff[i1] < goal) ++i1;
                if (p + 1 == parts) i1 = nm;
                if (p + 1 < parts) th.emplace_back(pack, i0, i1);
                else pack(i0, i1);
                i0 = i1;
            }
            for (std::thread &t : th) t.join();
        }
        cleora::DevBuf &st = staging[g->slot];
        st.ensure(total);
        CLEORA_HIP(hipMemcpyAsync(st.p, host.p, total, hipMemcpyHostToDevice, s));
        char *d = st.as<char>();
        // device-resident arrays go after the packed copy, over their ranges
        for (size_t i = 0; i < nm; ++i) {
            const cleora_request &q = g->members[i]->r;
            const bool *dv = g->members[i]->on_dev;
            const size_t at = 4 * (size_t)eoff[i], bytes = 4 * (size_t)q.n_edges;
            if (bytes == 0) continue;
            if (dv[0])
                CLEORA_HIP(hipMemcpyAsync(d + off_src + at, q.src, bytes, hipMemcpyDeviceToDevice, s));
            if (dv[1])
                CLEORA_HIP(hipMemcpyAsync(d + off_dst + at, q.dst, bytes, hipMemcpyDeviceToDevice, s));
            if (dv[2])
                CLEORA_HIP(hipMemcpyAsync(d + off_w + at, q.w, bytes, hipMemcpyDeviceToDevice, s));
        }
        cleora::build_group_and_init(
            ctxs[g->slot], (int32_t)nm, n_total, m_total, reinterpret_cast<int32_t *>(d + off_src),
            reinterpret_cast<int32_t *>(d + off_dst),
            any_w ? reinterpret_cast<float *>(d + off_w) : nullptr,
            reinterpret_cast<int64_t *>(d + off_tab),
            reinterpret_cast<int64_t *>(d + off_tab) + nm + 1,
            reinterpret_cast<uint64_t *>(reinterpret_cast<int64_t *>(d + off_tab) + 2 * nm + 2),
            flags, dim, dtype, s);
        // the pinned staging is reused by this thread's next group
        CLEORA_HIP(hipStreamSynchronize(s));
    }

    // Host check of one request's ids and weights (the error path only:
    // device-resident arrays are copied back for it).
    static bool request_ok(const SReq &q)
    {
        const int64_t m = q.r.n_edges;
        std::vector<int32_t> ids;
        std::vector<float> wts;
        const int32_t *src = q.r.src, *dst = q.r.dst;
        const float *w = q.r.w;
        if (m > 0 && (q.on_dev[0] || q.on_dev[1])) {
            ids.resize(2 * (size_t)m);
            if (hipMemcpy(ids.data(), src, 4 * (size_t)m, hipMemcpyDefault) != hipSuccess ||
                hipMemcpy(ids.data() + m, dst, 4 * (size_t)m, hipMemcpyDefault) != hipSuccess)
                return false;
            src = ids.data();
            dst = ids.data() + m;
        }
        if (m > 0 && w && q.on_dev[2]) {
            wts.resize((size_t)m);
            if (hipMemcpy(wts.data(), w, 4 * (size_t)m, hipMemcpyDefault) != hipSuccess)
                return false;
            w = wts.data();
        }
        for (int64_t e = 0; e < m; ++e)
            if (src[e] < 0 || src[e] >= q.r.n_nodes || dst[e] < 0 || dst[e] >= q.r.n_nodes)
                return false;
        if (w)
            for (int64_t e = 0; e < m; ++e)
                if (!(w[e] > 0.0f && w[e] <= 3.402823466e38f)) return false;
        return true;
    }

    void build_loop(int bi)
    {
        (void)hipSetDevice(device);
        hipStream_t s = bstreams[bi];
        HostBuf host;
        for (;;) {
            Group *g = nullptr;
            cleora::AdmitDecision dec;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_build.wait(lk, [&] { return stop || policy->can_admit(); });
                if (stop) return;
                dec = policy->admit();
                g = take_group_locked(dec);
                building.push_back(g);
            }
            if (!dec.trim.empty()) {
                // idle slots give their buffers back to make room (nothing
                // runs on them: a slot is freed after its last copy ended)
                for (int t : dec.trim) release_slot(t);
                std::lock_guard<std::mutex> lk(mu);
                for (int t : dec.trim)
                    if (t != g->slot) policy->trimmed(t);
                cv_build.notify_all();
            }
            int32_t status = CLEORA_OK;
            try {
                build_group(g, s, host);
            } catch (const cleora::Error &e) {
                status = e.code;
            } catch (...) {
                status = CLEORA_E_DEVICE;
            }
            if (status == CLEORA_E_INPUT && g->members.size() > 1) {
                // find the bad members on the host, rebuild without them
                std::vector<SReq *> keep, bad;
                for (SReq *q : g->members) (request_ok(*q) ? keep : bad).push_back(q);
                for (SReq *q : bad) q->status = CLEORA_E_INPUT;
                g->members = keep;
                status = keep.empty() ? CLEORA_E_INPUT : CLEORA_OK;
                if (!keep.empty()) {
                    try {
                        build_group(g, s, host);
                    } catch (const cleora::Error &e) {
                        status = e.code;
                    } catch (...) {
                        status = CLEORA_E_DEVICE;
                    }
                }
                std::lock_guard<std::mutex> lk(mu);
                const double t = seconds_since(t0);
                for (SReq *q : bad) {
                    q->done_s = t;
                    done.push_back(q);
                }
                if (!bad.empty()) cv_done.notify_all();
            }
            const int64_t held = slot_bytes(g->slot);
            std::lock_guard<std::mutex> lk(mu);
            if (!policy->built(g->slot, held)) ++bound_exceeded;
            building.erase(std::find(building.begin(), building.end(), g));
            g->status = status;
            const double t = seconds_since(t0);
            for (SReq *q : g->members) q->ready_s = t;
            if (stop) {
                // nobody steps it any more (destroy, or a device error)
                if (g->status == CLEORA_OK) g->status = CLEORA_E_DEVICE;
                finish(g);
                continue;
            }
            ready.push_back(g);
            cv_sched.notify_one();
            cv_build.notify_one();
        }
    }

    hipEvent_t take_event()
    {
        if (!ev_pool.empty()) {
            hipEvent_t e = ev_pool.back();
            ev_pool.pop_back();
            return e;
        }
        hipEvent_t e;
        CLEORA_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        return e;
    }

    // The group the policy formed: the first dec.count waiting requests.
    Group *take_group_locked(const cleora::AdmitDecision &dec)
    {
        Group *g = new Group();
        const double t = seconds_since(t0);
        for (int32_t i = 0; i < dec.count; ++i) {
            SReq *q = pending.front();
            pending.pop_front();
            q->admit_s = t;
            g->members.push_back(q);
        }
        g->slot = dec.slot;
        g->footprint = dec.footprint;
        return g;
    }

    // Device bytes slot `i` holds: its context's buffers and its staging.
    int64_t slot_bytes(int i)
    {
        return cleora::ctx_device_bytes(ctxs[i]) + (int64_t)staging[i].cap;
    }

    void release_slot(int i)
    {
        cleora::release_buffers(ctxs[i]);
        staging[i].release();
    }

    void sched_loop()
    {
        (void)hipSetDevice(device);
        const size_t es = dtype == CLEORA_BF16 ? 2 : 4;
        std::vector<cleora_ctx *> list;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu);
                if (stop) return;
                for (Group *g : ready) {
                    if (g->status != CLEORA_OK || k == 0) {
                        if (g->status != CLEORA_OK || g->members.empty()) {
                            finish(g);
                            continue;
                        }
                        g->iteration = k;  // k = 0: retire straight away below
                    }
                    active.push_back(g);
                }
                ready.clear();
                if (active.empty() && retiring.empty()) {
                    cv_sched.wait_for(lk, std::chrono::microseconds(200));
                    continue;
                }
            }
            try {
                for (size_t i = 0; i < retiring.size();) {
                    if (hipEventQuery(retiring[i].first) == hipSuccess) {
                        ev_pool.push_back(retiring[i].first);
                        std::lock_guard<std::mutex> lk(mu);
                        finish(retiring[i].second);
                        retiring[i] = retiring.back();
                        retiring.pop_back();
                    } else {
                        ++i;
                    }
                }
                if (active.empty()) {
                    std::this_thread::sleep_for(std::chrono::microseconds(20));
                    continue;
                }
                list.clear();
                for (Group *g : active)
                    if (g->iteration < k) list.push_back(ctxs[g->slot]);
                if (!list.empty()) {
                    cleora::TraceRange trace_range("cleora_server step");
                    cleora::step_contexts(list.data(), (int32_t)list.size(), main_s);
                    ++steps;
                    max_active = std::max(max_active, (int32_t)list.size());
                }
                std::vector<Group *> still;
                for (Group *g : active) {
                    if (g->iteration < k) {
                        ++g->iteration;
                        stepped += (int64_t)g->members.size();
                    }
                    if (g->iteration < k) {
                        still.push_back(g);
                        continue;
                    }
                    cleora_ctx *c = ctxs[g->slot];
                    for (SReq *q : g->members)
                        CLEORA_HIP(hipMemcpy2DAsync(
                            q->r.out, (size_t)dim * es,
                            c->E[c->cur].as<char>() + (size_t)q->row0 * c->ld * es,
                            (size_t)c->ld * es, (size_t)dim * es, (size_t)q->r.n_nodes,
                            hipMemcpyDefault, main_s));
                    hipEvent_t e = take_event();
                    CLEORA_HIP(hipEventRecord(e, main_s));
                    retiring.emplace_back(e, g);
                }
                active.swap(still);
            } catch (const std::exception &e) {
                // the server stops: every request not yet completed
                // completes now with E_DEVICE (groups still building do so
                // when their builder returns)
                std::lock_guard<std::mutex> lk(mu);
                fatal = e.what();
                for (Group *g : active) {
                    g->status = CLEORA_E_DEVICE;
                    finish(g);
                }
                active.clear();
                for (auto &p : retiring) {
                    ev_pool.push_back(p.first);
                    p.second->status = CLEORA_E_DEVICE;
                    finish(p.second);
                }
                retiring.clear();
                for (Group *g : ready) {
                    g->status = CLEORA_E_DEVICE;
                    finish(g);
                }
                ready.clear();
                const double t = seconds_since(t0);
                for (SReq *q : pending) {
                    q->status = CLEORA_E_DEVICE;
                    q->done_s = t;
                    done.push_back(q);
                }
                policy->drop_front(pending.size());
                pending.clear();
                stop = true;
                cv_build.notify_all();
                cv_done.notify_all();
                return;
            }
        }
    }
};

extern "C" {

int cleora_server_create(cleora_server **out, int device, int32_t dim, int32_t dtype, int32_t k,
                         int32_t slots, int64_t budget_bytes, int32_t builders, int32_t max_group,
                         uint32_t flags)
{
    if (!out) {
        cleora::set_last_error("out is NULL");
        return CLEORA_E_INVAL;
    }
    *out = nullptr;
    if (dim < 1 || (dtype != CLEORA_F32 && dtype != CLEORA_BF16) ||
        dim > (dtype == CLEORA_BF16 ? CLEORA_MAX_DIM_BF16 : CLEORA_MAX_DIM_F32) || k < 0 ||
        slots < 1 || budget_bytes < 0 || builders < 1 || max_group < 1 ||
        (flags & ~(CLEORA_DIRECTED | CLEORA_EMPTY_KEEP))) {
        cleora::set_last_error("bad server parameters");
        return CLEORA_E_INVAL;
    }
    cleora_server *s = new cleora_server();
    s->device = device;
    s->dim = dim;
    s->dtype = dtype;
    s->k = k;
    s->max_group = max_group;
    s->flags = flags;
    s->budget = budget_bytes;
    s->t0 = std::chrono::steady_clock::now();
    int rc = CLEORA_OK;
    for (int32_t i = 0; i < slots && rc == CLEORA_OK; ++i) {
        cleora_ctx *c = nullptr;
        rc = cleora_create(&c, device);
        if (rc == CLEORA_OK) {
            s->ctxs.push_back(c);
        }
    }
    s->staging.resize(s->ctxs.size());
    for (cleora::DevBuf &b : s->staging) b.exact = true;
    if (rc == CLEORA_OK && hipSetDevice(device) != hipSuccess) rc = CLEORA_E_DEVICE;
    if (rc == CLEORA_OK && budget_bytes == 0) {
        // 80% of what is free on the device now
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) rc = CLEORA_E_DEVICE;
        else s->budget = (int64_t)(0.8 * (double)free_b);
        if (rc == CLEORA_OK && s->budget < 1) rc = CLEORA_E_NOMEM;
    }
    if (rc == CLEORA_OK) {
        try {
            s->policy.reset(new cleora::Admission(slots, s->budget, max_group));
            for (int32_t i = 0; i < slots; ++i) {
                cleora_ctx *c = s->ctxs[i];
                cleora::set_exact_growth(c);
                // the step's descriptor table for every slot, at its final
                // size, so that stepping allocates nothing
                c->multi_desc.ensure(sizeof(cleora::StepDesc) * (size_t)slots);
                s->policy->set_idle_held(i, s->slot_bytes(i));
            }
        } catch (const cleora::Error &e) {
            rc = e.code;
        }
    }
    if (rc == CLEORA_OK && hipStreamCreateWithFlags(&s->main_s, hipStreamNonBlocking) != hipSuccess)
        rc = CLEORA_E_DEVICE;
    for (int32_t i = 0; i < builders && rc == CLEORA_OK; ++i) {
        hipStream_t b;
        if (hipStreamCreateWithFlags(&b, hipStreamNonBlocking) != hipSuccess) rc = CLEORA_E_DEVICE;
        else s->bstreams.push_back(b);
    }
    if (rc != CLEORA_OK) {
        for (cleora_ctx *c : s->ctxs) cleora_destroy(c);
        for (hipStream_t b : s->bstreams) (void)hipStreamDestroy(b);
        if (s->main_s) (void)hipStreamDestroy(s->main_s);
        delete s;
        return rc;
    }
    for (int32_t i = 0; i < builders; ++i) s->builders.emplace_back([s, i] { s->build_loop(i); });
    s->sched = std::thread([s] { s->sched_loop(); });
    *out = s;
    return CLEORA_OK;
}

double cleora_server_now(cleora_server *s) { return s ? seconds_since(s->t0) : 0.0; }

int cleora_server_submit(cleora_server *s, const cleora_request *req, int64_t *ticket)
{
    if (!s || !req || !req->out) {
        cleora::set_last_error("NULL argument");
        return CLEORA_E_INVAL;
    }
    if (req->n_nodes < 1 || req->n_nodes > 0x7fffffffLL || req->n_edges < 0 ||
        (req->n_edges > 0 && (!req->src || !req->dst))) {
        cleora::set_last_error("bad request sizes or pointers");
        return CLEORA_E_INVAL;
    }
    const int64_t fp =
        (int64_t)cleora_footprint_bytes(req->n_nodes, req->n_edges, s->flags, s->dim, s->dtype) +
        staging_bytes(req->n_edges);
    if (fp > s->budget) {
        cleora::set_last_error("request footprint exceeds the whole budget");
        return CLEORA_E_INVAL;
    }
    SReq *q = new SReq();
    q->r = *req;
    q->footprint = fp;
    if (req->n_edges > 0) {
        q->on_dev[0] = is_device_ptr(req->src);
        q->on_dev[1] = is_device_ptr(req->dst);
        q->on_dev[2] = is_device_ptr(req->w);
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
        delete q;
        cleora::set_last_error("server stopped: " + s->fatal);
        return CLEORA_E_DEVICE;
    }
    q->ticket = s->next_ticket++;
    q->submit_s = seconds_since(s->t0);
    s->policy->push(fp, req->n_nodes);
    s->pending.push_back(q);
    s->in_system++;
    s->cv_build.notify_one();
    if (ticket) *ticket = q->ticket;
    return CLEORA_OK;
}

int cleora_server_poll(cleora_server *s, cleora_completion *out, int32_t max, int32_t *n_out,
                       double wait_s)
{
    if (!s || !n_out || (max > 0 && !out)) {
        cleora::set_last_error("NULL argument");
        return CLEORA_E_INVAL;
    }
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->done.empty() && wait_s > 0 && !s->stop)
        s->cv_done.wait_for(lk, std::chrono::duration<double>(wait_s));
    int32_t n = 0;
    while (n < max && !s->done.empty()) {
        SReq *q = s->done.front();
        s->done.pop_front();
        out[n].ticket = q->ticket;
        out[n].status = q->status;
        out[n].submit_s = q->submit_s;
        out[n].admit_s = q->admit_s;
        out[n].ready_s = q->ready_s;
        out[n].done_s = q->done_s;
        ++n;
        s->in_system--;
        delete q;
    }
    *n_out = n;
    return CLEORA_OK;
}

int cleora_server_stats(cleora_server *s, int64_t *steps, int64_t *stepped, int32_t *max_active,
                        int64_t *peak_bytes, int64_t *groups, int64_t *in_system)
{
    if (!s) {
        cleora::set_last_error("NULL server");
        return CLEORA_E_INVAL;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (steps) *steps = s->steps;
    if (stepped) *stepped = s->stepped;
    if (max_active) *max_active = s->max_active;
    if (peak_bytes) *peak_bytes = s->policy->peak();
    if (groups) *groups = s->policy->groups();
    if (in_system) *in_system = s->in_system;
    return CLEORA_OK;
}

int cleora_server_memory(cleora_server *s, int64_t *budget, int64_t *charged, int64_t *peak,
                         int64_t *bound_exceeded)
{
    if (!s) {
        cleora::set_last_error("NULL server");
        return CLEORA_E_INVAL;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (budget) *budget = s->policy->budget();
    if (charged) *charged = s->policy->used();
    if (peak) *peak = s->policy->peak();
    if (bound_exceeded) *bound_exceeded = s->bound_exceeded;
    return CLEORA_OK;
}

void cleora_server_destroy(cleora_server *s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_build.notify_all();
    s->cv_sched.notify_all();
    s->cv_done.notify_all();
    if (s->sched.joinable()) s->sched.join();
    for (std::thread &t : s->builders)
        if (t.joinable()) t.join();
    (void)hipSetDevice(s->device);
    if (s->main_s) (void)hipStreamSynchronize(s->main_s);
    for (hipStream_t b : s->bstreams) (void)hipStreamSynchronize(b);
    for (auto &p : s->retiring) (void)hipEventDestroy(p.first);
    for (hipEvent_t e : s->ev_pool) (void)hipEventDestroy(e);
    for (cleora::DevBuf &b : s->staging) b.release();
    for (cleora_ctx *c : s->ctxs) cleora_destroy(c);
    for (hipStream_t b : s->bstreams) (void)hipStreamDestroy(b);
    if (s->main_s) (void)hipStreamDestroy(s->main_s);
    auto drop_reqs = [](std::deque<SReq *> &d) {
        for (SReq *q : d) delete q;
        d.clear();
    };
    auto drop_group = [](Group *g) {
        for (SReq *q : g->members) delete q;
        delete g;
    };
    drop_reqs(s->pending);
    drop_reqs(s->done);
    for (Group *g : s->building) drop_group(g);
    for (Group *g : s->ready) drop_group(g);
    for (Group *g : s->active) drop_group(g);
    for (auto &p : s->retiring) drop_group(p.second);
    delete s;
}

}  // extern "C"
