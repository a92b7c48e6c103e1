// C ABI of the library: contexts, argument checks, launches, errors.
// Every entry point catches everything and returns a CLEORA_* status.
#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include "internal.hpp"

using cleora::DevBuf;
using cleora::Error;
using cleora::StepDesc;

namespace {

thread_local std::string g_last_error;

// autotuner choices: (N, nnz, dim, dtype, split size) -> schedule and its time
struct TuneChoice {
    int32_t pack = 0, persist = 0;
    float ms = -1.0f;
};
std::mutex g_tune_mu;
std::map<std::tuple<int64_t, int64_t, int32_t, int32_t, int32_t>, TuneChoice> g_tune_cache;

// CLEORA_TUNE_CACHE=<path>: choices are read from that text file once per
// process and every new choice is appended to it, one line each:
//   n nnz dim dtype split pack persistent ms
// Caller holds g_tune_mu.
const char *tune_file() { return std::getenv("CLEORA_TUNE_CACHE"); }

void load_tune_file_locked()
{
    static bool loaded = false;
    if (loaded) return;
    loaded = true;
    const char *path = tune_file();
    if (!path || !*path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char line[256];
    while (std::fgets(line, sizeof(line), f)) {
        long long n, nnz;
        int dim, dtype, split, pack, persist;
        float ms;
        if (line[0] == '#' || std::sscanf(line, "%lld %lld %d %d %d %d %d %f", &n, &nnz, &dim,
                                          &dtype, &split, &pack, &persist, &ms) != 8)
            continue;
        if (pack < 16 || pack > (1 << 20) || persist < 0 || persist > 8) continue;
        TuneChoice t;
        t.pack = pack;
        t.persist = persist;
        t.ms = ms;
        g_tune_cache.emplace(std::make_tuple((int64_t)n, (int64_t)nnz, dim, dtype, split), t);
    }
    std::fclose(f);
}

void append_tune_file_locked(const std::tuple<int64_t, int64_t, int32_t, int32_t, int32_t> &k,
                             const TuneChoice &t)
{
    const char *path = tune_file();
    if (!path || !*path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%lld %lld %d %d %d %d %d %.4f\n", (long long)std::get<0>(k),
                 (long long)std::get<1>(k), std::get<2>(k), std::get<3>(k), std::get<4>(k), t.pack,
                 t.persist, t.ms);
    std::fclose(f);
}

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

#define ABI_BEGIN try {
#define ABI_END                                                                 \
    }                                                                           \
    catch (const Error &e) { return fail(e.code, e.what()); }                   \
    catch (const std::bad_alloc &) { return fail(CLEORA_E_NOMEM, "host allocation failed"); } \
    catch (const std::exception &e) { return fail(CLEORA_E_DEVICE, e.what()); } \
    catch (...) { return fail(CLEORA_E_DEVICE, "unknown error"); }

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) CLEORA_HIP(hipSetDevice(dev));
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

int elem_size(int dtype) { return dtype == CLEORA_BF16 ? 2 : 4; }

int32_t padded_ld(int32_t dim, int dtype)
{
    const int epv = 16 / elem_size(dtype);
    return (dim + epv - 1) / epv * epv;
}

// Split size: rows with more entries are split into pieces of this many
// entries (and recombined in order).  The same for every graph, so that a
// graph is summed the same way alone and in any batch; small enough that
// one piece is a short latency chain, large enough that the float32 partial
// rows it writes (d*4 bytes per piece) stay under 1% of the gathered bytes.
// Measured on the 1M-node power-law graph: 512 is fastest for 1 KiB rows
// (FP32, d = 256) and for 512-byte rows (BF16, d = 256: the recombination
// halves against 256, the SpMM is unchanged; 1024 slows the SpMM).
constexpr int32_t DEFAULT_SPLIT = 512;

// Column slices of iterations: requested width in columns (0: whole rows)
// -> width in use.  A bfloat16 width is rounded up to whole 16-byte
// vectors; a slice as wide as the row is whole rows.
int32_t slice_width(int32_t req, int32_t dtype, int32_t ld)
{
    const int32_t epv = dtype == CLEORA_BF16 ? 8 : 4;
    const int32_t w = (req + epv - 1) / epv * epv;
    return w >= ld ? 0 : w;
}

// The width asked for: the set one, or under CLEORA_SLICES_AUTO the
// autotuner's choice for this layout (whole rows until it has measured).
int32_t slice_request(const cleora_ctx *c, int32_t dim, int32_t dtype)
{
    if (c->slice_req != CLEORA_SLICES_AUTO) return c->slice_req;
    return c->slice_auto_dim == dim && c->slice_auto_dtype == dtype ? c->slice_auto : 0;
}

void check_dim(int32_t dim, int32_t dtype)
{
    if (dtype != CLEORA_F32 && dtype != CLEORA_BF16) throw Error(CLEORA_E_INVAL, "unknown dtype");
    const int32_t mx = dtype == CLEORA_BF16 ? CLEORA_MAX_DIM_BF16 : CLEORA_MAX_DIM_F32;
    if (dim < 1 || dim > mx)
        throw Error(CLEORA_E_INVAL, "dim must be in [1, " + std::to_string(mx) + "]");
}

void check_graph_sizes(int64_t n, int64_t m)
{
    if (n < 1 || n > 0x7fffffffLL) throw Error(CLEORA_E_INVAL, "n_nodes must be in [1, 2^31-1]");
    if (m < 0 || m > ((int64_t)1 << 40)) throw Error(CLEORA_E_INVAL, "n_edges out of range");
}

hipEvent_t take_event(cleora_ctx *c)
{
    if (c->ev_next < c->ev_pool.size()) return c->ev_pool[c->ev_next++];
    hipEvent_t e;
    CLEORA_HIP(hipEventCreate(&e));
    c->ev_pool.push_back(e);
    c->ev_next = c->ev_pool.size();
    return e;
}

// One spmm (+ combine) launch of enqueue_steps, with timing events when on.
void launch_step(cleora_ctx *c, const cleora::Variant &v, const StepDesc &d,
                 const StepDesc *dev_desc, hipStream_t s)
{
    hipEvent_t a = nullptr, b = nullptr;
    if (c->timing) {
        a = take_event(c);
        b = take_event(c);
        CLEORA_HIP(hipEventRecord(a, s));
    }
    cleora::launch_spmm(v, d, s);
    if (c->timing) {
        CLEORA_HIP(hipEventRecord(b, s));
        c->ev_spmm.emplace_back(a, b);
    }
    if (c->n_long > 0) {
        if (c->timing) {
            a = take_event(c);
            b = take_event(c);
            CLEORA_HIP(hipEventRecord(a, s));
        }
        cleora::launch_combine(v, dev_desc, 1, c->n_long, s);
        if (c->timing) {
            CLEORA_HIP(hipEventRecord(b, s));
            c->ev_comb.emplace_back(a, b);
        }
    }
}

// k iterations as column slices.  Each slice's SpMM gathers that
// part of the neighbour rows (a narrower gather keeps more of the most-used
// rows in cache), stores its rows unscaled and adds its share of each row's
// squared norm; 1/norm per row follows.  The factors are not applied to
// the rows: the next iteration reads M diag(1/norm) instead of M (one pass
// over the stored values), so T_t = diag(1/norm) U_t is never written
// between iterations.  At the end of the call T_k is written once, out of
// place, into the other buffer; the unscaled rows and their factors stay
// for the next call, which continues from them (deferred = true).
void enqueue_sliced_steps(cleora_ctx *c, int32_t k, int cur, bool deferred, hipStream_t s)
{
    const int64_t n = c->n;
    const int32_t B = c->slice_cols, S = (c->ld + B - 1) / B;
    float *ss = c->slice_norms.as<float>(), *inv = ss + n;
    int in = deferred ? cur ^ 1 : cur;
    for (int32_t t = 0; t < k; ++t) {
        const bool unscaled_in = t > 0 || deferred;
        if (unscaled_in)
            cleora::launch_scale_values(c->val.as<float>(), c->col.as<int32_t>(), inv, c->nnz,
                                        c->val2.as<float>(), s);
        cleora::launch_fill_zero(ss, n, s);
        for (int32_t j = 0; j < S; ++j) {
            const int32_t c0 = j * B;
            const cleora::Variant v = cleora::choose_variant(c->dtype, std::min(B, c->ld - c0));
            StepDesc d = cleora::slice_desc(c, in, c0);
            if (unscaled_in) d.val = c->val2.as<float>();
            launch_step(c, v, d, c->slice_desc.as<StepDesc>() + (size_t)in * S + j, s);
        }
        cleora::launch_inv_norm(ss, inv, n, s);
        in ^= 1;
    }
    cleora::launch_scale_rows_to(c->dtype, c->E[in].p, c->E[in ^ 1].p, n, c->ld, inv, s);
}

// Queue k iterations starting from buffer parity `cur` (no state change).
void enqueue_steps(cleora_ctx *c, int32_t k, int cur, bool deferred, hipStream_t s)
{
    if (c->slice_cols > 0) return enqueue_sliced_steps(c, k, cur, deferred, s);
    const cleora::Variant v = cleora::choose_variant(c->dtype, c->ld);
    for (int32_t t = 0; t < k; ++t) {
        launch_step(c, v, cleora::host_desc(c, cur), c->desc.as<StepDesc>() + cur, s);
        cur ^= 1;
    }
}

// CLEORA_SLICES_AUTO: time one whole-row iteration (the schedule in use)
// against one steady-state iteration in slices of 1 KiB and of 512 bytes
// (values of M diag(1/norm), the slices' SpMM and combines, 1/norm), each
// plus the final out-of-place scaling spread over the iterations of the
// context's last propagate call (4 if none yet), on this embedding; the
// fastest slicing is kept only if at least 1% faster than whole rows.
// The trials read E[cur] and write only the other buffer and the slices'
// scratch (their values are not used), so the embedding stays as it was.
void choose_slices(cleora_ctx *c, hipStream_t s)
{
    const int32_t esz = (int32_t)elem_size(c->dtype);
    int32_t chosen = 0;
    std::vector<int32_t> widths;
    for (int32_t bytes : {1024, 512}) {
        const int32_t W = slice_width(bytes / esz, c->dtype, c->ld);
        if (W > 0) widths.push_back(W);
    }
    if (!widths.empty() && c->n > 0) {
        hipEvent_t a = nullptr, b = nullptr;
        auto timed = [&](int reps, const std::function<void()> &f) {
            f();  // warm-up
            CLEORA_HIP(hipEventRecord(a, s));
            for (int r = 0; r < reps; ++r) f();
            CLEORA_HIP(hipEventRecord(b, s));
            CLEORA_HIP(hipEventSynchronize(b));
            float ms = 0;
            CLEORA_HIP(hipEventElapsedTime(&ms, a, b));
            return ms / (float)reps;
        };
        const bool timing = c->timing;
        c->timing = false;
        try {
            CLEORA_HIP(hipEventCreate(&a));
            CLEORA_HIP(hipEventCreate(&b));
            const int cur = c->cur;
            const int32_t per_call = c->last_k > 0 ? c->last_k : 4;
            c->slice_cols = 0;
            cleora::plan_schedule(c, s);
            c->partial.ensure(sizeof(float) * (size_t)std::max<int64_t>(c->n_split, 1) *
                              (size_t)c->ld);
            cleora::write_descs(c, s);
            const cleora::Variant vw = cleora::choose_variant(c->dtype, c->ld);
            const float whole = timed(2, [&]() {
                launch_step(c, vw, cleora::host_desc(c, cur), c->desc.as<StepDesc>() + cur, s);
            });
            float best = 0.99f * whole;
            for (int32_t W : widths) {
                c->slice_cols = W;
                cleora::write_descs(c, s);
                const int32_t S = (c->ld + W - 1) / W;
                float *ss = c->slice_norms.as<float>(), *inv = ss + c->n;
                cleora::launch_fill_zero(inv, c->n, s);
                const float sliced = timed(2, [&]() {
                    cleora::launch_scale_values(c->val.as<float>(), c->col.as<int32_t>(), inv,
                                                c->nnz, c->val2.as<float>(), s);
                    cleora::launch_fill_zero(ss, c->n, s);
                    for (int32_t j = 0; j < S; ++j) {
                        const int32_t c0 = j * W;
                        const cleora::Variant v =
                            cleora::choose_variant(c->dtype, std::min(W, c->ld - c0));
                        StepDesc d = cleora::slice_desc(c, cur, c0);
                        d.val = c->val2.as<float>();
                        launch_step(c, v, d, c->slice_desc.as<StepDesc>() + (size_t)cur * S + j,
                                    s);
                    }
                    cleora::launch_inv_norm(ss, inv, c->n, s);
                });
                const float final_scale = timed(1, [&]() {
                    cleora::launch_scale_rows_to(c->dtype, c->E[cur].p, c->E[cur ^ 1].p, c->n,
                                                 c->ld, inv, s);
                });
                const float per_it = sliced + final_scale / (float)per_call;
                if (per_it < best) {
                    best = per_it;
                    chosen = W;
                }
                if (std::getenv("CLEORA_TUNE_VERBOSE"))
                    std::fprintf(stderr,
                                 "[cleora autotune] n=%lld d=%d: whole rows %.4f ms, %d-column "
                                 "slices %.4f + final scaling %.4f / %d ms\n",
                                 (long long)c->n, c->dim, whole, W, sliced, final_scale, per_call);
            }
            if (std::getenv("CLEORA_TUNE_VERBOSE"))
                std::fprintf(stderr, "[cleora autotune] n=%lld d=%d: slice width %d kept\n",
                             (long long)c->n, c->dim, chosen);
        } catch (...) {
            c->timing = timing;
            c->slice_cols = 0;
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
            throw;
        }
        c->timing = timing;
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
    }
    c->slice_auto = chosen;
    c->slice_auto_dim = c->dim;
    c->slice_auto_dtype = c->dtype;
    c->slice_cols = chosen;
}

// Release a captured loop after its last replay has finished.
void free_loop(cleora::LoopGraph &L)
{
    if (L.done && L.launched) (void)hipEventSynchronize(L.done);
    if (L.exec) (void)hipGraphExecDestroy(L.exec);
    if (L.done) (void)hipEventDestroy(L.done);
    L = cleora::LoopGraph{};
}

void drop_graphs(cleora_ctx *c)
{
    for (auto &kv : c->graphs) free_loop(kv.second);
    c->graphs.clear();
}

// Everything a captured k-iteration loop depends on: kernel arguments of
// both parities (buffers, schedule sizes, layout, flags, grid choice), the
// device descriptor tables and the slicing.  Equal signatures mean
// the captured launches are exactly the ones enqueue_steps would queue now.
std::vector<int64_t> loop_signature(const cleora_ctx *c, int32_t k, int cur)
{
    std::vector<int64_t> g;
    auto P = [&](const void *p) { g.push_back((int64_t)reinterpret_cast<uintptr_t>(p)); };
    g.insert(g.end(), {k, cur, c->deferred ? 1 : 0, c->dtype, c->ld, c->slice_cols, c->n,
                       c->nnz, c->n_long});
    P(c->desc.p);
    P(c->slice_desc.p);
    P(c->slice_norms.p);
    P(c->val2.p);
    for (int p = 0; p < 2; ++p) {
        const StepDesc d = cleora::host_desc(c, p);
        P(d.rp);
        P(d.col);
        P(d.val);
        P(d.Ein);
        P(d.Eout);
        P(d.partial);
        P(d.split_items);
        P(d.bucket_row);
        P(d.long_rows);
        P(d.chunk_base);
        g.insert(g.end(), {d.n_split, d.n_buckets, d.n_long, d.ld, d.chunk, (int64_t)d.flags,
                           d.persist});
    }
    return g;
}

// The captured loop of k iterations from the current parity, captured (and
// instantiated) only when no loop with the current launch parameters
// exists.
cleora::LoopGraph &loop_graph(cleora_ctx *c, int32_t k)
{
    cleora::LoopGraph &L = c->graphs[std::make_tuple(k, c->cur, c->deferred)];
    std::vector<int64_t> sig = loop_signature(c, k, c->cur);
    if (L.exec && L.sig == sig) return L;
    free_loop(L);
    if (!c->cap_stream) CLEORA_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    try {
        CLEORA_HIP(hipEventCreateWithFlags(&L.done, hipEventDisableTiming));
        CLEORA_HIP(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        try {
            enqueue_steps(c, k, c->cur, c->deferred, c->cap_stream);
        } catch (...) {
            (void)hipStreamEndCapture(c->cap_stream, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        CLEORA_HIP(hipStreamEndCapture(c->cap_stream, &g));
        const hipError_t e = hipGraphInstantiate(&L.exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        CLEORA_HIP(e);
    } catch (...) {
        free_loop(L);
        throw;
    }
    L.sig = std::move(sig);
    c->graph_instantiations++;
    return L;
}

// k >= 2 iterations without timing run as one captured graph (cached per
// k and starting parity, and reused while its launch parameters hold): the
// 2k launches cost one graph launch.  With timing on, launches are eager,
// each between two events (events recorded inside a graph carry no time).
void run_steps(cleora_ctx *c, int32_t k, hipStream_t s)
{
    if (k <= 0) return;
    if (k >= 2 && !c->timing) {
        cleora::LoopGraph &L = loop_graph(c, k);
        CLEORA_HIP(hipGraphLaunch(L.exec, s));
        CLEORA_HIP(hipEventRecord(L.done, s));
        L.launched = true;
        c->graph_launches++;
    } else {
        enqueue_steps(c, k, c->cur, c->deferred, s);
    }
    if (c->slice_cols > 0) {
        // the last unscaled rows are in the buffer the k iterations ended
        // in; T_k was written into the other one
        const int in0 = c->deferred ? c->cur ^ 1 : c->cur;
        c->cur = in0 ^ (k & 1) ^ 1;
        c->deferred = true;
    } else {
        c->cur ^= (k & 1);
    }
    c->iteration += k;
}

int device_cus(int device)
{
    static std::atomic<int> cached[64] = {};
    if (device >= 0 && device < 64 && cached[device].load() > 0) return cached[device].load();
    int cus = 0;
    CLEORA_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
    if (device >= 0 && device < 64) cached[device].store(cus);
    return cus;
}

// The two embedding buffers for n rows (the schedule comes later).
void alloc_embedding(cleora_ctx *c, int64_t n, int32_t dim, int32_t dtype)
{
    c->has_emb = false;
    c->dim = dim;
    c->dtype = dtype;
    c->ld = padded_ld(dim, dtype);
    c->chunk = c->chunk_req > 0 ? c->chunk_req : DEFAULT_SPLIT;
    c->deferred = false;
    c->slice_cols = slice_width(slice_request(c, dim, dtype), dtype, c->ld);
    const size_t ebytes = (size_t)n * (size_t)c->ld * elem_size(dtype);
    c->E[0].ensure(ebytes);
    c->E[1].ensure(ebytes);
}

// The propagation schedule of the current graph and embedding layout.
void plan_embedding(cleora_ctx *c, hipStream_t s)
{
    cleora::plan_schedule(c, s);
    c->partial.ensure(sizeof(float) * (size_t)std::max<int64_t>(c->n_split, 1) * (size_t)c->ld);
    cleora::write_descs(c, s);
    c->cur = 0;
    c->iteration = 0;
}

void setup_embedding(cleora_ctx *c, int32_t dim, int32_t dtype, hipStream_t s)
{
    alloc_embedding(c, c->n, dim, dtype);
    plan_embedding(c, s);
}

// Build the CSR on s while T_0 is written on the context's side stream:
// T_0 needs only N, d and the seed, so the ALU-bound init overlaps the
// memory-bound build.  s waits for the init before the call returns (also
// when the build fails, so that E is not released under it).
void build_overlapping_init(cleora_ctx *c, int64_t n, int32_t dim, int32_t dtype, hipStream_t s,
                            const std::function<void()> &build,
                            const std::function<void(hipStream_t)> &init)
{
    alloc_embedding(c, n, dim, dtype);
    if (!c->side_stream) {
        CLEORA_HIP(hipStreamCreateWithFlags(&c->side_stream, hipStreamNonBlocking));
        CLEORA_HIP(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
        CLEORA_HIP(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
    }
    // earlier work on s may still read E
    CLEORA_HIP(hipEventRecord(c->ev_fork, s));
    CLEORA_HIP(hipStreamWaitEvent(c->side_stream, c->ev_fork, 0));
    init(c->side_stream);
    CLEORA_HIP(hipEventRecord(c->ev_join, c->side_stream));
    try {
        build();
        plan_embedding(c, s);
    } catch (...) {
        (void)hipStreamWaitEvent(s, c->ev_join, 0);
        throw;
    }
    CLEORA_HIP(hipStreamWaitEvent(s, c->ev_join, 0));
    c->has_emb = true;
}

__global__ void k_offset_edges(int64_t m, const int32_t *__restrict__ src,
                               const int32_t *__restrict__ dst, const float *__restrict__ w,
                               int64_t n_g, int64_t node_off, int32_t *__restrict__ osrc,
                               int32_t *__restrict__ odst, float *__restrict__ ow)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = src[e], b = dst[e];
        // an id outside its own graph stays invalid in the concatenation
        osrc[e] = (a >= 0 && a < n_g) ? (int32_t)(a + node_off) : -1;
        odst[e] = (b >= 0 && b < n_g) ? (int32_t)(b + node_off) : -1;
        if (ow) ow[e] = w ? w[e] : 1.0f;
    }
}

}  // namespace

namespace cleora {
int32_t tuned_pack(const cleora_ctx *c)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_file_locked();
    auto it = g_tune_cache.find(std::make_tuple(c->n, c->nnz, c->dim, c->dtype, c->chunk));
    return it == g_tune_cache.end() ? 0 : it->second.pack;
}

std::vector<DevBuf *> ctx_buffers(cleora_ctx *c)
{
    return {&c->rp,         &c->col,        &c->val,         &c->deg,        &c->E[0],
            &c->E[1],       &c->split_items, &c->bucket_row, &c->long_rows,  &c->chunk_base,
            &c->partial,    &c->desc,       &c->blk_norms,   &c->chunk_ids,  &c->chunk_occ,
            &c->t_local,    &c->t_expand,   &c->t_edges,     &c->t_wts,      &c->t_cnt,
            &c->t_off,      &c->t_keys,     &c->t_tmp,       &c->t_head,     &c->t_pos,
            &c->t_esum,     &c->t_lists,    &c->t_scan,      &c->t_small,    &c->multi_desc,
            &c->slice_desc, &c->slice_norms, &c->val2};
}

int64_t ctx_device_bytes(cleora_ctx *c)
{
    int64_t b = 0;
    for (DevBuf *d : ctx_buffers(c)) b += (int64_t)d->cap;
    return b;
}

void set_exact_growth(cleora_ctx *c)
{
    for (DevBuf *d : ctx_buffers(c)) d->exact = true;
}

void release_buffers(cleora_ctx *c)
{
    DeviceGuard g(c->device);
    drop_graphs(c);
    for (DevBuf *d : ctx_buffers(c))
        if (d != &c->t_small) d->release();  // t_small: the build's status words
    c->has_graph = false;
    c->has_emb = false;
    c->is_chunk = false;
}

int32_t tuned_persist(const cleora_ctx *c)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_file_locked();
    auto it = g_tune_cache.find(std::make_tuple(c->n, c->nnz, c->dim, c->dtype, c->chunk));
    return it == g_tune_cache.end() ? 0 : it->second.persist;
}
}  // namespace cleora

namespace cleora {

// One iteration for each context in one set of launches; synchronises s.
void step_contexts(cleora_ctx *const *ctxs, int32_t n, hipStream_t s)
{
    cleora_ctx *c0 = ctxs[0];
    std::vector<StepDesc> tab((size_t)n);
    int64_t waves = 0, blocks = 0;
    for (int32_t i = 0; i < n; ++i) {
        tab[i] = host_desc(ctxs[i], ctxs[i]->cur);
        tab[i].wave_begin = waves;
        tab[i].block_begin = blocks;
        waves += ctxs[i]->n_split + ctxs[i]->n_buckets;
        blocks += ctxs[i]->n_long;
    }
    c0->multi_desc.ensure(sizeof(StepDesc) * tab.size());
    CLEORA_HIP(hipMemcpyAsync(c0->multi_desc.p, tab.data(), sizeof(StepDesc) * tab.size(),
                              hipMemcpyHostToDevice, s));
    const Variant v = choose_variant(c0->dtype, c0->ld);
    const StepDesc *d = c0->multi_desc.as<StepDesc>();
    launch_spmm_multi(v, d, n, waves, c0->persist, s);
    if (blocks > 0) launch_combine(v, d, n, blocks, s);
    for (int32_t i = 0; i < n; ++i) {
        // a whole-row step from the normalised rows (the other buffer, which
        // held a sliced context's unscaled rows, now holds the result)
        ctxs[i]->cur ^= 1;
        ctxs[i]->deferred = false;
        ctxs[i]->iteration++;
    }
    // the descriptor table is host memory read by the copy above
    CLEORA_HIP(hipStreamSynchronize(s));
}

void set_last_error(const std::string &msg) { g_last_error = msg; }

void check_rows_args(int64_t n_rows, int64_t n_cols, int64_t m, const int32_t *rows,
                     const int32_t *cols, const void *T_in, int64_t ld_in, int32_t dim,
                     int32_t dtype, const void *out, int64_t ld_out)
{
    if (!T_in || !out) throw Error(CLEORA_E_INVAL, "NULL argument");
    check_graph_sizes(n_rows, m);
    check_graph_sizes(n_cols, 0);
    if (m > 0 && (!rows || !cols)) throw Error(CLEORA_E_INVAL, "rows/cols is NULL");
    check_dim(dim, dtype);
    if (ld_in != padded_ld(dim, dtype))
        throw Error(CLEORA_E_INVAL, "ld_in must be dim rounded up to a multiple of 16 bytes");
    if (ld_out < dim) throw Error(CLEORA_E_INVAL, "ld_out < dim");
    if ((reinterpret_cast<uintptr_t>(T_in) & 15) != 0)
        throw Error(CLEORA_E_INVAL, "T_in must be 16-byte aligned");
}

void propagate_rows_into(cleora_ctx *c, int64_t n_rows, int64_t n_cols, int64_t m,
                         const int32_t *rows, const int32_t *cols, const float *w,
                         const void *T_in, int32_t dim, int32_t dtype, void *out, int64_t ld_out,
                         hipStream_t s)
{
    c->is_chunk = false;
    build_graph(c, n_rows, n_cols, m, rows, cols, w, CLEORA_DIRECTED, s);
    c->dim = dim;
    c->dtype = dtype;
    c->ld = padded_ld(dim, dtype);
    c->chunk = c->chunk_req > 0 ? c->chunk_req : DEFAULT_SPLIT;
    const size_t ebytes = (size_t)n_rows * (size_t)c->ld * elem_size(dtype);
    c->E[1].ensure(ebytes);
    plan_schedule(c, s);
    c->partial.ensure(sizeof(float) * (size_t)std::max<int64_t>(c->n_split, 1) * (size_t)c->ld);
    StepDesc d = host_desc(c, 0);
    d.Ein = T_in;
    d.Eout = c->E[1].p;
    c->desc.ensure(sizeof(StepDesc) * 2);
    CLEORA_HIP(hipMemcpyAsync(c->desc.p, &d, sizeof(d), hipMemcpyHostToDevice, s));
    const Variant v = choose_variant(dtype, c->ld);
    launch_spmm(v, d, s);
    if (c->n_long > 0) launch_combine(v, c->desc.as<StepDesc>(), 1, c->n_long, s);
    const size_t es = elem_size(dtype);
    CLEORA_HIP(hipMemcpy2DAsync(out, (size_t)ld_out * es, c->E[1].p, (size_t)c->ld * es,
                                (size_t)dim * es, (size_t)n_rows, hipMemcpyDefault, s));
    // the descriptor above lives on this stack frame
    CLEORA_HIP(hipStreamSynchronize(s));
    c->has_emb = false;  // the scratch context holds no propagatable embedding
}

namespace {
// Concatenated per-graph edges -> block-diagonal ids, in place: edge e of
// graph g (edges [eoff[g], eoff[g+1])) gets node offset row0[g]; an id
// outside [0, n_g) becomes -1, which the build reports.
__global__ void k_offset_edges_table(int64_t m, int32_t *__restrict__ src,
                                     int32_t *__restrict__ dst,
                                     const int64_t *__restrict__ eoff,
                                     const int64_t *__restrict__ row0, int n_graphs)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        int lo = 0, hi = n_graphs - 1;  // last g with eoff[g] <= e
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (eoff[mid] <= e) lo = mid;
            else hi = mid - 1;
        }
        const int64_t n_g = row0[lo + 1] - row0[lo];
        const int32_t a = src[e], b = dst[e];
        src[e] = (a >= 0 && a < n_g) ? (int32_t)(a + row0[lo]) : -1;
        dst[e] = (b >= 0 && b < n_g) ? (int32_t)(b + row0[lo]) : -1;
    }
}
}  // namespace

void build_group_and_init(cleora_ctx *c, int32_t n_graphs, int64_t n_total, int64_t m_total,
                          int32_t *src, int32_t *dst, const float *w, const int64_t *d_row0,
                          const int64_t *d_eoff, const uint64_t *d_seeds, uint32_t flags,
                          int32_t dim, int32_t dtype, hipStream_t s)
{
    check_graph_sizes(n_total, m_total);
    check_dim(dim, dtype);
    c->is_chunk = false;
    if (m_total > 0) {
        const unsigned blocks = (unsigned)std::min<int64_t>(ceil_div(m_total, 256), 65536);
        k_offset_edges_table<<<blocks, 256, 0, s>>>(m_total, src, dst, d_eoff, d_row0, n_graphs);
        CLEORA_LAUNCH_CHECK();
    }
    build_graph(c, n_total, n_total, m_total, src, dst, w, flags, s);
    setup_embedding(c, dim, dtype, s);
    launch_init(dtype, c->E[0].p, n_total, dim, c->ld, d_row0, d_seeds, n_graphs, 0, s);
    c->has_emb = true;
}

}  // namespace cleora

extern "C" {

const char *cleora_last_error(void) { return g_last_error.c_str(); }

int cleora_create(cleora_ctx **out, int device)
{
    ABI_BEGIN
    if (!out) return fail(CLEORA_E_INVAL, "out is NULL");
    *out = nullptr;
    int count = 0;
    CLEORA_HIP(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return fail(CLEORA_E_DEVICE, "no such device");
    DeviceGuard g(device);
    cleora_ctx *c = new cleora_ctx();
    c->device = device;
    if (hipHostMalloc(reinterpret_cast<void **>(&c->h_small), 8 * sizeof(int64_t),
                      hipHostMallocDefault) != hipSuccess) {
        delete c;
        return fail(CLEORA_E_NOMEM, "pinned host allocation failed");
    }
    try {
        c->t_small.ensure(8 * sizeof(int64_t));
    } catch (...) {
        (void)hipHostFree(c->h_small);
        delete c;
        throw;
    }
    *out = c;
    return CLEORA_OK;
    ABI_END
}

void cleora_destroy(cleora_ctx *c)
{
    if (!c) return;
    try {
        DeviceGuard g(c->device);
        (void)hipDeviceSynchronize();
        drop_graphs(c);
        if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
        if (c->side_stream) (void)hipStreamDestroy(c->side_stream);
        if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
        if (c->ev_join) (void)hipEventDestroy(c->ev_join);
        for (DevBuf *b : cleora::ctx_buffers(c)) b->release();
        for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
        if (c->h_small) (void)hipHostFree(c->h_small);
    } catch (...) {
    }
    delete c;
}

size_t cleora_footprint_bytes(int64_t n, int64_t m, uint32_t flags, int32_t dim, int32_t dtype)
{
    if (n < 1 || m < 0 || dim < 1 || (dtype != CLEORA_F32 && dtype != CLEORA_BF16)) return 0;
    const double t = (flags & CLEORA_DIRECTED) ? (double)m : 2.0 * (double)m;
    const int32_t ld = padded_ld(dim, dtype);
    const double N = (double)n;
    const double S = DEFAULT_SPLIT, P = 16;  // split size; smallest packing size
    double b = 0;
    b += 8 * N + 8 * (N + 1) + 8 * t + 8 * t + t + 8 * (t + 1) + 8 * t + 8 * N;  // build
    b += 8 * t;                                                                // weights
    b += 8 * 16.0 * ceil(std::max(t, N) / 4096.0);                             // scan
    b += 8 * (N + 1) + 4 * t + 4 * t + 8 * N;                                  // CSR + D
    b += 2.0 * N * ld * elem_size(dtype);                                      // T ping-pong
    const double split = 2.0 * t / S + 1;
    b += 8 * (N + 1) + split * (4.0 * ld + 8) + 4 * ((t + N) / P + 2) + 4 * N;  // schedule
    b += 1 << 20;                                                               // slack
    return (size_t)b;
}

int cleora_build_csr(cleora_ctx *c, int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                     const float *w, uint32_t flags, void *stream)
{
    ABI_BEGIN
    cleora::TraceRange trace_range("cleora_build_csr");
    if (!c) return fail(CLEORA_E_INVAL, "ctx is NULL");
    check_graph_sizes(n, m);
    if (m > 0 && (!src || !dst)) return fail(CLEORA_E_INVAL, "src/dst is NULL");
    if (flags & ~(CLEORA_DIRECTED | CLEORA_EMPTY_KEEP)) return fail(CLEORA_E_INVAL, "unknown flag");
    DeviceGuard g(c->device);
    c->is_chunk = false;
    cleora::build_graph(c, n, n, m, src, dst, w, flags, cleora::as_stream(stream));
    return CLEORA_OK;
    ABI_END
}

int cleora_init(cleora_ctx *c, int32_t dim, int32_t dtype, uint64_t seed, void *stream)
{
    ABI_BEGIN
    cleora::TraceRange trace_range("cleora_init");
    if (!c) return fail(CLEORA_E_INVAL, "ctx is NULL");
    if (!c->has_graph) return fail(CLEORA_E_STATE, "no graph: call cleora_build_csr first");
    check_dim(dim, dtype);
    DeviceGuard g(c->device);
    hipStream_t s = cleora::as_stream(stream);
    setup_embedding(c, dim, dtype, s);
    cleora::launch_init(dtype, c->E[0].p, c->n, dim, c->ld, nullptr, nullptr, 1, seed, s,
                        c->is_chunk ? c->chunk_ids.as<int32_t>() : nullptr);
    c->has_emb = true;
    return CLEORA_OK;
    ABI_END
}

int cleora_build_init(cleora_ctx *c, int64_t n_nodes, int64_t n_edges, const int32_t *src,
                      const int32_t *dst, const float *w, uint32_t flags, int32_t dim,
                      int32_t dtype, uint64_t seed, void *stream)
{
    ABI_BEGIN
    cleora::TraceRange trace_range("cleora_build_init");
    if (!c) return fail(CLEORA_E_INVAL, "ctx is NULL");
    check_graph_sizes(n_nodes, n_edges);
    if (n_edges > 0 && (!src || !dst)) return fail(CLEORA_E_INVAL, "src/dst NULL");
    if (flags & ~(CLEORA_DIRECTED | CLEORA_EMPTY_KEEP)) return fail(CLEORA_E_INVAL, "bad flags");
    check_dim(dim, dtype);
    DeviceGuard g(c->device);
    hipStream_t s = cleora::as_stream(stream);
    c->is_chunk = false;
    build_overlapping_init(
        c, n_nodes, dim, dtype, s,
        [&] { cleora::build_graph(c, n_nodes, n_nodes, n_edges, src, dst, w, flags, s); },
        [&](hipStream_t side) {
            // two blocks per CU: the init shares the CUs with the build
            cleora::launch_init(dtype, c->E[0].p, n_nodes, dim, c->ld, nullptr, nullptr, 1, seed,
                                side, nullptr, 2 * (int64_t)device_cus(c->device));
        });
    return CLEORA_OK;
    ABI_END
}

int cleora_propagate(cleora_ctx *c, int32_t k, void *stream)
{
    ABI_BEGIN
    cleora::TraceRange trace_range("cleora_propagate");
    if (!c) return fail(CLEORA_E_INVAL, "ctx is NULL");
    if (k < 0) return fail(CLEORA_E_INVAL, "k must be >= 0");
    if (!c->has_emb) return fail(CLEORA_E_STATE, "no embedding: call cleora_init first");
    DeviceGuard g(c->device);
    run_steps(c, k, cleora::as_stream(stream));
    if (k > 0) c->last_k = k;
    return CLEORA_OK;
    ABI_END
}

int cleora_embed_blocked(cleora_ctx *c, int32_t dim, int32_t block, int32_t dtype, uint64_t seed,
                         int32_t k, void *out, int64_t ld_out, void *stream)
{
    ABI_BEGIN
    cleora::TraceRange trace_range("cleora_embed_blocked");
    if (!c || !out) return fail(CLEORA_E_INVAL, "NULL argument");
    if (!c->has_graph) return fail(CLEORA_E_STATE, "no graph: call cleora_build_csr first");
    check_dim(dim, dtype);
    if (block < 1) return fail(CLEORA_E_INVAL, "block must be >= 1");
    if (k < 0) return fail(CLEORA_E_INVAL, "k must be >= 0");
    if (ld_out < dim) return fail(CLEORA_E_INVAL, "ld_out < dim");
    DeviceGuard g(c->device);
    hipStream_t s = cleora::as_stream(stream);
    const int32_t bw = std::min(block, dim);
    // block buffers and the schedule for the widest block; no embedding
    // remains afterwards
    alloc_embedding(c, c->n, bw, dtype);
    c->slice_cols = 0;  // blocks are propagated whole
    plan_embedding(c, s);
    cleora::embed_blocked(c, dim, bw, dtype, seed, k, out, ld_out, s);
    return CLEORA_OK;
    ABI_END
}

int cleora_release_scratch(cleora_ctx *c)
{
    ABI_BEGIN
    cleora::TraceRange trace_range("cleora_release_scratch");
    if (!c) return fail(CLEORA_E_INVAL, "ctx is NULL");
    DeviceGuard g(c->device);
    CLEORA_HIP(hipDeviceSynchronize());  // nothing in flight may still use them
    // every user of these ensures them again before use (t_small stays: it
    // carries the build's status words and is allocated at creation)
    DevBuf *tmp[] = {&c->t_edges, &c->t_wts,  &c->t_cnt,   &c->t_off,   &c->t_keys,
                     &c->t_tmp,   &c->t_head, &c->t_pos,   &c->t_esum,  &c->t_lists,
                     &c->t_scan,  &c->t_local, &c->t_expand, &c->multi_desc};
    for (DevBuf *b : tmp) b->release();
    if (!c->has_emb) {
        drop_graphs(c);  // captured iterations point at the buffers below
        DevBuf *emb[] = {&c->E[0],      &c->E[1],       &c->split_items, &c->bucket_row,
                         &c->long_rows, &c->chunk_base, &c->partial,     &c->desc,
                         &c->blk_norms, &c->slice_desc, &c->slice_norms, &c->val2};
        for (DevBuf *b : emb) b->release();
    }
    return CLEORA_OK;
    ABI_END
}

int cleora_get_embedding(cleora_ctx *c, void *dst, int64_t ld, int32_t dst_dtype, void *stream)
{
    ABI_BEGIN
    cleora::TraceRange trace_range("cleora_get_embedding");
    if (!c || !dst) return fail(CLEORA_E_INVAL, "NULL argument");
    if (!c->has_emb) return fail(CLEORA_E_STATE, "no embedding");
    if (ld < c->dim) return fail(CLEORA_E_INVAL, "ld < dim");
    DeviceGuard g(c->device);
    hipStream_t s = cleora::as_stream(stream);
    if (dst_dtype == c->dtype) {
        const size_t es = elem_size(c->dtype);
        CLEORA_HIP(hipMemcpy2DAsync(dst, (size_t)ld * es, c->E[c->cur].p, (size_t)c->ld * es,
                                    (size_t)c->dim * es, (size_t)c->n, hipMemcpyDefault, s));
    } else if (c->dtype == CLEORA_BF16 && dst_dtype == CLEORA_F32) {
        cleora::launch_widen_bf16(c->E[c->cur].p, c->n, c->dim, c->ld,
                                  reinterpret_cast<float *>(dst), ld, s);
    } else {
        return fail(CLEORA_E_INVAL, "unsupported dst_dtype for this context");
    }
    return CLEORA_OK;
    ABI_END
}

int cleora_embedding_ptr(cleora_ctx *c, const void **ptr, int64_t *ld)
{
    ABI_BEGIN
    if (!c || !ptr) return fail(CLEORA_E_INVAL, "NULL argument");
    if (!c->has_emb) return fail(CLEORA_E_STATE, "no embedding");
    *ptr = c->E[c->cur].p;
    if (ld) *ld = c->ld;
    return CLEORA_OK;
    ABI_END
}

int cleora_previous_embedding_ptr(cleora_ctx *c, const void **ptr, int64_t *ld)
{
    ABI_BEGIN
    if (!c || !ptr) return fail(CLEORA_E_INVAL, "NULL argument");
    if (!c->has_emb || c->iteration < 1)
        return fail(CLEORA_E_STATE, "no previous iteration (propagate at least once)");
    if (c->deferred)
        return fail(CLEORA_E_STATE,
                    "column-sliced iterations keep T_t's unscaled rows, not T_{t-1} "
                    "(cleora_set_slices(ctx, 0) before cleora_init keeps whole rows)");
    *ptr = c->E[c->cur ^ 1].p;
    if (ld) *ld = c->ld;
    return CLEORA_OK;
    ABI_END
}

int cleora_propagate_rows(cleora_ctx *c, int64_t n_rows, int64_t n_cols, int64_t m,
                          const int32_t *rows, const int32_t *cols, const float *w,
                          const void *T_in, int64_t ld_in, int32_t dim, int32_t dtype, void *out,
                          int64_t ld_out, void *stream)
{
    ABI_BEGIN
    cleora::TraceRange trace_range("cleora_propagate_rows");
    if (!c) return fail(CLEORA_E_INVAL, "NULL argument");
    cleora::check_rows_args(n_rows, n_cols, m, rows, cols, T_in, ld_in, dim, dtype, out, ld_out);
    DeviceGuard g(c->device);
    cleora::propagate_rows_into(c, n_rows, n_cols, m, rows, cols, w, T_in, dim, dtype, out,
                                ld_out, cleora::as_stream(stream));
    return CLEORA_OK;
    ABI_END
}

int cleora_get_csr(cleora_ctx *c, int64_t *row_ptr, int32_t *col, float *val, double *deg,
                   void *stream)
{
    ABI_BEGIN
    if (!c) return fail(CLEORA_E_INVAL, "ctx is NULL");
    if (!c->has_graph) return fail(CLEORA_E_STATE, "no graph");
    DeviceGuard g(c->device);
    hipStream_t s = cleora::as_stream(stream);
    if (row_ptr)
        CLEORA_HIP(hipMemcpyAsync(row_ptr, c->rp.p, sizeof(int64_t) * (c->n + 1), hipMemcpyDefault, s));
    if (col && c->nnz)
        CLEORA_HIP(hipMemcpyAsync(col, c->col.p, sizeof(int32_t) * c->nnz, hipMemcpyDefault, s));
    if (val && c->nnz)
        CLEORA_HIP(hipMemcpyAsync(val, c->val.p, sizeof(float) * c->nnz, hipMemcpyDefault, s));
    if (deg) CLEORA_HIP(hipMemcpyAsync(deg, c->deg.p, sizeof(double) * c->n, hipMemcpyDefault, s));
    return CLEORA_OK;
    ABI_END
}

int cleora_info(cleora_ctx *c, int64_t *n, int64_t *nnz, int32_t *dim, int32_t *dtype,
                int32_t *iteration)
{
    ABI_BEGIN
    if (!c) return fail(CLEORA_E_INVAL, "ctx is NULL");
    if (n) *n = c->has_graph ? c->n : 0;
    if (nnz) *nnz = c->has_graph ? c->nnz : 0;
    if (dim) *dim = c->has_emb ? c->dim : 0;
    if (dtype) *dtype = c->dtype;
    if (iteration) *iteration = c->has_emb ? c->iteration : 0;
    return CLEORA_OK;
    ABI_END
}

int cleora_schedule_info(cleora_ctx *c, int32_t *chunk, int64_t *n_split, int64_t *n_long,
                         int64_t *n_buckets, int32_t *pack, int32_t *persistent,
                         int32_t *slice_cols)
{
    ABI_BEGIN
    if (!c) return fail(CLEORA_E_INVAL, "ctx is NULL");
    if (!c->has_emb) return fail(CLEORA_E_STATE, "no embedding");
    if (pack) *pack = c->pack;
    if (persistent) *persistent = c->persist;
    if (chunk) *chunk = c->chunk;
    if (n_split) *n_split = c->n_split;
    if (n_long) *n_long = c->n_long;
    if (n_buckets) *n_buckets = c->n_buckets;
    if (slice_cols) *slice_cols = c->slice_cols;
    return CLEORA_OK;
    ABI_END
}

int cleora_sync(cleora_ctx *c, void *stream)
{
    ABI_BEGIN
    if (!c) return fail(CLEORA_E_INVAL, "ctx is NULL");
    DeviceGuard g(c->device);
    CLEORA_HIP(hipStreamSynchronize(cleora::as_stream(stream)));
    return CLEORA_OK;
    ABI_END
}

int cleora_set_chunk(cleora_ctx *c, int32_t chunk)
{
    ABI_BEGIN
    if (!c) return fail(CLEORA_E_INVAL, "ctx is NULL");
    if (chunk < 0 || chunk > (1 << 20)) return fail(CLEORA_E_INVAL, "chunk out of range");
    c->chunk_req = chunk;
    return CLEORA_OK;
    ABI_END
}

int cleora_set_slices(cleora_ctx *c, int32_t cols)
{
    ABI_BEGIN
    if (!c) return fail(CLEORA_E_INVAL, "ctx is NULL");
    if (cols < CLEORA_SLICES_AUTO || (cols > 0 && (cols % 4 != 0 || cols > CLEORA_MAX_DIM_BF16)))
        return fail(CLEORA_E_INVAL,
                    "cols must be 0, CLEORA_SLICES_AUTO or a multiple of 4 up to 8192");
    c->slice_req = cols;
    return CLEORA_OK;
    ABI_END
}

int cleora_set_schedule(cleora_ctx *c, int32_t pack, int32_t persistent)
{
    ABI_BEGIN
    if (!c) return fail(CLEORA_E_INVAL, "ctx is NULL");
    if (pack != 0 && (pack < 16 || pack > (1 << 20)))
        return fail(CLEORA_E_INVAL, "pack must be 0 or in [16, 2^20]");
    if (persistent < -1 || persistent > 8)
        return fail(CLEORA_E_INVAL, "persistent must be in [-1, 8]");
    c->pack_req = pack;
    c->persist_req = persistent;
    return CLEORA_OK;
    ABI_END
}

int cleora_autotune(cleora_ctx *c, int32_t *pack, int32_t *persistent, float *step_ms,
                    void *stream)
{
    ABI_BEGIN
    cleora::TraceRange trace_range("cleora_autotune");
    if (!c) return fail(CLEORA_E_INVAL, "ctx is NULL");
    if (!c->has_emb) return fail(CLEORA_E_STATE, "no embedding: call cleora_init first");
    DeviceGuard g(c->device);
    hipStream_t s = cleora::as_stream(stream);
    const auto key = std::make_tuple(c->n, c->nnz, c->dim, c->dtype, c->chunk);
    TuneChoice best;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        load_tune_file_locked();
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) best = it->second;
    }
    if (best.pack == 0) {
        hipEvent_t a, b;
        CLEORA_HIP(hipEventCreate(&a));
        CLEORA_HIP(hipEventCreate(&b));
        const cleora::Variant v = cleora::choose_variant(c->dtype, c->ld);
        const bool timing = c->timing;
        c->timing = false;
        auto restore = [&]() {
            c->timing = timing;
            c->pack_req = 0;
            c->persist_req = -1;
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        };
        try {
            // packing size x grid (one wave per item, or the resident waves
            // looping over the items)
            for (int32_t p = 16; p <= c->chunk; p *= 2) {
                c->pack_req = p;
                c->persist_req = 0;
                cleora::plan_schedule(c, s);
                c->partial.ensure(sizeof(float) * (size_t)std::max<int64_t>(c->n_split, 1) *
                                  (size_t)c->ld);
                cleora::write_descs(c, s);
                for (int32_t persist = 0; persist <= 1; ++persist) {
                    // steps read T_t and write the other buffer; cur is not
                    // flipped, so the embedding and iteration count stay as
                    // they were
                    StepDesc d = cleora::host_desc(c, c->cur);
                    d.persist = persist;
                    auto one = [&]() {
                        cleora::launch_spmm(v, d, s);
                        if (c->n_long > 0)
                            cleora::launch_combine(v, c->desc.as<StepDesc>() + c->cur, 1,
                                                   c->n_long, s);
                    };
                    one();
                    CLEORA_HIP(hipEventRecord(a, s));
                    for (int r = 0; r < 3; ++r) one();
                    CLEORA_HIP(hipEventRecord(b, s));
                    CLEORA_HIP(hipEventSynchronize(b));
                    float ms = 0;
                    CLEORA_HIP(hipEventElapsedTime(&ms, a, b));
                    ms /= 3.0f;
                    if (std::getenv("CLEORA_TUNE_VERBOSE"))
                        std::fprintf(stderr,
                                     "[cleora autotune] n=%lld nnz=%lld d=%d pack=%d persist=%d: "
                                     "%.4f ms\n",
                                     (long long)c->n, (long long)c->nnz, c->dim, p, persist, ms);
                    if (best.pack == 0 || ms < best.ms) {
                        best.pack = p;
                        best.persist = persist;
                        best.ms = ms;
                    }
                }
            }
        } catch (...) {
            restore();
            // put the default schedule back: the trial one may not match
            // the buffers any more; without a schedule the embedding can no
            // longer be propagated
            try {
                cleora::plan_schedule(c, s);
                c->partial.ensure(sizeof(float) * (size_t)std::max<int64_t>(c->n_split, 1) *
                                  (size_t)c->ld);
                cleora::write_descs(c, s);
            } catch (...) {
                c->has_emb = false;
            }
            throw;
        }
        restore();
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = best;
        append_tune_file_locked(key, best);
    }
    c->pack_req = 0;  // the cache entry now applies to this and later inits
    c->persist_req = -1;
    // trial steps wrote the other buffer: a sliced context's unscaled rows
    // are gone, so it continues from the normalised rows
    c->deferred = false;
    if (c->slice_req == CLEORA_SLICES_AUTO) {
        try {
            choose_slices(c, s);
        } catch (...) {
            try {
                cleora::plan_schedule(c, s);
                c->partial.ensure(sizeof(float) * (size_t)std::max<int64_t>(c->n_split, 1) *
                                  (size_t)c->ld);
                cleora::write_descs(c, s);
            } catch (...) {
                c->has_emb = false;
            }
            throw;
        }
    }
    cleora::plan_schedule(c, s);
    c->partial.ensure(sizeof(float) * (size_t)std::max<int64_t>(c->n_split, 1) * (size_t)c->ld);
    cleora::write_descs(c, s);
    if (pack) *pack = best.pack;
    if (persistent) *persistent = best.persist;
    if (step_ms) *step_ms = best.ms;
    return CLEORA_OK;
    ABI_END
}

int cleora_set_timing(cleora_ctx *c, int on)
{
    ABI_BEGIN
    if (!c) return fail(CLEORA_E_INVAL, "ctx is NULL");
    c->timing = on != 0;
    return CLEORA_OK;
    ABI_END
}

int cleora_kernel_time(cleora_ctx *c, double *spmm_ms, int64_t *spmm_n, double *comb_ms,
                       int64_t *comb_n)
{
    ABI_BEGIN
    if (!c) return fail(CLEORA_E_INVAL, "ctx is NULL");
    DeviceGuard g(c->device);
    double a = 0, b = 0;
    for (auto &p : c->ev_spmm) {
        CLEORA_HIP(hipEventSynchronize(p.second));
        float ms = 0;
        CLEORA_HIP(hipEventElapsedTime(&ms, p.first, p.second));
        a += ms;
    }
    for (auto &p : c->ev_comb) {
        CLEORA_HIP(hipEventSynchronize(p.second));
        float ms = 0;
        CLEORA_HIP(hipEventElapsedTime(&ms, p.first, p.second));
        b += ms;
    }
    if (spmm_ms) *spmm_ms = a;
    if (spmm_n) *spmm_n = (int64_t)c->ev_spmm.size();
    if (comb_ms) *comb_ms = b;
    if (comb_n) *comb_n = (int64_t)c->ev_comb.size();
    c->ev_spmm.clear();
    c->ev_comb.clear();
    c->ev_next = 0;
    return CLEORA_OK;
    ABI_END
}

int cleora_launch_stats(cleora_ctx *c, int64_t *graph_instantiations, int64_t *graph_launches)
{
    ABI_BEGIN
    if (!c) return fail(CLEORA_E_INVAL, "ctx is NULL");
    if (graph_instantiations) *graph_instantiations = c->graph_instantiations;
    if (graph_launches) *graph_launches = c->graph_launches;
    return CLEORA_OK;
    ABI_END
}

int cleora_expand_clique(cleora_ctx *c, int64_t n_hyper, const int64_t *offsets,
                         const int32_t *members, int32_t *src, int32_t *dst, int64_t capacity,
                         int64_t *n_edges, void *stream)
{
    ABI_BEGIN
    cleora::TraceRange trace_range("cleora_expand_clique");
    if (!c || !offsets || !n_edges) return fail(CLEORA_E_INVAL, "NULL argument");
    if (n_hyper < 0) return fail(CLEORA_E_INVAL, "n_hyper < 0");
    if (src && !dst) return fail(CLEORA_E_INVAL, "NULL dst");
    if (src && !members && n_hyper > 0) return fail(CLEORA_E_INVAL, "NULL members");
    DeviceGuard g(c->device);
    *n_edges = cleora::expand_clique(n_hyper, offsets, members, src, dst, capacity, c->t_expand,
                                     c->h_small + 5, cleora::as_stream(stream));
    if (src) CLEORA_HIP(hipStreamSynchronize(cleora::as_stream(stream)));
    return CLEORA_OK;
    ABI_END
}

int cleora_expand_star(cleora_ctx *c, int64_t n_nodes, int64_t n_hyper, const int64_t *offsets,
                       const int32_t *members, int32_t *src, int32_t *dst, int64_t capacity,
                       int64_t *n_edges, void *stream)
{
    ABI_BEGIN
    cleora::TraceRange trace_range("cleora_expand_star");
    if (!c || !offsets || !n_edges) return fail(CLEORA_E_INVAL, "NULL argument");
    if (n_hyper < 0 || n_nodes < 0 || n_nodes + n_hyper > 0x7fffffffLL)
        return fail(CLEORA_E_INVAL, "n_nodes + n_hyper must stay below 2^31");
    if (src && !dst) return fail(CLEORA_E_INVAL, "NULL dst");
    DeviceGuard g(c->device);
    hipStream_t s = cleora::as_stream(stream);
    CLEORA_HIP(hipMemcpyAsync(c->h_small + 5, offsets, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    CLEORA_HIP(hipMemcpyAsync(c->h_small + 6, offsets + n_hyper, sizeof(int64_t),
                              hipMemcpyDeviceToHost, s));
    CLEORA_HIP(hipStreamSynchronize(s));
    const int64_t total = c->h_small[6] - c->h_small[5];
    *n_edges = total;
    if (!src) return CLEORA_OK;
    if (total > capacity) return fail(CLEORA_E_INVAL, "output capacity below the edge count");
    if (total > 0 && !members) return fail(CLEORA_E_INVAL, "NULL members");
    cleora::expand_star(n_nodes, n_hyper, offsets, members, src, dst, s);
    CLEORA_HIP(hipStreamSynchronize(s));
    return CLEORA_OK;
    ABI_END
}

int cleora_build_chunk(cleora_ctx *c, int64_t n_global, int64_t m, const int32_t *src,
                       const int32_t *dst, const float *w, uint32_t flags, void *stream)
{
    ABI_BEGIN
    cleora::TraceRange trace_range("cleora_build_chunk");
    if (!c) return fail(CLEORA_E_INVAL, "ctx is NULL");
    check_graph_sizes(n_global, m);
    if (m < 1 || !src || !dst) return fail(CLEORA_E_INVAL, "a chunk needs edges");
    if (flags & ~(CLEORA_DIRECTED | CLEORA_EMPTY_KEEP)) return fail(CLEORA_E_INVAL, "unknown flag");
    DeviceGuard g(c->device);
    cleora::build_chunk(c, n_global, m, src, dst, w, flags, cleora::as_stream(stream));
    return CLEORA_OK;
    ABI_END
}

int cleora_chunk_info(cleora_ctx *c, int64_t *n_local, int32_t *ids, float *occ, void *stream)
{
    ABI_BEGIN
    if (!c) return fail(CLEORA_E_INVAL, "ctx is NULL");
    if (!c->is_chunk || !c->has_graph) return fail(CLEORA_E_STATE, "not a chunk");
    DeviceGuard g(c->device);
    hipStream_t s = cleora::as_stream(stream);
    if (n_local) *n_local = c->n;
    if (ids)
        CLEORA_HIP(hipMemcpyAsync(ids, c->chunk_ids.p, sizeof(int32_t) * c->n, hipMemcpyDefault, s));
    if (occ)
        CLEORA_HIP(hipMemcpyAsync(occ, c->chunk_occ.p, sizeof(float) * c->n, hipMemcpyDefault, s));
    return CLEORA_OK;
    ABI_END
}

int cleora_merge_chunk(cleora_ctx *c, float *acc, int64_t ld_acc, float *wsum, void *stream)
{
    ABI_BEGIN
    cleora::TraceRange trace_range("cleora_merge_chunk");
    if (!c || !acc || !wsum) return fail(CLEORA_E_INVAL, "NULL argument");
    if (!c->is_chunk || !c->has_emb) return fail(CLEORA_E_STATE, "not an embedded chunk");
    if (ld_acc < c->dim) return fail(CLEORA_E_INVAL, "ld_acc < dim");
    DeviceGuard g(c->device);
    cleora::launch_merge_rows(c->dtype, c->E[c->cur].p, c->n, c->dim, c->ld,
                              c->chunk_ids.as<int32_t>(), c->chunk_occ.as<float>(), acc, ld_acc,
                              wsum, cleora::as_stream(stream));
    return CLEORA_OK;
    ABI_END
}

int cleora_merge_finish(int device, const float *acc, int64_t ld_acc, const float *wsum,
                        int64_t n_global, int32_t dim, void *out, int64_t ld_out,
                        int32_t out_dtype, void *stream)
{
    ABI_BEGIN
    if (!acc || !wsum || !out) return fail(CLEORA_E_INVAL, "NULL argument");
    if (n_global < 1 || dim < 1 || ld_acc < dim || ld_out < dim)
        return fail(CLEORA_E_INVAL, "bad sizes");
    if (out_dtype != CLEORA_F32 && out_dtype != CLEORA_BF16)
        return fail(CLEORA_E_INVAL, "unknown dtype");
    DeviceGuard g(device);
    cleora::launch_merge_finish(acc, ld_acc, wsum, n_global, dim, out, ld_out, out_dtype,
                                cleora::as_stream(stream));
    return CLEORA_OK;
    ABI_END
}

}  // extern "C"

namespace {

// Host check of one graph's edges (the error path of a batch only): ids in
// [0, n), weights finite and positive, as the build's key kernel requires.
int32_t graph_status(const cleora_graph &G)
{
    const int64_t m = G.n_edges;
    if (m <= 0) return CLEORA_OK;
    std::vector<int32_t> ids(2 * (size_t)m);
    if (hipMemcpy(ids.data(), G.src, 4 * (size_t)m, hipMemcpyDefault) != hipSuccess ||
        hipMemcpy(ids.data() + m, G.dst, 4 * (size_t)m, hipMemcpyDefault) != hipSuccess) {
        (void)hipGetLastError();
        return CLEORA_E_DEVICE;
    }
    for (int32_t id : ids)
        if (id < 0 || id >= G.n_nodes) return CLEORA_E_INPUT;
    if (G.w) {
        std::vector<float> w((size_t)m);
        if (hipMemcpy(w.data(), G.w, 4 * (size_t)m, hipMemcpyDefault) != hipSuccess) {
            (void)hipGetLastError();
            return CLEORA_E_DEVICE;
        }
        for (float x : w)
            if (!(x > 0.0f && x <= 3.402823466e38f)) return CLEORA_E_INPUT;
    }
    return CLEORA_OK;
}

void embed_batch_impl(cleora_ctx *c, int32_t n_graphs, const cleora_graph *graphs,
                      uint32_t flags, int32_t dim, int32_t dtype, int32_t k, void *const *out,
                      void *stream);

}  // namespace

extern "C" {

int cleora_embed_batch(cleora_ctx *c, int32_t n_graphs, const cleora_graph *graphs,
                       uint32_t flags, int32_t dim, int32_t dtype, int32_t k, void *const *out,
                       void *stream)
{
    ABI_BEGIN
    cleora::TraceRange trace_range("cleora_embed_batch");
    if (!c || !graphs || !out) return fail(CLEORA_E_INVAL, "NULL argument");
    if (n_graphs < 1) return fail(CLEORA_E_INVAL, "n_graphs must be >= 1");
    c->batch_status.assign((size_t)n_graphs, CLEORA_OK);
    auto all = [&](int32_t code) {
        std::fill(c->batch_status.begin(), c->batch_status.end(), code);
    };
    try {
        embed_batch_impl(c, n_graphs, graphs, flags, dim, dtype, k, out, stream);
    } catch (const Error &e) {
        if (e.code != CLEORA_E_INPUT) {
            all(e.code);
        } else {
            DeviceGuard dg(c->device);
            for (int32_t g = 0; g < n_graphs; ++g) c->batch_status[g] = graph_status(graphs[g]);
        }
        throw;
    } catch (const std::bad_alloc &) {
        all(CLEORA_E_NOMEM);
        throw;
    } catch (...) {
        all(CLEORA_E_DEVICE);
        throw;
    }
    return CLEORA_OK;
    ABI_END
}

int cleora_batch_status(cleora_ctx *c, int32_t n_graphs, int32_t *status)
{
    ABI_BEGIN
    if (!c || !status) return fail(CLEORA_E_INVAL, "NULL argument");
    if (c->batch_status.empty()) return fail(CLEORA_E_STATE, "no cleora_embed_batch call yet");
    if (n_graphs != (int32_t)c->batch_status.size())
        return fail(CLEORA_E_INVAL, "n_graphs differs from the last batch");
    std::copy(c->batch_status.begin(), c->batch_status.end(), status);
    return CLEORA_OK;
    ABI_END
}

}  // extern "C"

namespace {

void embed_batch_impl(cleora_ctx *c, int32_t n_graphs, const cleora_graph *graphs,
                      uint32_t flags, int32_t dim, int32_t dtype, int32_t k, void *const *out,
                      void *stream)
{
    if (k < 0) throw Error(CLEORA_E_INVAL, "k must be >= 0");
    if (flags & ~(CLEORA_DIRECTED | CLEORA_EMPTY_KEEP)) throw Error(CLEORA_E_INVAL, "unknown flag");
    check_dim(dim, dtype);
    std::vector<int64_t> row0((size_t)n_graphs + 1, 0), eoff((size_t)n_graphs + 1, 0);
    std::vector<uint64_t> seeds((size_t)n_graphs);
    bool any_w = false;
    for (int32_t g = 0; g < n_graphs; ++g) {
        const cleora_graph &G = graphs[g];
        check_graph_sizes(G.n_nodes, G.n_edges);
        if (G.n_edges > 0 && (!G.src || !G.dst)) throw Error(CLEORA_E_INVAL, "graph src/dst NULL");
        if (!out[g]) throw Error(CLEORA_E_INVAL, "output pointer NULL");
        row0[g + 1] = row0[g] + G.n_nodes;
        eoff[g + 1] = eoff[g] + G.n_edges;
        seeds[g] = G.seed;
        any_w = any_w || G.w != nullptr;
    }
    const int64_t N = row0[n_graphs], M = eoff[n_graphs];
    check_graph_sizes(N, M);
    DeviceGuard dg(c->device);
    hipStream_t s = cleora::as_stream(stream);
    c->is_chunk = false;
    // concatenated edge list with node offsets, then the ordinary build
    const size_t ebytes = ((size_t)std::max<int64_t>(M, 1) * (any_w ? 12 : 8) + 255) / 256 * 256;
    c->t_edges.ensure(ebytes + sizeof(int64_t) * (row0.size() + seeds.size()) + 64);
    int32_t *osrc = c->t_edges.as<int32_t>(), *odst = osrc + std::max<int64_t>(M, 1);
    float *ow = any_w ? reinterpret_cast<float *>(odst + std::max<int64_t>(M, 1)) : nullptr;
    char *tail = c->t_edges.as<char>() + ebytes;
    int64_t *d_row0 = reinterpret_cast<int64_t *>(tail);
    uint64_t *d_seeds = reinterpret_cast<uint64_t *>(d_row0 + row0.size());
    for (int32_t g = 0; g < n_graphs; ++g) {
        const cleora_graph &G = graphs[g];
        if (G.n_edges == 0) continue;
        const unsigned blocks = (unsigned)std::min<int64_t>(cleora::ceil_div(G.n_edges, 256), 65536);
        k_offset_edges<<<blocks, 256, 0, s>>>(G.n_edges, G.src, G.dst, G.w, G.n_nodes, row0[g],
                                              osrc + eoff[g], odst + eoff[g],
                                              ow ? ow + eoff[g] : nullptr);
        CLEORA_LAUNCH_CHECK();
    }
    CLEORA_HIP(hipMemcpyAsync(d_row0, row0.data(), sizeof(int64_t) * row0.size(),
                              hipMemcpyHostToDevice, s));
    CLEORA_HIP(hipMemcpyAsync(d_seeds, seeds.data(), sizeof(uint64_t) * seeds.size(),
                              hipMemcpyHostToDevice, s));
    cleora::build_graph(c, N, N, M, osrc, odst, ow, flags, s);  // synchronises
    setup_embedding(c, dim, dtype, s);
    cleora::launch_init(dtype, c->E[0].p, N, dim, c->ld, d_row0, d_seeds, n_graphs, 0, s);
    c->has_emb = true;
    run_steps(c, k, s);
    const size_t es = elem_size(dtype);
    for (int32_t g = 0; g < n_graphs; ++g) {
        const char *src = c->E[c->cur].as<char>() + (size_t)row0[g] * c->ld * es;
        CLEORA_HIP(hipMemcpy2DAsync(out[g], (size_t)dim * es, src, (size_t)c->ld * es,
                                    (size_t)dim * es, (size_t)graphs[g].n_nodes, hipMemcpyDefault,
                                    s));
    }
    // the host vectors above must outlive the copies that read them
    CLEORA_HIP(hipStreamSynchronize(s));
}

}  // namespace

extern "C" {

int cleora_step_multi(cleora_ctx *const *ctxs, int32_t n, void *stream)
{
    ABI_BEGIN
    cleora::TraceRange trace_range("cleora_step_multi");
    if (n < 0 || (n > 0 && !ctxs)) return fail(CLEORA_E_INVAL, "bad context list");
    if (n == 0) return CLEORA_OK;
    for (int32_t i = 0; i < n; ++i) {
        if (!ctxs[i]) return fail(CLEORA_E_INVAL, "NULL context");
        if (!ctxs[i]->has_emb) return fail(CLEORA_E_STATE, "context without embedding");
        if (ctxs[i]->dtype != ctxs[0]->dtype || ctxs[i]->ld != ctxs[0]->ld ||
            ctxs[i]->device != ctxs[0]->device)
            return fail(CLEORA_E_INVAL, "contexts differ in dim, dtype or device");
        for (int32_t j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return fail(CLEORA_E_INVAL, "context listed twice");
    }
    DeviceGuard dg(ctxs[0]->device);
    cleora::step_contexts(ctxs, n, cleora::as_stream(stream));
    return CLEORA_OK;
    ABI_END
}

}  // extern "C"
